"""Pins of the oracle's Wilson-Dirac operator against facts fixed outside it.

Closed forms (free field, abelian twist), gauge covariance, gamma5-Hermiticity
(Sec. 4), adjointness, the dense matrix built block by block, and a worked
example under tests/golden/.
"""
import os

import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import wilson as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _match_spectra(a, b):
    """Max distance between two multisets of complex numbers under the best pairing."""
    from scipy.optimize import linear_sum_assignment

    a, b = np.asarray(a), np.asarray(b)
    assert a.shape == b.shape
    cost = np.abs(a[:, None] - b[None, :])
    i, j = linear_sum_assignment(cost)
    return cost[i, j].max()


def test_gamma_algebra():
    g = W.gammas()
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T, atol=0)
        for nu in range(4):
            ac = g[mu] @ g[nu] + g[nu] @ g[mu]
            assert np.allclose(ac, 2 * np.eye(4) * (mu == nu), atol=1e-15)
    # gamma5 = g1 g2 g3 g4 = diag(1, 1, -1, -1) in this chiral basis (by hand)
    assert np.allclose(W.gamma5(), np.diag([1, 1, -1, -1]), atol=1e-15)


def test_links_are_su3():
    U = synth.random_su3_links((4, 2, 2, 4), 0.3, 7)
    uu = np.einsum("mvab,mvcb->mvac", U, U.conj())
    assert np.abs(uu - np.eye(3)).max() < 1e-14
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-14
    # exp(i eps H) with eps = 0.3 stays close to the identity but not at it
    dev = np.abs(U - np.eye(3)).max()
    assert 0.05 < dev < 2.0


def test_free_field_golden_2x2x2x2():
    """Hand-derived eigenvalues of the free operator on 2^4 (tests/golden)."""
    rows = np.loadtxt(os.path.join(GOLDEN, "free_field_2x2x2x2_kappa0.125.txt"))
    expect = np.concatenate([np.full(int(m), re + 1j * im) for re, im, m in rows])
    dims = (2, 2, 2, 2)
    D = W.dense_D(synth.unit_links(dims), 0.125, dims, bc_t=-1)
    lam = np.linalg.eigvals(D)
    assert len(expect) == 192
    assert _match_spectra(lam, expect) < 1e-13


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 2, 2, 4), (2, 4, 2, 2)])
@pytest.mark.parametrize("bc_t", [-1, 1])
def test_free_field_closed_form(dims, bc_t):
    kappa = 0.11
    D = W.dense_D(synth.unit_links(dims), kappa, dims, bc_t=bc_t)
    lam = np.linalg.eigvals(D)
    assert _match_spectra(lam, W.free_field_spectrum(kappa, dims, bc_t)) < 1e-13


def test_abelian_twist_closed_form():
    """U_mu = exp(i theta_mu) 1 shifts every momentum by theta_mu (catches U vs U^+)."""
    dims = (2, 2, 4, 2)
    th = (0.3, -0.7, 0.45, 1.1)
    kappa = 0.09
    D = W.dense_D(synth.unit_links(dims, th), kappa, dims, bc_t=-1)
    lam = np.linalg.eigvals(D)
    assert _match_spectra(lam, W.free_field_spectrum(kappa, dims, -1, th)) < 1e-13
    # the twist must matter: the untwisted spectrum is different
    assert _match_spectra(lam, W.free_field_spectrum(kappa, dims, -1)) > 1e-3


def test_plane_wave_action_4x4x4x4():
    """D on one plane wave in a chiral eigenvector of sum gamma_mu sin p_mu (no dense matrix)."""
    dims = (4, 4, 4, 4)
    kappa = 0.1
    V = 256
    n = (1, 3, 0, 2)
    p = np.array([2 * np.pi * n[0] / 4, 2 * np.pi * n[1] / 4, 2 * np.pi * n[2] / 4, np.pi * (2 * n[3] + 1) / 4])
    g = W.gammas()
    S = sum(g[mu] * np.sin(p[mu]) for mu in range(4))
    ev, evec = np.linalg.eigh(S)
    chi = evec[:, -1]
    s = np.arange(V)
    c = np.stack(W.site_coords(s, dims), axis=1)
    # antiperiodic t: the phase of a plane wave with p_t = pi(2n+1)/Lt already
    # flips sign across the boundary, so the lattice field is just exp(i p.x)
    phase = np.exp(1j * (c @ p))
    colour = np.array([0.3, -1.0j, 0.5])
    psi = phase[:, None, None] * chi[None, :, None] * colour[None, None, :]
    lam = 1 - 2 * kappa * np.cos(p).sum() + 2j * kappa * ev[-1]
    out = W.apply_D(synth.unit_links(dims), psi, kappa, dims)
    assert np.abs(out - lam * psi).max() < 1e-14


def _random_setup(dims, seed=11, kappa=0.12):
    U = synth.random_su3_links(dims, 0.3, seed)
    V = synth.volume(dims)
    x = synth.gaussian_spinor(V, seed + 1)
    y = synth.gaussian_spinor(V, seed + 2)
    return U, V, x, y, kappa


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 4, 2, 4), (3, 2, 4, 2)])
def test_gamma5_hermiticity(dims):
    """gamma5 D gamma5 = D^+ (Sec. 4), with D^+ coded independently."""
    U, V, x, _, kappa = _random_setup(dims)
    lhs = W.apply_gamma5(W.apply_D(U, W.apply_gamma5(x), kappa, dims))
    rhs = W.apply_Ddag(U, x, kappa, dims)
    assert np.abs(lhs - rhs).max() < 1e-14 * np.abs(rhs).max() * 10


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 2, 4, 4)])
def test_adjointness(dims):
    U, V, x, y, kappa = _random_setup(dims, seed=21)
    a = np.vdot(y, W.apply_D(U, x, kappa, dims))
    b = np.vdot(W.apply_Ddag(U, y, kappa, dims), x)
    assert abs(a - b) <= 1e-13 * abs(a)


def test_gauge_covariance():
    """D[U^G](G psi) = G D[U] psi, U^G_mu(x) = G(x) U_mu(x) G(x+mu)^+."""
    dims = (4, 2, 2, 4)
    U, V, x, _, kappa = _random_setup(dims, seed=31)
    G = synth.random_su3_links(dims, 2.0, 99)[0]  # one random SU(3) matrix per site
    UG = np.empty_like(U)
    for mu in range(4):
        for s in range(V):
            c = list(W.site_coords(s, dims))
            c[mu] += 1
            sf = W.site_index(*c, dims)
            UG[mu, s] = G[s] @ U[mu, s] @ G[sf].conj().T
    Gx = np.einsum("vab,vsb->vsa", G, x)
    lhs = W.apply_D(UG, Gx, kappa, dims)
    rhs = np.einsum("vab,vsb->vsa", G, W.apply_D(U, x, kappa, dims))
    assert np.abs(lhs - rhs).max() < 1e-13
    # and a wrong transform (G(x+mu) on the left) must break it
    UB = np.empty_like(U)
    for mu in range(4):
        for s in range(V):
            c = list(W.site_coords(s, dims))
            c[mu] += 1
            sf = W.site_index(*c, dims)
            UB[mu, s] = G[sf] @ U[mu, s] @ G[s].conj().T
    assert np.abs(W.apply_D(UB, Gx, kappa, dims) - rhs).max() > 1e-3


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 4, 4, 4), (2, 4, 2, 4)])
def test_stencil_equals_dense(dims):
    U, V, x, _, kappa = _random_setup(dims, seed=41)
    for dag in (False, True):
        M = W.dense_D(U, kappa, dims, dagger=dag, sparse=True)
        f = W.apply_Ddag if dag else W.apply_D
        assert np.abs(M @ x.ravel() - f(U, x, kappa, dims).ravel()).max() < 1e-14
    # the dense D^+ is the conjugate transpose of the dense D
    M = W.dense_D(U, kappa, dims, sparse=True)
    Md = W.dense_D(U, kappa, dims, dagger=True, sparse=True)
    assert abs(M.conj().T - Md).max() < 1e-16


def test_site_formula_equals_stencil():
    dims = (4, 4, 2, 4)
    U, V, x, _, kappa = _random_setup(dims, seed=51)
    sites = [0, 1, 7, 31, 64, 127]
    for dag in (False, True):
        f = W.apply_Ddag if dag else W.apply_D
        full = f(U, x, kappa, dims)
        part = W.apply_D_sites(U, x, kappa, dims, sites, dagger=dag)
        assert np.abs(full[sites] - part).max() < 1e-14


def test_spectrum_conjugate_symmetric():
    """gamma5-Hermiticity: eigenvalues are real or come in conjugate pairs (Sec. 4)."""
    dims = (2, 2, 2, 2)
    U = synth.random_su3_links(dims, 0.8, 61)
    lam = np.linalg.eigvals(W.dense_D(U, 0.14, dims))
    assert _match_spectra(lam, lam.conj()) < 1e-12


def test_reject_short_extent():
    U = synth.unit_links((2, 2, 2, 2))
    with pytest.raises(ValueError):
        W.apply_D(U[:, :8], np.zeros((8, 4, 3), complex), 0.1, (1, 2, 2, 2))


def test_boundary_sign_matters():
    """bc_t = -1 and +1 give different operators; bc only touches t-hops."""
    dims = (2, 2, 2, 4)
    U, V, x, _, kappa = _random_setup(dims, seed=71)
    a = W.apply_D(U, x, kappa, dims, bc_t=-1)
    b = W.apply_D(U, x, kappa, dims, bc_t=1)
    c = np.array(W.site_coords(np.arange(V), dims)).T
    inner = (c[:, 3] > 0) & (c[:, 3] < dims[3] - 1)
    assert np.abs(a[inner] - b[inner]).max() < 1e-15
    assert np.abs(a[~inner] - b[~inner]).max() > 1e-3


# --------------------------------------------------------------- even-odd
def _dense_Dhat(U, kappa, dims, dagger=False):
    Ve = synth.volume(dims) // 2
    I = np.eye(12 * Ve, dtype=np.complex128)
    return np.column_stack([W.apply_Dhat(U, I[:, k].reshape(Ve, 4, 3), kappa, dims, dagger=dagger).ravel()
                            for k in range(12 * Ve)])


def test_eo_schur_complement_solves_the_full_system():
    """D x = b  <=>  Dhat x_e = b_e + kappa H_eo b_o and x_o = b_o + kappa H_oe x_e,
    checked against LAPACK on the full matrix built site by site."""
    dims, kappa = (4, 2, 2, 4), 0.12
    V = synth.volume(dims)
    U = synth.random_su3_links(dims, 0.5, 31)
    b = synth.gaussian_spinor(V, 32)
    x = np.linalg.solve(W.dense_D(U, kappa, dims), b.ravel()).reshape(V, 4, 3)
    par = W.parity(dims)
    be = W.eo_prepare(U, b, kappa, dims)
    xe = x[par == 0]
    assert np.abs(W.apply_Dhat(U, xe, kappa, dims) - be).max() <= 1e-12 * np.abs(be).max()
    xr = W.eo_reconstruct(U, xe, b, kappa, dims)
    assert np.abs(xr - x).max() <= 1e-12 * np.abs(x).max()


def test_eo_spectrum_is_lambda_times_two_minus_lambda():
    """H anticommutes with the parity sign, so spec(D) comes in pairs (lambda,
    2 - lambda) and spec(Dhat) = {lambda (2 - lambda)}, each value once."""
    dims, kappa = (4, 2, 2, 4), 0.13
    U = synth.random_su3_links(dims, 0.5, 41)
    lam = np.linalg.eigvals(W.dense_D(U, kappa, dims))
    mu = np.linalg.eigvals(_dense_Dhat(U, kappa, dims))
    assert _match_spectra(lam * (2 - lam), np.concatenate([mu, mu])) < 1e-10


def test_eo_free_field_closed_form():
    """Unit links: spec(Dhat) = {lambda (2 - lambda)} with the free-field closed form of lambda."""
    dims, kappa = (4, 2, 2, 4), 0.11
    lam = W.free_field_spectrum(kappa, dims)
    mu = np.linalg.eigvals(_dense_Dhat(synth.unit_links(dims), kappa, dims))
    assert _match_spectra(lam * (2 - lam), np.concatenate([mu, mu])) < 1e-12


def test_eo_adjoint_and_gamma5():
    """<y, Dhat x> = <Dhat^+ y, x> and gamma5 Dhat gamma5 = Dhat^+ (Dhat^+ from the adjoint hops)."""
    dims, kappa = (4, 4, 2, 4), 0.12
    U = synth.random_su3_links(dims, 0.3, 51)
    Ve = synth.volume(dims) // 2
    x, y = synth.gaussian_spinor(Ve, 52), synth.gaussian_spinor(Ve, 53)
    a = np.vdot(y, W.apply_Dhat(U, x, kappa, dims))
    b = np.vdot(W.apply_Dhat(U, y, kappa, dims, dagger=True), x)
    assert abs(a - b) <= 1e-13 * abs(a)
    lhs = W.apply_gamma5(W.apply_Dhat(U, W.apply_gamma5(x), kappa, dims))
    rhs = W.apply_Dhat(U, x, kappa, dims, dagger=True)
    assert np.abs(lhs - rhs).max() <= 1e-14 * np.abs(rhs).max() * 10


def test_eo_rejects_odd_extent():
    with pytest.raises(ValueError):
        W.apply_Dhat(synth.unit_links((3, 2, 2, 2)), np.zeros((12, 4, 3), complex), 0.1, (3, 2, 2, 2))
