"""Pins of the oracle's BiCG / eigBiCG / incremental / BiCGStab code.

Each check is fixed by something other than the oracle itself: LAPACK solves
and eigenvalues, the explicit projection W^+ A V, textbook CG on Hermitian
matrices, closed forms of the arrow entries, the biorthogonality identities
the algorithms promise, and gamma5 relations of Sec. 4.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import krylov as K
from oracle import wilson as W
from oracle.eig import eig, sort_order


def _generic(N=240, seed=3):
    """Non-normal matrix with six small isolated eigenvalues and a bulk in [0.6, 2]."""
    rng = np.random.default_rng(seed)
    small = np.array([0.01, 0.02 + 0.01j, 0.02 - 0.01j, 0.035, 0.05 + 0.02j, 0.05 - 0.02j])
    rest = 0.6 + 1.4 * rng.random(N - 6) + 1j * (rng.random(N - 6) - 0.5) * 0.8
    lam = np.concatenate([small, rest])
    S = np.eye(N) + 0.1 * (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))) / np.sqrt(N)
    M = S @ np.diag(lam) @ np.linalg.inv(S)
    return M, lam, rng


def _ops(M):
    Md = M.conj().T.copy()
    return (lambda v: M @ v), (lambda v: Md @ v)


def _wilson(dims, kappa, seed):
    U = synth.random_su3_links(dims, 0.3, seed)
    V = synth.volume(dims)
    A = lambda v: W.apply_D(U, v.reshape(V, 4, 3), kappa, dims).ravel()
    Ad = lambda v: W.apply_Ddag(U, v.reshape(V, 4, 3), kappa, dims).ravel()
    return U, V, A, Ad


def _nearest_rel(vals, exact):
    return np.array([np.min(np.abs(exact - v)) / abs(v) for v in vals])


# ----------------------------------------------------------------------------- eig(C)
def test_eig_contract():
    rng = np.random.default_rng(0)
    C = rng.standard_normal((12, 12)) + 1j * rng.standard_normal((12, 12))
    y, z, lam = eig(C)
    assert np.abs(C @ y - y * lam).max() < 1e-12
    assert np.abs(z.conj().T @ C - lam[:, None] * z.conj().T).max() < 1e-12
    assert np.abs(z.conj().T @ y - np.eye(12)).max() < 1e-10
    assert np.allclose(np.linalg.norm(y, axis=0), 1)
    assert np.all(np.diff(np.abs(lam)) >= -1e-15)


def test_sort_ties_imag_descending():
    lam = np.array([1 - 1j, 0.5, 1 + 1j, -0.5j])
    order = sort_order(lam)
    assert [lam[i] for i in order] == [0.5, -0.5j, 1 + 1j, 1 - 1j]


def test_sort_criteria():
    """The three criteria of eig()'s sort (Sec. 1, end: a user-chosen criterion)."""
    lam = np.array([2 + 0.1j, -0.3, 0.5j, 1.0, -1 - 1j, 0.2 + 1j, 0.2 - 1j])
    got = {w: [lam[i] for i in sort_order(lam, w)] for w in ("SM", "SR", "LM")}
    assert got["SM"] == [-0.3, 0.5j, 1.0, 0.2 + 1j, 0.2 - 1j, -1 - 1j, 2 + 0.1j]
    assert got["SR"] == [-1 - 1j, -0.3, 0.5j, 0.2 + 1j, 0.2 - 1j, 1.0, 2 + 0.1j]
    assert got["LM"] == [2 + 0.1j, -1 - 1j, 0.2 + 1j, 0.2 - 1j, 1.0, 0.5j, -0.3]
    with pytest.raises(ValueError):
        sort_order(lam, "LR")


@pytest.mark.parametrize("normal", [True, False])
def test_bicg_eigen_keeps_the_criterion_pairs(normal):
    """Alg. BiCG-eigen on an H with a known spectrum: the eigenvectors of H^(m) it keeps
    are exact, so the restarted H = diag(Lam) leads with the nev eigenvalues the
    criterion selects (smallest modulus, smallest real part, largest modulus)."""
    rng = np.random.default_rng(2)
    m, nev = 16, 4
    left = [0.05 + 1.5j, 0.05 - 1.5j, 0.08 + 1.6j, 0.08 - 1.6j]  # smallest real parts, |lambda| ~ 1.5
    small = [0.3, 0.35, 0.4 + 0.05j, 0.4 - 0.05j]  # smallest moduli
    large = [4.0, 4.5 + 0.2j, 4.5 - 0.2j, 5.0]
    mu = np.array(left + small + large + [1.0 + 0.1j, 1.5, 2.0 - 0.2j, 2.5])
    X = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    S = np.linalg.qr(X)[0] if normal else np.eye(m) + 0.2 * X / np.sqrt(m)
    H = S @ np.diag(mu) @ np.linalg.inv(S)
    for which, want in (("SM", small), ("SR", left), ("LM", large)):
        CV, CW, Lam = K.bicg_eigen(nev, m, H, which)
        assert len(Lam) == 2 * nev
        assert sorted(np.round(Lam[:nev], 10), key=lambda z: (z.real, z.imag)) == sorted(
            np.round(np.array(want), 10), key=lambda z: (z.real, z.imag))
        assert np.abs(CW.conj().T @ H @ CV - np.diag(Lam)).max() < 1e-12


# ------------------------------------------------------------------------- BiCG core
@pytest.mark.parametrize("dims,kappa", [((2, 2, 2, 2), 0.13), ((4, 4, 4, 4), 0.115)])
def test_bicg_matches_lapack_solve(dims, kappa):
    U, V, A, Ad = _wilson(dims, kappa, 1000)
    b = synth.z2_source(V, 10**6).ravel()
    x, it, hist = K.bicg(A, Ad, b, np.zeros_like(b), 1e-11)
    Msp = W.dense_D(U, kappa, dims, sparse=True).tocsc()
    import scipy.sparse.linalg as spla

    xs = spla.spsolve(Msp, b)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-9
    assert np.linalg.norm(b - A(x)) / np.linalg.norm(b) < 1e-10


def test_bicg_equals_cg_on_hpd():
    """Hermitian A with rhat0 = r0: rhat_j = r_j and BiCG is CG iterate for iterate."""
    rng = np.random.default_rng(5)
    N = 150
    X = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    M = X @ X.conj().T / N + 0.05 * np.eye(N)
    A, Ad = _ops(M)
    b = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    xb, itb, hb = K.bicg(A, Ad, b, np.zeros(N, complex), 1e-10, maxiter=25)
    xc, itc, hc = K.cg(A, b, np.zeros(N, complex), 1e-10, maxiter=25)
    assert itb == itc
    assert np.allclose(hb, hc, rtol=1e-9, atol=0)
    assert np.linalg.norm(xb - xc) / np.linalg.norm(xc) < 1e-10


def test_eigbicg_iterate_equals_bicg():
    """The eigenvalue part does not touch the BiCG iterate (Sec. 1 on eigCG, Sec. 2)."""
    M, _, rng = _generic()
    A, Ad = _ops(M)
    b = rng.standard_normal(M.shape[0]) + 0j
    x1, it1, h1 = K.bicg(A, Ad, b, np.zeros_like(b), 1e-10)
    r = K.eigbicg(A, Ad, b, np.zeros_like(b), 4, 16, 1e-10)
    assert r.iters == it1
    assert np.abs(r.x - x1).max() == 0.0


def test_unrestarted_H_is_projection():
    """No restart (m > iterations): H from the BiCG scalars = W^+ A V and W^+ V = I."""
    M, _, rng = _generic()
    A, Ad = _ops(M)
    b = rng.standard_normal(M.shape[0]) + 1j * rng.standard_normal(M.shape[0])
    r = K.eigbicg(A, Ad, b, np.zeros_like(b), 2, 40, 1e-30, maxiter=14)
    Vw, Ww, H = r.V_final, r.W_final, r.H_final
    assert H.shape == (14, 14)
    assert np.abs(Ww.conj().T @ Vw - np.eye(14)).max() < 1e-10
    assert np.allclose(np.linalg.norm(Vw, axis=0), 1)
    P = Ww.conj().T @ (M @ Vw)
    assert np.abs(P - H).max() < 1e-10 * np.abs(H).max()
    # tridiagonal
    assert np.abs(np.triu(H, 2)).max() == 0 and np.abs(np.tril(H, -2)).max() == 0


# ------------------------------------------------------------------ window restarts
def test_restart_invariants():
    """After every restart: W^+V = I, W^+ A V = diag(Lambda), arrow dots = closed forms."""
    M, _, rng = _generic()
    A, Ad = _ops(M)
    b = rng.standard_normal(M.shape[0]) + 0j
    r = K.eigbicg(A, Ad, b, np.zeros_like(b), 4, 16, 1e-12, keep_restarts=True)
    assert len(r.restarts) >= 4
    for i, rec in enumerate(r.restarts):
        k = rec.CV.shape[1]
        assert k == 8
        # Lambda are the eigenvalues of the oblique projection of H onto the kept space
        assert np.abs(rec.CW.conj().T @ rec.H_before @ rec.CV - np.diag(rec.Lam)).max() < 1e-12
        if i >= 4:
            # once Ritz vectors converge, finite precision erodes biorthogonality
            # (as in any Lanczos process); the identities below are exact only
            # while it holds
            continue
        Vn, Wn = rec.V_new, rec.W_new
        assert np.abs(Wn.conj().T @ Vn - np.eye(k)).max() < 1e-10
        assert np.abs(Wn.conj().T @ (M @ Vn) - np.diag(rec.Lam)).max() < 1e-10
        # only A v_m leaves span V (and A^+ w_m leaves span W): the arrow entries
        # are H_{m+1,m} (C_V)_{m,k} and conj((C_W)_{m,k}) H_{m,m+1}
        row = rec.h_next_prev * rec.CV[-1, :]
        col = np.conj(rec.CW[-1, :]) * rec.h_prev_next
        assert np.abs(rec.arrow_row - row).max() < 1e-10 * np.abs(row).max()
        assert np.abs(rec.arrow_col - col).max() < 1e-10 * np.abs(col).max()


def test_eigbicg_converged_ritz_values():
    """Ritz values with small residuals match LAPACK eigenvalues of A within 1e-8."""
    M, lam_exact, rng = _generic()
    A, Ad = _ops(M)
    b = rng.standard_normal(M.shape[0]) + 0j
    r = K.eigbicg(A, Ad, b, np.zeros_like(b), 4, 16, 1e-12)
    rr, rl = K.ritz_residuals(A, Ad, r.lam, r.U, r.Q)
    conv = (rr < 1e-4) & (rl < 1e-4)
    assert conv.sum() >= 4
    assert np.all(_nearest_rel(r.lam[conv], sla.eigvals(M)) < 1e-8)
    # the four smallest exact eigenvalues are the ones found
    assert np.all(_nearest_rel(lam_exact[:4], r.lam) < 1e-8)
    # returned vectors: ||U_i|| = 1 and Q_i^+ U_i = 1
    assert np.allclose(np.linalg.norm(r.U, axis=0), 1)
    assert np.allclose(np.einsum("ij,ij->j", r.Q.conj(), r.U), 1)


def test_windowed_vs_unrestarted_ritz():
    """Table 1 pattern: limited-window eigBiCG agrees with un-restarted BiCG on the lowest values."""
    M, _, rng = _generic(seed=4)
    A, Ad = _ops(M)
    b = rng.standard_normal(M.shape[0]) + 0j
    win = K.eigbicg(A, Ad, b, np.zeros_like(b), 4, 16, 1e-12)
    full = K.eigbicg(A, Ad, b, np.zeros_like(b), 4, 400, 1e-12)
    assert len(full.restarts) == 0 and len(win.restarts) > 0
    assert np.all(_nearest_rel(win.lam[:3], full.lam) < 1e-7)


def test_hermitian_reduction_gives_real_ritz():
    rng = np.random.default_rng(8)
    N = 200
    Qm, _ = np.linalg.qr(rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N)))
    ev = np.concatenate([[0.01, 0.02, 0.03, 0.045], np.linspace(0.5, 3, N - 4)])
    M = Qm @ np.diag(ev) @ Qm.conj().T
    M = (M + M.conj().T) / 2
    A, Ad = _ops(M)
    b = rng.standard_normal(N) + 0j
    r = K.eigbicg(A, Ad, b, np.zeros_like(b), 4, 16, 1e-12)
    assert np.abs(r.lam.imag).max() < 1e-8
    assert np.all(_nearest_rel(r.lam, ev) < 1e-8)


def test_m_must_exceed_2nev():
    M, _, rng = _generic()
    A, Ad = _ops(M)
    b = np.ones(M.shape[0], complex)
    with pytest.raises(ValueError):
        K.eigbicg(A, Ad, b, np.zeros_like(b), 4, 8, 1e-8)


# --------------------------------------------------------------- gamma5 relations
def test_gamma5_shadow_breakdown_with_z2_source():
    """rhat0 = gamma5 r0 with a Z2 source and x0 = 0: (rhat0, r0) = 6V - 6V = 0."""
    dims = (2, 2, 2, 2)
    U, V, A, Ad = _wilson(dims, 0.12, 1000)
    b = synth.z2_source(V, 10**6).ravel()
    g5b = W.apply_gamma5(b.reshape(V, 4, 3)).ravel()
    assert np.vdot(g5b, b) == 0
    with pytest.raises(K.Breakdown):
        K.eigbicg(A, Ad, b, np.zeros_like(b), 2, 10, 1e-10, rhat0=g5b)


def test_gamma5_shadow_keeps_rhat_gamma5_r():
    """rhat0 = gamma5 r0 gives rhat_j = gamma5 r_j (Sec. 4): the left window is gamma5 (right)."""
    dims = (2, 2, 2, 2)
    U, V, A, Ad = _wilson(dims, 0.12, 1000)
    b = synth.gaussian_spinor(V, 3).ravel()
    g5 = lambda v: W.apply_gamma5(v.reshape(V, 4, 3)).ravel()
    r = K.eigbicg(A, Ad, b, np.zeros_like(b), 2, 60, 1e-30, maxiter=20, rhat0=g5(b))
    Vw, Ww = r.V_final, r.W_final
    for i in range(Vw.shape[1]):
        g = g5(Vw[:, i])
        c = np.vdot(g, Ww[:, i]) / np.vdot(g, g)
        assert np.linalg.norm(Ww[:, i] - c * g) <= 1e-9 * np.linalg.norm(Ww[:, i])


# --------------------------------------------------------------- incremental phase
def test_incremental_invariants_and_deflation():
    M, lam_exact, rng = _generic()
    A, Ad = _ops(M)
    N = M.shape[0]
    space = K.DeflationSpace.empty(N)
    iters = []
    for k in range(3):
        b = rng.standard_normal(N) + 0j
        x0 = K.deflate_guess(A, space, b, np.zeros(N, complex))
        if space.K:
            r0 = b - A(x0)
            assert np.linalg.norm(space.Ul.conj().T @ r0) <= 1e-10 * np.linalg.norm(r0)
        x, res, space, tr, extra = K.solve_eigbicg(A, Ad, b, np.zeros(N, complex), space, 4, 16, 1e-10)
        iters.append(res.iters)
        assert tr <= 1e-10
        assert np.abs(space.Ul.conj().T @ space.Ur - np.eye(space.K)).max() < 1e-9
        assert np.abs(space.Ul.conj().T @ (M @ space.Ur) - space.H).max() < 1e-9
    assert space.K == 12
    lam, Ur, Ul = K.rayleigh_ritz(space)
    assert np.all(_nearest_rel(lam_exact[:4], lam) < 1e-7)


def test_deflated_bicgstab_matches_lapack():
    M, _, rng = _generic()
    A, Ad = _ops(M)
    N = M.shape[0]
    _, _, space = K.incremental_eigbicg(A, Ad, [rng.standard_normal(N) + 0j for _ in range(2)],
                                        [np.zeros(N, complex)] * 2, 4, 16, 1e-10, n1=2)
    b = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    xs = np.linalg.solve(M, b)
    plain = K.bicgstab(A, b, np.zeros(N, complex), 1e-10)
    x0 = K.deflate_guess(A, space, b, np.zeros(N, complex))
    defl = K.bicgstab(A, b, x0, 1e-10, space=space)
    for st in (plain, defl):
        assert st.converged and st.true_res <= 1e-10
        assert np.linalg.norm(st.x - xs) / np.linalg.norm(xs) < 1e-8
    assert defl.iters < plain.iters


def test_deftol_restart_path():
    M, _, rng = _generic()
    A, Ad = _ops(M)
    N = M.shape[0]
    _, _, space = K.incremental_eigbicg(A, Ad, [rng.standard_normal(N) + 0j for _ in range(2)],
                                        [np.zeros(N, complex)] * 2, 4, 16, 1e-10, n1=2)
    b = rng.standard_normal(N) + 0j
    x0 = K.deflate_guess(A, space, b, np.zeros(N, complex))
    # one restart per threshold DefTol^k ||b|| above tol ||b|| (Alg. Incremental
    # eigBiCG, step 3; a residual already below tol ends the solve instead):
    # 1e-3, 1e-6, 1e-9; 3e-3, 9e-6, 2.7e-8 (8.1e-11 is below tol); 1e-2 ...
    # 1e-8 (the fifth threshold equals tol: the converged solve ends there)
    for deftol, n in ((1e-3, 3), (3e-3, 3), (1e-2, 4)):
        st = K.bicgstab(A, b, x0, 1e-10, space=space, deftol=deftol)
        assert st.defl_restarts == n, (deftol, st.defl_restarts)
        assert st.converged
        assert np.linalg.norm(st.x - np.linalg.solve(M, b)) / np.linalg.norm(st.x) < 1e-8


def test_wilson_incremental_small_config():
    """4^4 at kappa 0.115: four eigBiCG solves then deflated BiCGStab, all to 1e-10."""
    dims = (4, 4, 4, 4)
    U, V, A, Ad = _wilson(dims, 0.115, 1000)
    B = [synth.z2_source(V, synth.rhs_seed(0, i)).ravel() for i in range(6)]
    X0 = [np.zeros_like(B[0])] * 6
    xs, info, space = K.incremental_eigbicg(A, Ad, B, X0, 4, 16, 1e-10, n1=4)
    assert space.K == 16
    for x, b, inf in zip(xs, B, info):
        assert np.linalg.norm(b - A(x)) / np.linalg.norm(b) <= 1e-10
    assert np.abs(space.Ul.conj().T @ space.Ur - np.eye(16)).max() < 1e-8
    # gamma5-Hermiticity: the Rayleigh-Ritz spectrum of a gamma5-symmetric space
    # need not be conjugate-symmetric, but every value lies in the field of values
    lam, Ur, Ul = K.rayleigh_ritz(space)
    assert np.all(lam.real > 0) and np.all(np.abs(lam) < 2)


# ------------------------------------------------- library routines (SciPy) as pins
def _scipy_iterates(solver, M, b, k):
    import scipy.sparse.linalg as spla

    N = M.shape[0]
    A, Ad = _ops(M)
    op = spla.LinearOperator((N, N), matvec=A, rmatvec=Ad, dtype=complex)
    xs = []
    solver(op, b, x0=np.zeros(N, complex), rtol=1e-30, atol=0, maxiter=k, callback=lambda x: xs.append(x.copy()))
    return xs


def test_bicgstab_iterates_equal_scipy():
    """Textbook BiCGStab (van der Vorst): SciPy's implementation gives the same iterates."""
    import scipy.sparse.linalg as spla

    M, _, rng = _generic()
    A, _ = _ops(M)
    N = M.shape[0]
    b = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    ref = _scipy_iterates(spla.bicgstab, M, b, 8)
    for k in (1, 2, 5, 8):
        st = K.bicgstab(A, b, np.zeros(N, complex), 1e-30, maxiter=k)
        assert np.linalg.norm(st.x - ref[k - 1]) <= 1e-13 * np.linalg.norm(ref[k - 1])


def test_bicg_iterates_equal_scipy():
    """Two-sided BiCG with rhat0 = r0: SciPy's bicg gives the same iterates."""
    import scipy.sparse.linalg as spla

    M, _, rng = _generic()
    A, Ad = _ops(M)
    N = M.shape[0]
    b = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    ref = _scipy_iterates(spla.bicg, M, b, 8)
    for k in (1, 3, 8):
        x, _, _ = K.bicg(A, Ad, b, np.zeros(N, complex), 1e-30, maxiter=k)
        assert np.linalg.norm(x - ref[k - 1]) <= 1e-13 * np.linalg.norm(ref[k - 1])
        r = K.eigbicg(A, Ad, b, np.zeros(N, complex), 2, 40, 1e-30, maxiter=k)
        assert np.linalg.norm(r.x - ref[k - 1]) <= 1e-13 * np.linalg.norm(ref[k - 1])
