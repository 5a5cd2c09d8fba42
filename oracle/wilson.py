"""Oracle: Wilson-Dirac operator (test infrastructure only).

The paper's matrices are quenched Wilson-Dirac operators (Sec. 3, "Results")
and Sec. 4 uses their gamma5-Hermiticity.  The paper does not write the
operator out; this file implements the standard form

    (D psi)(x) = psi(x) - kappa * sum_mu [ (1 - gamma_mu) U_mu(x) psi(x+mu)
                                         + (1 + gamma_mu) U_mu(x-mu)^+ psi(x-mu) ]

periodic in x, y, z and antiperiodic in t (every hop across the t boundary
picks up the factor ``bc_t``).  D^+ is coded independently (the projectors
swapped), not as gamma5 D gamma5, so that the identity gamma5 D gamma5 = D^+
of Sec. 4 is a test and not a tautology.

Layouts follow ``synth``: spinor complex128 [V][4][3], gauge [4][V][3][3],
s = x + Lx*(y + Ly*(z + Lz*t)).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

# Euclidean Hermitian gamma matrices in a chiral basis:
#   gamma_k = [[0, -i sigma_k], [i sigma_k, 0]] (k = 1,2,3),
#   gamma_4 = [[0, 1], [1, 0]],  gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4.
_SIGMA = [
    np.array([[0, 1], [1, 0]], dtype=np.complex128),
    np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    np.array([[1, 0], [0, -1]], dtype=np.complex128),
]
_Z2 = np.zeros((2, 2), dtype=np.complex128)
_I2 = np.eye(2, dtype=np.complex128)


def gammas() -> np.ndarray:
    """gamma_mu for mu = x, y, z, t, shape (4, 4, 4)."""
    g = [np.block([[_Z2, -1j * s], [1j * s, _Z2]]) for s in _SIGMA]
    g.append(np.block([[_Z2, _I2], [_I2, _Z2]]))
    return np.array(g)


def gamma5() -> np.ndarray:
    g = gammas()
    return g[0] @ g[1] @ g[2] @ g[3]


def _grid(dims):
    lx, ly, lz, lt = dims
    return (lt, lz, ly, lx)


# axis of the (t, z, y, x) grid that direction mu runs along
_AXIS = {0: 3, 1: 2, 2: 1, 3: 0}


def _shift(field, mu, step, dims, bc_t):
    """field(x + step*mu) on the (t,z,y,x,...) grid, with the t-boundary sign."""
    ax = _AXIS[mu]
    out = np.roll(field, -step, axis=ax)
    if mu == 3 and bc_t != 1:
        lt = dims[3]
        if step == 1:  # x at t = Lt-1 reads t = 0 across the boundary
            out[lt - 1] *= bc_t
        else:  # x at t = 0 reads t = Lt-1 across the boundary
            out[0] *= bc_t
    return out


def _hop(gauge, psi, dims, bc_t, fwd_proj, bwd_proj):
    """sum_mu [ fwd_proj[mu] U_mu(x) psi(x+mu) + bwd_proj[mu] U_mu(x-mu)^+ psi(x-mu) ]."""
    grid = _grid(dims)
    p = psi.reshape(grid + (4, 3))
    acc = np.zeros_like(p)
    for mu in range(4):
        U = gauge[mu].reshape(grid + (3, 3))
        fwd = _shift(p, mu, +1, dims, bc_t)
        t = np.einsum("...ab,...sb->...sa", U, fwd)
        acc += np.einsum("st,...tc->...sc", fwd_proj[mu], t)
        Ub = np.roll(U, 1, axis=_AXIS[mu])  # U_mu(x - mu)
        bwd = _shift(p, mu, -1, dims, bc_t)
        t = np.einsum("...ba,...sb->...sa", Ub.conj(), bwd)
        acc += np.einsum("st,...tc->...sc", bwd_proj[mu], t)
    return acc.reshape(psi.shape)


def _check(dims):
    if len(dims) != 4 or any(int(d) < 2 for d in dims):
        raise ValueError(f"every lattice extent must be >= 2, got {dims}")


def apply_D(gauge, psi, kappa, dims, bc_t=-1):
    """D psi (see module docstring)."""
    _check(dims)
    one = np.eye(4)
    g = gammas()
    return psi - kappa * _hop(gauge, psi, dims, bc_t, one - g, one + g)


def apply_Ddag(gauge, psi, kappa, dims, bc_t=-1):
    """D^+ psi, coded from the adjoint of each hop: projectors (1 +- gamma) swapped."""
    _check(dims)
    one = np.eye(4)
    g = gammas()
    return psi - kappa * _hop(gauge, psi, dims, bc_t, one + g, one - g)


def apply_gamma5(psi):
    return np.einsum("st,vtc->vsc", gamma5(), psi.reshape(-1, 4, 3)).reshape(psi.shape)


def site_coords(s, dims):
    lx, ly, lz, lt = dims
    return (s % lx, (s // lx) % ly, (s // (lx * ly)) % lz, s // (lx * ly * lz))


def site_index(x, y, z, t, dims):
    lx, ly, lz, lt = dims
    return (x % lx) + lx * ((y % ly) + ly * ((z % lz) + lz * (t % lt)))


def apply_D_sites(gauge, psi, kappa, dims, sites, bc_t=-1, dagger=False):
    """(D psi) or (D^+ psi) at a list of sites only, one site at a time.

    A direct transcription of the operator's definition, used to check large
    lattices at sampled outputs.  Returns complex128 [len(sites)][4][3].
    """
    _check(dims)
    g = gammas()
    one = np.eye(4)
    sgn = 1.0 if dagger else -1.0
    psi = psi.reshape(-1, 4, 3)
    out = np.empty((len(sites), 4, 3), dtype=np.complex128)
    for i, s in enumerate(sites):
        c = list(site_coords(int(s), dims))
        acc = np.zeros((4, 3), dtype=np.complex128)
        for mu in range(4):
            cf = list(c)
            cf[mu] += 1
            sf = site_index(*cf, dims)
            phase_f = bc_t if (mu == 3 and c[3] == dims[3] - 1) else 1.0
            acc += phase_f * (one + sgn * g[mu]) @ (psi[sf] @ gauge[mu, s].T)
            cb = list(c)
            cb[mu] -= 1
            sb = site_index(*cb, dims)
            phase_b = bc_t if (mu == 3 and c[3] == 0) else 1.0
            acc += phase_b * (one - sgn * g[mu]) @ (psi[sb] @ gauge[mu, sb].conj())
        out[i] = psi[int(s)] - kappa * acc
    return out


def dense_D(gauge, kappa, dims, bc_t=-1, dagger=False, sparse=False):
    """The matrix of D (or D^+) built block by block from the definition.

    Row/column index (s*4 + spin)*3 + colour.  Forward and backward hops that
    land on the same site (an extent of 2) are added, never overwritten.
    """
    _check(dims)
    V = int(np.prod(dims))
    g = gammas()
    one = np.eye(4)
    sgn = 1.0 if dagger else -1.0
    rows, cols, vals = [], [], []
    blk_r = np.repeat(np.arange(12), 12)
    blk_c = np.tile(np.arange(12), 12)
    for s in range(V):
        c = list(site_coords(s, dims))
        rows.append(s * 12 + np.arange(12))
        cols.append(s * 12 + np.arange(12))
        vals.append(np.ones(12, dtype=np.complex128))
        for mu in range(4):
            cf = list(c)
            cf[mu] += 1
            sf = site_index(*cf, dims)
            ph = bc_t if (mu == 3 and c[3] == dims[3] - 1) else 1.0
            blk = -kappa * ph * np.kron(one + sgn * g[mu], gauge[mu, s])
            rows.append(s * 12 + blk_r)
            cols.append(sf * 12 + blk_c)
            vals.append(blk.ravel())
            cb = list(c)
            cb[mu] -= 1
            sb = site_index(*cb, dims)
            ph = bc_t if (mu == 3 and c[3] == 0) else 1.0
            blk = -kappa * ph * np.kron(one - sgn * g[mu], gauge[mu, sb].conj().T)
            rows.append(s * 12 + blk_r)
            cols.append(sb * 12 + blk_c)
            vals.append(blk.ravel())
    M = sp.coo_matrix(
        (np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
        shape=(12 * V, 12 * V),
    ).tocsr()  # duplicate (row, col) entries are summed
    return M if sparse else M.toarray()


def free_field_spectrum(kappa, dims, bc_t=-1, phases=(0.0, 0.0, 0.0, 0.0)):
    """Closed-form eigenvalues of D for constant abelian links exp(i*theta_mu).

    A plane wave e^{i p.x} chi turns each direction's hop pair into
    2 cos(p'_mu) - 2 i gamma_mu sin(p'_mu) with p'_mu = p_mu + theta_mu, and
    (sum_mu gamma_mu s_mu)^2 = |s|^2, so
        lambda = 1 - 2 kappa sum_mu cos p'_mu  +-  2 i kappa sqrt(sum_mu sin^2 p'_mu),
    each sign six-fold (2 spins x 3 colours).  Momenta: 2 pi n / L in x,y,z;
    pi (2n+1) / Lt in t when bc_t = -1.
    """
    lx, ly, lz, lt = dims
    ks = []
    for L, mu in zip((lx, ly, lz, lt), range(4)):
        n = np.arange(L)
        if mu == 3 and bc_t == -1:
            ks.append(np.pi * (2 * n + 1) / L + phases[mu])
        else:
            ks.append(2 * np.pi * n / L + phases[mu])
    P = np.stack(np.meshgrid(*ks, indexing="ij"), axis=-1).reshape(-1, 4)
    re = 1 - 2 * kappa * np.cos(P).sum(axis=1)
    im = 2 * kappa * np.sqrt((np.sin(P) ** 2).sum(axis=1))
    lam = np.concatenate([re + 1j * im, re - 1j * im])
    return np.repeat(lam, 6)


# --------------------------------------------------------------- even-odd
# The paper's test matrices are even-odd preconditioned Wilson operators
# (Sec. 3, "Results"); the paper does not spell the form out, and this is the
# standard Schur complement.  With the sites split by parity (x+y+z+t even or
# odd) and H the hop sum above (D = 1 - kappa H), H only connects sites of
# opposite parity, so
#     D = [[1, -kappa H_eo], [-kappa H_oe, 1]],
#     Dhat = 1 - kappa^2 H_eo H_oe            (on the even sites),
#     D x = b  <=>  Dhat x_e = b_e + kappa H_eo b_o,  x_o = b_o + kappa H_oe x_e.
# Half-lattice vectors hold the sites of one parity in increasing site order.


def parity(dims):
    """(x + y + z + t) mod 2 for every site s, shape (V,)."""
    lx, ly, lz, lt = dims
    s = np.arange(lx * ly * lz * lt)
    x, y, z, t = s % lx, (s // lx) % ly, (s // (lx * ly)) % lz, s // (lx * ly * lz)
    return (x + y + z + t) % 2


def _check_eo(dims):
    _check(dims)
    if any(int(d) % 2 for d in dims):
        raise ValueError(f"even-odd ordering needs even extents, got {dims}")


def _embed(half, par, p):
    full = np.zeros((par.size, 4, 3), dtype=np.complex128)
    full[par == p] = half.reshape(-1, 4, 3)
    return full


def _hop_full(gauge, psi, dims, bc_t, dagger):
    one = np.eye(4)
    g = gammas()
    if dagger:
        return _hop(gauge, psi, dims, bc_t, one + g, one - g)
    return _hop(gauge, psi, dims, bc_t, one - g, one + g)


def apply_Dhat(gauge, psi_e, kappa, dims, bc_t=-1, dagger=False):
    """Dhat psi_e (or Dhat^+ psi_e, built from the adjoint hops) on the even sites.

    psi_e: complex128 [V/2][4][3], the even sites in increasing site order.
    """
    _check_eo(dims)
    par = parity(dims)
    t = _hop_full(gauge, _embed(psi_e, par, 0), dims, bc_t, dagger)[par == 1]
    u = _hop_full(gauge, _embed(t, par, 1), dims, bc_t, dagger)[par == 0]
    return psi_e.reshape(-1, 4, 3) - kappa * kappa * u


def eo_prepare(gauge, b, kappa, dims, bc_t=-1):
    """b_e + kappa H_eo b_o: the right-hand side of the even system."""
    _check_eo(dims)
    par = parity(dims)
    b = b.reshape(-1, 4, 3)
    hb = _hop_full(gauge, _embed(b[par == 1], par, 1), dims, bc_t, False)[par == 0]
    return b[par == 0] + kappa * hb


def eo_reconstruct(gauge, x_e, b, kappa, dims, bc_t=-1):
    """The full solution from x_e: x_o = b_o + kappa H_oe x_e."""
    _check_eo(dims)
    par = parity(dims)
    b = b.reshape(-1, 4, 3)
    hx = _hop_full(gauge, _embed(x_e, par, 0), dims, bc_t, False)[par == 1]
    x = np.zeros_like(b)
    x[par == 0] = x_e.reshape(-1, 4, 3)
    x[par == 1] = b[par == 1] + kappa * hx
    return x
