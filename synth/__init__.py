"""Seeded synthetic inputs shared by the oracle and the GPU library's tests.

This module holds no arithmetic of the solver method: it only draws the inputs
that both sides consume (gauge links, Z2 noise sources, initial guesses), so
that the oracle and the HIP path see bit-identical data.

Canonical layouts (the library's C-ABI uses the same ones):

* site index  s = x + Lx*(y + Ly*(z + Lz*t)), directions mu = 0,1,2,3 <-> x,y,z,t
* gauge field complex128 [4][V][3][3]; U[mu, s, a, b] is row a, column b of U_mu(s)
* spinor      complex128 [V][4][3];  element (s, spin, colour)

The paper tests on quenched Wilson gauge configurations that are not available
here (Sec. 3); these generators stand in for them with smooth random SU(3)
links U = exp(i*eps*H), H a traceless Hermitian Gaussian matrix.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "volume",
    "gell_mann",
    "random_su3_links",
    "unit_links",
    "z2_source",
    "gauge_seed",
    "rhs_seed",
    "gaussian_spinor",
]


def volume(dims) -> int:
    lx, ly, lz, lt = (int(d) for d in dims)
    return lx * ly * lz * lt


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices, shape (8, 3, 3), complex128."""
    g = np.zeros((8, 3, 3), dtype=np.complex128)
    g[0][0, 1] = g[0][1, 0] = 1
    g[1][0, 1], g[1][1, 0] = -1j, 1j
    g[2][0, 0], g[2][1, 1] = 1, -1
    g[3][0, 2] = g[3][2, 0] = 1
    g[4][0, 2], g[4][2, 0] = -1j, 1j
    g[5][1, 2] = g[5][2, 1] = 1
    g[6][1, 2], g[6][2, 1] = -1j, 1j
    g[7][0, 0] = g[7][1, 1] = 1 / np.sqrt(3)
    g[7][2, 2] = -2 / np.sqrt(3)
    return g


def random_su3_links(dims, eps: float, seed: int, chunk: int = 1 << 18) -> np.ndarray:
    """SU(3) links U = exp(i*eps*H), H = sum_a c_a lambda_a / 2, c_a ~ N(0,1).

    Coefficients are drawn from PCG64(seed) in the order (mu, site, a).  The
    exponential is taken exactly through the eigendecomposition of H, so
    U is unitary with unit determinant to rounding.  Returns complex128
    [4][V][3][3].
    """
    V = volume(dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    c = rng.standard_normal((4 * V, 8))
    lam = gell_mann() / 2
    out = np.empty((4 * V, 3, 3), dtype=np.complex128)
    for lo in range(0, 4 * V, chunk):
        hi = min(4 * V, lo + chunk)
        H = np.einsum("na,aij->nij", c[lo:hi], lam)
        w, Q = np.linalg.eigh(H)
        ph = np.exp(1j * eps * w)
        out[lo:hi] = np.einsum("nij,nj,nkj->nik", Q, ph, Q.conj())
    return out.reshape(4, V, 3, 3)


def unit_links(dims, phases=(0.0, 0.0, 0.0, 0.0)) -> np.ndarray:
    """Links U_mu(x) = exp(i*phases[mu]) * 1 (free field when all phases are 0)."""
    V = volume(dims)
    out = np.zeros((4, V, 3, 3), dtype=np.complex128)
    for mu in range(4):
        out[mu] = np.exp(1j * phases[mu]) * np.eye(3)
    return out


def z2_source(V: int, seed: int) -> np.ndarray:
    """Z2 noise: every complex entry is +1 or -1 (real), complex128 [V][4][3]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    s = rng.choice(np.array([-1.0, 1.0]), size=12 * V)
    return s.astype(np.complex128).reshape(V, 4, 3)


def gaussian_spinor(V: int, seed: int) -> np.ndarray:
    """Complex Gaussian spinor (re, im ~ N(0,1)), complex128 [V][4][3]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.standard_normal((12 * V, 2))
    return (a[:, 0] + 1j * a[:, 1]).reshape(V, 4, 3)


def gauge_seed(config_index: int, operator_index: int = 0) -> int:
    """Seed of the gauge field of a workload (1000 + index, +40 + operator for the mixes)."""
    return 1000 + int(config_index) if operator_index == 0 else 1040 + int(operator_index)


def rhs_seed(operator_index: int, i: int) -> int:
    """Seed of right-hand side i of operator o: 10^6 + 10^3 * o + i."""
    return 10**6 + 10**3 * int(operator_index) + int(i)
