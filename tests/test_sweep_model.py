"""The reordered QR sweep of the device eigensolver (winla.h, win_sweep_lanes)
against the entry-by-entry chase, as numpy models of both: the same rotations
applied to the same entries in the same order, so T and Q agree bit for bit.

The reordering: one lane per column carries its entry of the row that the next
row rotation mixes (the row below is still original); the 2 x 2 diagonal block
and the bulge are kept uniformly; the column rotations of the entries above the
block and of Q commute with the rest of the chase and run after it, one row per
lane.  The eigensolver itself is checked against LAPACK on the GPU
(test_gpu_wineig.py); this pins the argument that the two orders agree.
"""
import numpy as np
import pytest


def _givens(x, y):
    ax2, ay2 = abs(x) ** 2, abs(y) ** 2
    if ay2 == 0:
        return 1.0, 0j
    if ax2 == 0:
        return 0.0, np.conj(y) / abs(y)
    ax, r = np.sqrt(ax2), np.sqrt(ax2 + ay2)
    inv = 1 / (ax * r)
    return ax2 * inv, inv * (x * np.conj(y))


def chase(T, Z, l, ihi, mu):
    """Entry by entry: row rotation k on rows k, k+1, then column rotation k on
    columns k, k+1 of T (rows up to k+2) and of Z."""
    n = T.shape[0]
    for k in range(l, ihi):
        col = k if k == l else k - 1
        c, s = _givens(T[k, col] - (mu if k == l else 0), T[k + 1, col])
        sc = np.conj(s)
        for j in range(col, n):
            a, b = T[k, j], T[k + 1, j]
            T[k, j], T[k + 1, j] = c * a + s * b, c * b - sc * a
        if k > l:
            T[k + 1, k - 1] = 0
        for i in range(min(k + 2, ihi) + 1):
            a, b = T[i, k], T[i, k + 1]
            T[i, k], T[i, k + 1] = c * a + b * sc, c * b - a * s
        for i in range(n):
            a, b = Z[i, k], Z[i, k + 1]
            Z[i, k], Z[i, k + 1] = c * a + b * sc, c * b - a * s


def lane_sweep(T, Z, l, ihi, mu):
    """The device order: uniform 2 x 2 block (ua0, ua1 / ub0, ub1), one carried
    entry per far column, deferred column rotations of rows above the block and of Z."""
    n = T.shape[0]
    ua0, ua1, ub0, ub1 = T[l, l], T[l, l + 1], T[l + 1, l], T[l + 1, l + 1]
    cur = np.array([T[l, j] if j >= l + 2 else 0 for j in range(n)], complex)
    bnx = np.array([T[l + 1, j] if j >= l + 2 else 0 for j in range(n)], complex)
    x, y = ua0 - mu, ub0
    rots = []
    for k in range(l, ihi):
        more = k + 2 <= ihi
        F = T[k + 2, k + 1] if more else 0
        G = T[k + 2, k + 2] if more else 0
        bn2 = np.array([T[k + 2, j] if k + 2 < n else 0 for j in range(n)], complex)
        c, s = _givens(x, y)
        sc = np.conj(s)
        rots.append((c, s))
        A, C = c * ua0 + s * ub0, c * ub0 - sc * ua0
        B, D = c * ua1 + s * ub1, c * ub1 - sc * ua1
        for j in range(k + 2, n):
            top = c * cur[j] + s * bnx[j]
            cur[j] = c * bnx[j] - sc * cur[j]
            T[k, j] = top
        xn, dn = c * C + D * sc, c * D - C * s
        if k > l:
            T[k, k - 1] = c * x + s * y
            T[k + 1, k - 1] = 0
        T[k, k], T[k, k + 1] = c * A + B * sc, c * B - A * s
        x, ua0 = xn, dn
        if more:
            y, ub0, ub1, ua1 = F * sc, c * F, G, cur[k + 2]
        bnx = bn2
    T[ihi, ihi - 1], T[ihi, ihi] = x, ua0
    for j in range(ihi + 1, n):
        T[ihi, j] = cur[j]
    for i in range(n):
        k0 = max(l, i + 1)
        tdo = i <= ihi and k0 < ihi
        tc = T[i, k0] if tdo else 0
        zc = Z[i, l]
        for k in range(l, ihi):
            c, s = rots[k - l]
            sc = np.conj(s)
            zb = Z[i, k + 1]
            Z[i, k], zc = c * zc + zb * sc, c * zb - zc * s
            if tdo and k >= k0:
                tb = T[i, k + 1]
                T[i, k], tc = c * tc + tb * sc, c * tb - tc * s
        Z[i, ihi] = zc
        if tdo:
            T[i, ihi] = tc


@pytest.mark.parametrize("seed", range(6))
def test_lane_sweep_equals_chase(seed):
    rng = np.random.default_rng(seed)
    for _ in range(40):
        n = int(rng.integers(2, 24))
        l = int(rng.integers(0, n - 1))
        ihi = int(rng.integers(l + 1, n))
        T = np.triu(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)), -1)
        if l > 0:
            T[l, l - 1] = 0
        if ihi + 1 < n:
            T[ihi + 1, ihi] = 0
        Z = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        mu = complex(rng.standard_normal(), rng.standard_normal())
        T1, Z1, T2, Z2 = T.copy(), Z.copy(), T.copy(), Z.copy()
        chase(T1, Z1, l, ihi, mu)
        lane_sweep(T2, Z2, l, ihi, mu)
        assert np.array_equal(T1, T2) and np.array_equal(Z1, Z2), (n, l, ihi)


def test_sweep_is_a_similarity():
    """The chase itself: Z^+ T Z unchanged (T' = G^+ T G, Z' = Z G)."""
    rng = np.random.default_rng(7)
    n = 12
    T = np.triu(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)), -1)
    Z = np.eye(n, dtype=complex)
    A = T.copy()
    lane_sweep(T, Z, 0, n - 1, 0.3 + 0.1j)
    assert np.allclose(Z @ T @ Z.conj().T, A, atol=1e-12)
    assert np.allclose(Z.conj().T @ Z, np.eye(n), atol=1e-12)
    assert np.allclose(np.tril(T, -2), 0)
