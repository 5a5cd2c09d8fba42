"""The one-workgroup device eigensolver of the window (eb_small_eig_device) against LAPACK
(the oracle's eig) and the host solver: eigenvalues, right and left residuals, the
biorthonormal normalisation, and the order (Sec. 1, end: sorted by |lambda|).  Sizes
cover the LDS-resident Schur chase (n <= 56) and the global-memory one (n > 56)."""
import numpy as np
import pytest

from oracle.eig import eig as oracle_eig

pytestmark = pytest.mark.gpu


def _check(eb, C, tol=1e-11):
    n = C.shape[0]
    y, z, lam = eb.small_eig_device(C)
    yh, zh, lh = eb.small_eig(C)
    _, _, lr = oracle_eig(C)
    sc = max(1.0, np.abs(C).max())
    err_l = np.abs(lam - lr).max() / max(1.0, np.abs(lr).max())
    res_r = np.abs(C @ y - y * lam).max() / sc
    res_l = np.abs(z.conj().T @ C - lam[:, None] * z.conj().T).max() / sc
    print(f"n {n}: eigenvalues vs LAPACK {err_l:.1e}, right residual {res_r:.1e}, left {res_l:.1e}, "
          f"vs host solver {np.abs(lam - lh).max():.1e}")
    assert err_l <= tol and np.abs(lam - lh).max() <= tol * max(1.0, np.abs(lh).max())
    assert res_r < tol * n and res_l < tol * n
    assert np.abs(np.diag(z.conj().T @ y) - 1).max() < 1e-11
    assert np.allclose(np.linalg.norm(y, axis=0), 1)
    return lam


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (7, 2), (16, 3), (40, 4), (56, 5), (57, 6), (100, 7), (128, 8)])
def test_device_eig_random(gpu_lib, n, seed):
    rng = np.random.default_rng(seed)
    C = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    _check(gpu_lib, C)


def test_device_eig_structured(gpu_lib):
    """The shapes of the restarted window matrix: tridiagonal with an arrow row and column,
    real matrices (conjugate pairs), repeated eigenvalues, a diagonal matrix."""
    rng = np.random.default_rng(9)
    n = 40
    T = np.diag(rng.standard_normal(n) + 0.1j * rng.standard_normal(n)) + np.diag(rng.standard_normal(n - 1), 1)
    T += np.diag(rng.standard_normal(n - 1), -1)
    T[20, :20] = rng.standard_normal(20)
    T[:20, 20] = rng.standard_normal(20)
    D = np.diag([3.0, 1.0, 2.0, 1.0, 2.0 + 0.5j, 2.0 - 0.5j]).astype(complex)
    R = rng.standard_normal((30, 30)).astype(complex)
    for C in (T.astype(complex), R):
        _check(gpu_lib, C)
    y, z, lam = gpu_lib.small_eig_device(D)
    assert np.allclose(lam, [1.0, 1.0, 2.0, 2.0 + 0.5j, 2.0 - 0.5j, 3.0])
