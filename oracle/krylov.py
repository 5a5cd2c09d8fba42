"""Oracle: BiCG, eigBiCG, incremental eigBiCG and deflated BiCGStab (test infrastructure only).

Plain complex128 NumPy.  Operators are passed as callables ``A(v)`` and
``Ad(v)`` (for A and A^+), so the same code runs on the Wilson operator of
``oracle.wilson`` and on dense test matrices.  Vectors are 1-D arrays of
length N; (w, v) := w^+ v as in the paper (Sec. 1, end).

Readings of the paper used here (the paper is silent or garbled on them):

* index typos in Alg. eigBiCG are read as: x_j = x_{j-1} + alpha p_{j-1};
  rhat_j = rhat_{j-1} - conj(alpha) A^+ phat_{j-1}; beta_{j-2} in the
  diagonal of H; Q = W z^(nev) in the final step.
* w_vs = (||r||/conj(rho)) rhat, as in the listing (the text's w_1 would
  give w^+ v = 1/||r_0||).
* the default shadow residual is rhat_0 = r_0 (Sec. 2, "Normally ...").
* Alg. BiCG-eigen biorthogonalises the 2nev coefficient vectors with a
  two-sided Gram-Schmidt pass (twice) that leaves the first nev, already
  biorthogonal, untouched; a new pair whose pivot z^+ y falls below
  1e-12 |y||z| is dropped (vs then restarts at the number kept).
* the incremental step "biorthogonalize [V, W] against [U_r, U_l]" is a
  two-sided Gram-Schmidt (twice) of each new pair against the existing
  space and the earlier new pairs; columns are scaled to ||v|| = 1 and
  w^+ v = 1.
* DefTol: when ||r|| < thr, with thr = DefTol ||b|| at the start, deflate
  again from the current x, restart BiCGStab, and lower thr by the factor
  DefTol.  DefTol = 0 disables it (the setting of Fig. 1).
* convergence is declared on the recursive residual (Alg. eigBiCG, last
  step of the loop); a solve whose true residual ||b - A x|| is then above
  tol * ||b|| continues with a BiCGStab cycle from x.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .eig import eig, sort_order


def dot(w, v):
    """(w, v) = w^+ v."""
    return np.vdot(w, v)


def nrm(v):
    return float(np.linalg.norm(v))


class Breakdown(RuntimeError):
    """(rhat, r) or (phat, A p) vanished: BiCG cannot continue."""


# ---------------------------------------------------------------------------
# Alg. BiCG-eigen
# ---------------------------------------------------------------------------
@dataclass
class RestartRecord:
    """What one window restart computed (kept for the tests' invariants)."""

    H_before: np.ndarray
    CV: np.ndarray  # V_new = V_old @ CV   (m x kept)
    CW: np.ndarray  # W_new = W_old @ CW
    Lam: np.ndarray
    arrow_row: np.ndarray = None  # H[2nev+1, k], k <= kept, from the dot products
    arrow_col: np.ndarray = None  # H[k, 2nev+1]
    h_next_prev: complex = 0j  # H_{m+1,m} from the BiCG scalars (not stored in H)
    h_prev_next: complex = 0j  # H_{m,m+1}
    V_new: np.ndarray = None  # the restarted bases (only when the caller keeps records)
    W_new: np.ndarray = None


def _biorth_gs(Y, Z, start, passes=2, tol=1e-12):
    """Two-sided Gram-Schmidt of columns start.. of Y, Z against all earlier ones.

    Assumes Z[:, :start]^+ Y[:, :start] = I.  Returns (Y, Z) with the kept
    columns satisfying Z^+ Y = I, ||y_k|| = 1.
    """
    ys = [Y[:, i].copy() for i in range(start)]
    zs = [Z[:, i].copy() for i in range(start)]
    for k in range(start, Y.shape[1]):
        y, z = Y[:, k].copy(), Z[:, k].copy()
        for _ in range(passes):
            for yi, zi in zip(ys, zs):
                y = y - yi * dot(zi, y)
                z = z - zi * dot(yi, z)
        piv = dot(z, y)
        if abs(piv) <= tol * nrm(y) * nrm(z):
            continue
        y = y / nrm(y)
        z = z / np.conj(dot(z, y))
        ys.append(y)
        zs.append(z)
    return np.stack(ys, axis=1), np.stack(zs, axis=1)


def bicg_eigen(nev, m, H, which="SM"):
    """Alg. BiCG-eigen in coefficient space; ``which`` is the sort criterion of
    every eig() call (oracle.eig.sort_order).

    Returns (CV, CW, Lam): the restarted bases are V_old @ CV and W_old @ CW,
    and the restarted H is diag(Lam).
    """
    y, z, _ = eig(H[:m, :m], which)
    y1, z1, _ = eig(H[: m - 1, : m - 1], which)
    y1 = np.vstack([y1, np.zeros((1, m - 1))])  # append a zero to each vector
    z1 = np.vstack([z1, np.zeros((1, m - 1))])
    Y = np.hstack([y[:, :nev], y1[:, :nev]])
    Z = np.hstack([z[:, :nev], z1[:, :nev]])
    Yt, Zt = _biorth_gs(Y, Z, start=nev)
    T = Zt.conj().T @ H[:m, :m] @ Yt
    u, q, Lam = eig(T, which)
    CV = Yt @ u
    CW = Zt @ q
    sc = np.linalg.norm(CV, axis=0)
    CV = CV / sc
    CW = CW * sc  # keeps CW_i^+ CV_i = q_i^+ u_i = 1
    return CV, CW, Lam


# ---------------------------------------------------------------------------
# Alg. eigBiCG
# ---------------------------------------------------------------------------
@dataclass
class EigBiCGResult:
    x: np.ndarray
    iters: int
    converged: bool
    lam: np.ndarray
    U: np.ndarray  # right Ritz vectors, N x nev
    Q: np.ndarray  # left Ritz vectors
    res_hist: list = field(default_factory=list)
    restarts: list = field(default_factory=list)
    H_final: np.ndarray = None
    V_final: np.ndarray = None
    W_final: np.ndarray = None
    matvecs: int = 0


def eigbicg(A, Ad, b, x0, nev, m, tol, maxiter=10000, rhat0=None, keep_restarts=False, which="SM"):
    """Alg. eigBiCG: two-sided BiCG that keeps a window of m residuals.

    With m >= iterations + 1 no restart occurs and this is the un-restarted
    BiCG that stores every residual (the comparison run of Table 1).  ``which``
    selects the eigenpairs kept at each restart and returned (the sort
    criterion of eig(), Sec. 1, end).
    """
    if m <= 2 * nev:
        raise ValueError("eigBiCG needs m > 2 nev")
    N = b.shape[0]
    x = x0.astype(np.complex128).copy()
    r = b - A(x)
    rhat = r.copy() if rhat0 is None else rhat0.astype(np.complex128).copy()
    p, phat = r.copy(), rhat.copy()
    rho = dot(rhat, r)
    nb = nrm(b)
    rn = nrm(r)
    if abs(rho) <= 1e-14 * nrm(rhat) * rn:
        raise Breakdown("(rhat0, r0) = 0")
    V = np.zeros((N, m), dtype=np.complex128)
    W = np.zeros((N, m), dtype=np.complex128)
    H = np.zeros((m, m), dtype=np.complex128)
    vs = 0
    q = s = None
    alpha_prev = beta_prev = None
    res = EigBiCGResult(x=x, iters=0, converged=False, lam=None, U=None, Q=None)
    res.res_hist.append(rn)
    matvecs = 1
    if rn <= tol * nb:
        res.converged = True
    j = 0
    while not res.converged and j < maxiter:
        j += 1
        Ap = A(p)
        Adp = Ad(phat)
        matvecs += 2
        sigma = dot(phat, Ap)
        if abs(sigma) <= 1e-14 * nrm(phat) * nrm(Ap):
            raise Breakdown("(phat, A p) = 0")
        alpha = rho / sigma
        x = x + alpha * p
        if vs == m - 1:
            q, s = Ap.copy(), Adp.copy()
        if vs == m:
            rec = RestartRecord(H_before=H.copy(), CV=None, CW=None, Lam=None)
            CV, CW, Lam = bicg_eigen(nev, m, H, which)
            kept = CV.shape[1]
            Vn, Wn = V @ CV, W @ CW
            V[:] = 0
            W[:] = 0
            V[:, :kept], W[:, :kept] = Vn, Wn
            H[:] = 0
            H[np.arange(kept), np.arange(kept)] = Lam
            vs = kept
            # arrow entries of row and column 2nev+1 (0-based index `kept`)
            # A^+ rhat_{j-1} = A^+ phat_{j-1} - conj(beta_{j-2}) s and
            # A r_{j-1} = A p_{j-1} - beta_{j-2} q
            ga = Adp - np.conj(beta_prev) * s
            gb = Ap - beta_prev * q
            for k in range(kept):
                H[kept, k] = (rn / rho) * dot(ga, V[:, k])
                H[k, kept] = dot(W[:, k], gb) / rn
            if keep_restarts:
                rec.CV, rec.CW, rec.Lam = CV, CW, Lam
                rec.V_new, rec.W_new = Vn.copy(), Wn.copy()
                rec.arrow_row = H[kept, :kept].copy()
                rec.arrow_col = H[:kept, kept].copy()
                # H_{m+1,m}, H_{m,m+1} of the un-restarted process (rn = ||r_{j-1}||)
                rec.h_next_prev = -(rn / res._rn_prev) / alpha_prev
                rec.h_prev_next = -(res._rn_prev / rn) * beta_prev / alpha_prev
                res.restarts.append(rec)
            else:
                res.restarts.append(None)
        vs += 1
        V[:, vs - 1] = r / rn
        W[:, vs - 1] = (rn / np.conj(rho)) * rhat
        r_new = r - alpha * Ap
        rhat = rhat - np.conj(alpha) * Adp
        rho_new = dot(rhat, r_new)
        beta = rho_new / rho
        p = r_new + beta * p
        phat = rhat + np.conj(beta) * phat
        rn_new = nrm(r_new)
        if j == 1:
            H[vs - 1, vs - 1] = 1 / alpha
        else:
            H[vs - 1, vs - 1] = 1 / alpha + beta_prev / alpha_prev
        if vs < m:
            H[vs - 1, vs] = -(rn / rn_new) * beta / alpha
            H[vs, vs - 1] = -(rn_new / rn) / alpha
        res._rn_prev = rn
        r, rho, rn = r_new, rho_new, rn_new
        alpha_prev, beta_prev = alpha, beta
        res.res_hist.append(rn)
        if rn <= tol * nb:
            res.converged = True
        elif abs(rho) <= 1e-14 * nrm(rhat) * rn:
            raise Breakdown("(rhat_j, r_j) = 0")
    res.x, res.iters, res.matvecs = x, j, matvecs
    # final nev eigenpairs from V^(vs), W^(vs), H^(vs)
    if vs > 0:
        y, z, lam = eig(H[:vs, :vs], which)
        k = min(nev, vs)
        U = V[:, :vs] @ y[:, :k]
        Q = W[:, :vs] @ z[:, :k]
        U, Q = _normalise_pairs(U, Q)
        res.lam, res.U, res.Q = lam[:k], U, Q
    else:
        res.lam = np.zeros(0, dtype=np.complex128)
        res.U = np.zeros((N, 0), dtype=np.complex128)
        res.Q = np.zeros((N, 0), dtype=np.complex128)
    res.H_final, res.V_final, res.W_final = H[:vs, :vs].copy(), V[:, :vs].copy(), W[:, :vs].copy()
    return res


def _normalise_pairs(U, Q):
    """||U_i|| = 1 and Q_i^+ U_i = 1."""
    U = U / np.linalg.norm(U, axis=0)
    d = np.einsum("ij,ij->j", Q.conj(), U)
    return U, Q / d.conj()


def bicg(A, Ad, b, x0, tol, maxiter=10000, rhat0=None):
    """Plain two-sided BiCG (eigBiCG without the window); returns (x, iters, res_hist)."""
    x = x0.astype(np.complex128).copy()
    r = b - A(x)
    rhat = r.copy() if rhat0 is None else rhat0.astype(np.complex128).copy()
    p, phat = r.copy(), rhat.copy()
    rho = dot(rhat, r)
    nb = nrm(b)
    hist = [nrm(r)]
    j = 0
    while hist[-1] > tol * nb and j < maxiter:
        j += 1
        Ap, Adp = A(p), Ad(phat)
        alpha = rho / dot(phat, Ap)
        x = x + alpha * p
        r = r - alpha * Ap
        rhat = rhat - np.conj(alpha) * Adp
        rho_new = dot(rhat, r)
        beta = rho_new / rho
        p = r + beta * p
        phat = rhat + np.conj(beta) * phat
        rho = rho_new
        hist.append(nrm(r))
    return x, j, hist


def cg(A, b, x0, tol, maxiter=10000):
    """Textbook conjugate gradients (Hestenes-Stiefel), for the Hermitian reduction test."""
    x = x0.astype(np.complex128).copy()
    r = b - A(x)
    p = r.copy()
    rr = dot(r, r).real
    hist = [np.sqrt(rr)]
    nb = nrm(b)
    j = 0
    while hist[-1] > tol * nb and j < maxiter:
        j += 1
        Ap = A(p)
        alpha = rr / dot(p, Ap)
        x = x + alpha * p
        r = r - alpha * Ap
        rr_new = dot(r, r).real
        p = r + (rr_new / rr) * p
        rr = rr_new
        hist.append(np.sqrt(rr))
    return x, j, hist


# ---------------------------------------------------------------------------
# Alg. Incremental eigBiCG: the deflation space (U_l, U_r, H)
# ---------------------------------------------------------------------------
@dataclass
class DeflationSpace:
    Ul: np.ndarray  # left vectors, N x K
    Ur: np.ndarray  # right vectors, N x K
    H: np.ndarray  # Ul^+ A Ur, K x K

    @staticmethod
    def empty(N):
        z = np.zeros((N, 0), dtype=np.complex128)
        return DeflationSpace(z, z.copy(), np.zeros((0, 0), dtype=np.complex128))

    @property
    def K(self):
        return self.Ur.shape[1]


def deflate_guess(A, space, b, x0):
    """x0 + U_r d with H d = U_l^+ (b - A x0)  (step 2, first item, and step 3)."""
    if space.K == 0:
        return x0.copy()
    c = space.Ul.conj().T @ (b - A(x0))
    d = np.linalg.solve(space.H, c)
    return x0 + space.Ur @ d


def absorb(A, Ad, space, U, Q, passes=2, tol=1e-12):
    """Biorthogonalise the new pairs against [U_r, U_l] and extend H (step 2, items 3-5)."""
    Vn, Wn = [], []
    for k in range(U.shape[1]):
        v, w = U[:, k].copy(), Q[:, k].copy()
        for _ in range(passes):
            if space.K:
                v = v - space.Ur @ (space.Ul.conj().T @ v)
                w = w - space.Ul @ (space.Ur.conj().T @ w)
            for vi, wi in zip(Vn, Wn):
                v = v - vi * dot(wi, v)
                w = w - wi * dot(vi, w)
        piv = dot(w, v)
        if abs(piv) <= tol * nrm(v) * nrm(w):
            continue
        v = v / nrm(v)
        w = w / np.conj(dot(w, v))
        Vn.append(v)
        Wn.append(w)
    if not Vn:
        return space
    Vp, Wp = np.stack(Vn, axis=1), np.stack(Wn, axis=1)
    AV = np.stack([A(Vp[:, i]) for i in range(Vp.shape[1])], axis=1)
    AdW = np.stack([Ad(Wp[:, i]) for i in range(Wp.shape[1])], axis=1)
    H = np.block(
        [
            [space.H, space.Ul.conj().T @ AV],
            [AdW.conj().T @ space.Ur, Wp.conj().T @ AV],
        ]
    )
    return DeflationSpace(np.hstack([space.Ul, Wp]), np.hstack([space.Ur, Vp]), H)


def rayleigh_ritz(space):
    """Eigenpairs of A from the space: eig(H), H = U_l^+ A U_r (Sec. 2, closing remark)."""
    y, z, lam = eig(space.H)
    U, Q = _normalise_pairs(space.Ur @ y, space.Ul @ z)
    return lam, U, Q


# ---------------------------------------------------------------------------
# BiCGStab with deflation restarts
# ---------------------------------------------------------------------------
@dataclass
class SolveResult:
    x: np.ndarray
    iters: int
    converged: bool
    defl_restarts: int = 0
    true_res: float = np.nan
    res_hist: list = field(default_factory=list)


def bicgstab(A, b, x0, tol, maxiter=10000, space=None, deftol=0.0):
    """BiCGStab (van der Vorst 1992) with the DefTol deflation restart.

    The shadow vector is rhat = r at every (re)start.
    """
    nb = nrm(b)
    x = x0.astype(np.complex128).copy()
    out = SolveResult(x=x, iters=0, converged=False)
    thr = deftol * nb
    it = 0
    while True:
        r = b - A(x)
        rhat = r.copy()
        rho = alpha = omega = 1.0 + 0j
        v = np.zeros_like(r)
        p = np.zeros_like(r)
        rn = nrm(r)
        out.res_hist.append(rn)
        restart = False
        while rn > tol * nb and it < maxiter:
            it += 1
            rho_new = dot(rhat, r)
            beta = (rho_new / rho) * (alpha / omega)
            p = r + beta * (p - omega * v)
            v = A(p)
            alpha = rho_new / dot(rhat, v)
            s = r - alpha * v
            t = A(s)
            omega = dot(t, s) / dot(t, t)
            x = x + alpha * p + omega * s
            r = s - omega * t
            rho = rho_new
            rn = nrm(r)
            out.res_hist.append(rn)
            # a residual that already meets tol ends the solve; the DefTol
            # restart applies only above it
            if space is not None and space.K and rn < thr and rn > tol * nb:
                x = deflate_guess(A, space, b, x)
                out.defl_restarts += 1
                thr *= deftol
                restart = True
                break
        if restart:
            continue
        tr = nrm(b - A(x))
        if tr <= tol * nb or it >= maxiter:
            out.true_res = tr / nb
            out.converged = tr <= tol * nb
            break
    out.x, out.iters = x, it
    return out


def solve_eigbicg(A, Ad, b, x0, space, nev, m, tol, maxiter=10000):
    """One solve of the first phase: deflate x0, eigBiCG, true-residual check, absorb."""
    nb = nrm(b)
    x0 = deflate_guess(A, space, b, x0)
    res = eigbicg(A, Ad, b, x0, nev, m, tol, maxiter)
    x = res.x
    tr = nrm(b - A(x))
    extra = 0
    if tr > tol * nb:
        st = bicgstab(A, b, x, tol, maxiter)
        x, extra, tr = st.x, st.iters, st.true_res * nb
    new_space = absorb(A, Ad, space, res.U, res.Q)
    return x, res, new_space, tr / nb, extra


def incremental_eigbicg(A, Ad, B, X0, nev, m, tol, n1, deftol=0.0, maxiter=10000):
    """Alg. Incremental eigBiCG over the right-hand sides B[k] (a list of vectors).

    Returns (solutions, per-RHS info dicts, final deflation space).
    """
    N = B[0].shape[0]
    space = DeflationSpace.empty(N)
    xs, info = [], []
    for k, b in enumerate(B):
        if k < n1:
            x, res, space, tr, extra = solve_eigbicg(A, Ad, b, X0[k], space, nev, m, tol, maxiter)
            info.append(dict(kind="eigbicg", iters=res.iters + extra, true_res=tr, lam=res.lam, K=space.K))
        else:
            x0 = deflate_guess(A, space, b, X0[k])
            st = bicgstab(A, b, x0, tol, maxiter, space=space, deftol=deftol)
            x = st.x
            info.append(
                dict(kind="bicgstab", iters=st.iters, true_res=st.true_res, defl_restarts=st.defl_restarts)
            )
        xs.append(x)
    return xs, info, space


def ritz_residuals(A, Ad, lam, U, Q):
    """Right and left residual norms ||A u - lam u|| / ||u|| and ||A^+ q - conj(lam) q|| / ||q||."""
    rr = np.array([nrm(A(U[:, i]) - lam[i] * U[:, i]) / nrm(U[:, i]) for i in range(U.shape[1])])
    rl = np.array([nrm(Ad(Q[:, i]) - np.conj(lam[i]) * Q[:, i]) / nrm(Q[:, i]) for i in range(Q.shape[1])])
    return rr, rl


__all__ = [
    "dot",
    "nrm",
    "Breakdown",
    "bicg_eigen",
    "eigbicg",
    "bicg",
    "cg",
    "DeflationSpace",
    "deflate_guess",
    "absorb",
    "rayleigh_ritz",
    "bicgstab",
    "solve_eigbicg",
    "incremental_eigbicg",
    "ritz_residuals",
    "sort_order",
]
