"""GPU parity of the even-odd (Schur) form against the oracle.

The solvers of an operator made by eb_op_create_eo run on
Dhat = 1 - kappa^2 H_eo H_oe over the even sites (the paper's test matrices
are even-odd preconditioned, Sec. 3); the oracle's apply_Dhat, eo_prepare and
eo_reconstruct are pinned to the full matrix in test_oracle_wilson.py.
"""
import numpy as np
import pytest

import synth
from oracle import krylov as K
from oracle import wilson as W

pytestmark = pytest.mark.gpu


def _rel_match(a, b):
    return max(np.min(np.abs(np.asarray(b) - v)) / abs(v) for v in a)


def _even(v, dims):
    return v.reshape(-1, 4, 3)[W.parity(dims) == 0]


def _eo_ops(U, kappa, dims):
    Ve = synth.volume(dims) // 2
    A = lambda v: W.apply_Dhat(U, v.reshape(Ve, 4, 3), kappa, dims).ravel()
    Ad = lambda v: W.apply_Dhat(U, v.reshape(Ve, 4, 3), kappa, dims, dagger=True).ravel()
    return A, Ad


@pytest.fixture(scope="module")
def cfg0(gpu_lib):
    dims, kappa = (4, 4, 4, 4), 0.115
    U = synth.random_su3_links(dims, 0.3, synth.gauge_seed(0))
    return dims, kappa, U


@pytest.mark.parametrize("dims,dagger", [((4, 4, 4, 4), False), ((4, 4, 4, 4), True), ((2, 4, 6, 8), False),
                                         ((16, 16, 16, 32), False), ((16, 16, 16, 32), True)])
def test_schur_operator_parity(gpu_lib, dims, dagger):
    """Dhat and Dhat^+ on the GPU against the oracle, every site, 1e-12 relative."""
    import torch

    kappa = 0.122
    V = synth.volume(dims)
    U = synth.random_su3_links(dims, 0.3, 77)
    x = synth.gaussian_spinor(V, 78)
    op = gpu_lib.op_create(U, kappa, dims, eo=True)
    xt = torch.from_numpy(x).to("cuda:0")
    yt = torch.empty_like(xt)
    gpu_lib.op_apply_schur(op, yt, xt, dagger=dagger)
    y = yt.cpu().numpy()
    ref = W.apply_Dhat(U, _even(x, dims), kappa, dims, dagger=dagger)
    par = W.parity(dims)
    assert np.abs(y[par == 1]).max() == 0.0
    err = np.abs(y[par == 0] - ref).max() / np.abs(ref).max()
    print(dims, dagger, err)
    assert err <= 1e-12
    gpu_lib.op_destroy(op)


def test_eo_eigbicg_parity(gpu_lib, cfg0):
    """One eigBiCG solve on the even system (4^4, nev 4, m 16): iterations,
    restarts, Ritz values and the reconstructed full solution against the
    oracle's eigBiCG on Dhat; the full system's residual <= 1e-10."""
    import torch

    dims, kappa, U = cfg0
    V = synth.volume(dims)
    A, Ad = _eo_ops(U, kappa, dims)
    b = synth.z2_source(V, synth.rhs_seed(0, 0))
    bhat = W.eo_prepare(U, b, kappa, dims).ravel()
    tol_e = 1e-10 * np.linalg.norm(b) / np.linalg.norm(bhat)
    orc = K.eigbicg(A, Ad, bhat, np.zeros_like(bhat), 4, 16, tol_e)
    x_o = W.eo_reconstruct(U, orc.x, b, kappa, dims)
    op = gpu_lib.op_create(U, kappa, dims, defl_capacity=16, eo=True)
    bt = torch.from_numpy(b).to("cuda:0")
    xt = torch.zeros_like(bt)
    st, ritz = gpu_lib.eigbicg_solve(op, bt, xt, nev=4, m=16, tol=1e-10)
    print("gpu", st, ritz)
    print("oracle", orc.iters, len(orc.restarts), orc.lam)
    assert abs(st["iters"] - orc.iters) <= 1
    assert st["window_restarts"] == len(orc.restarts)
    assert _rel_match(ritz, orc.lam) < 1e-8 and _rel_match(orc.lam, ritz) < 1e-8
    xg = xt.cpu().numpy()
    D = lambda v: W.apply_D(U, v.reshape(V, 4, 3), kappa, dims).ravel()
    tr = np.linalg.norm(b.ravel() - D(xg)) / np.linalg.norm(b)
    assert tr <= 1e-10 and abs(st["true_rel_resid"] - tr) <= 1e-12
    assert np.linalg.norm(xg - x_o) / np.linalg.norm(x_o) < 1e-8
    K_, _ = gpu_lib.defl_info(op)
    assert K_ == 4
    gpu_lib.op_destroy(op)


def test_eo_incremental_parity(gpu_lib, cfg0):
    """4 eigBiCG solves then 2 deflated BiCGStab on the even system: iteration
    counts and the spectrum of the space against the oracle; eigenpairs come
    back as full-lattice vectors with zero odd part."""
    import torch

    dims, kappa, U = cfg0
    V = synth.volume(dims)
    Ve = V // 2
    A, Ad = _eo_ops(U, kappa, dims)
    B = [synth.z2_source(V, synth.rhs_seed(0, i)) for i in range(6)]
    space = K.DeflationSpace.empty(12 * Ve)
    op = gpu_lib.op_create(U, kappa, dims, defl_capacity=16, eo=True)
    D = lambda v: W.apply_D(U, v.reshape(V, 4, 3), kappa, dims).ravel()
    for i, b in enumerate(B):
        bhat = W.eo_prepare(U, b, kappa, dims).ravel()
        tol_e = 1e-10 * np.linalg.norm(b) / np.linalg.norm(bhat)
        x0 = K.deflate_guess(A, space, bhat, np.zeros_like(bhat))
        bt = torch.from_numpy(b).to("cuda:0")
        xt = torch.zeros_like(bt)
        if i < 4:
            orc = K.eigbicg(A, Ad, bhat, x0, 4, 16, tol_e)
            space = K.absorb(A, Ad, space, orc.U, orc.Q)
            st, ritz = gpu_lib.eigbicg_solve(op, bt, xt, nev=4, m=16, tol=1e-10)
            it_o = orc.iters
        else:
            so = K.bicgstab(A, bhat, x0, tol_e, 10000, space=space)
            st = gpu_lib.deflated_bicg_solve(op, bt, xt, tol=1e-10)
            it_o = so.iters
        print(i, st["iters"], it_o)
        assert abs(st["iters"] - it_o) <= max(2, 0.1 * it_o)
        tr = np.linalg.norm(b.ravel() - D(xt.cpu().numpy())) / np.linalg.norm(b)
        assert tr <= 1e-10 and st["true_rel_resid"] <= 1e-10
    K_, H = gpu_lib.defl_info(op)
    assert K_ == space.K == 16
    lam_g, lam_o = np.linalg.eigvals(H), np.linalg.eigvals(space.H)
    assert _rel_match(lam_g, lam_o) < 1e-7 and _rel_match(lam_o, lam_g) < 1e-7
    right = torch.zeros(4 * 12 * V, dtype=torch.complex128, device="cuda:0")
    ev = gpu_lib.get_eigenpairs(op, 4, right, None)
    R = right.cpu().numpy().reshape(4, V, 4, 3)
    par = W.parity(dims)
    for k in range(len(ev)):
        assert np.abs(R[k][par == 1]).max() == 0.0
        u = R[k][par == 0].ravel()
        assert abs(np.linalg.norm(u) - 1.0) < 1e-12
    gpu_lib.op_destroy(op)


def test_eo_full_size_solves(gpu_lib):
    """16^3 x 32: eigBiCG and a deflated BiCGStab on the even system reach the
    full system's 1e-10, in fewer iterations than on the full operator."""
    import torch

    dims, kappa = (16, 16, 16, 32), 0.122
    V = synth.volume(dims)
    U = synth.random_su3_links(dims, 0.3, synth.gauge_seed(1))
    b0 = torch.from_numpy(synth.z2_source(V, synth.rhs_seed(0, 0))).to("cuda:0")
    b1 = torch.from_numpy(synth.z2_source(V, synth.rhs_seed(0, 1))).to("cuda:0")
    its = {}
    for eo in (False, True):
        op = gpu_lib.op_create(U, kappa, dims, defl_capacity=10, eo=eo)
        x = torch.zeros_like(b0)
        st0, _ = gpu_lib.eigbicg_solve(op, b0, x, nev=10, m=40, tol=1e-10)
        y = torch.empty_like(x)
        gpu_lib.op_apply(op, y, x)
        tr = float((b0 - y).norm() / b0.norm())
        assert tr <= 1e-10 and st0["true_rel_resid"] <= 1e-10
        x1 = torch.zeros_like(b1)
        st1 = gpu_lib.deflated_bicg_solve(op, b1, x1, tol=1e-10)
        gpu_lib.op_apply(op, y, x1)
        assert float((b1 - y).norm() / b1.norm()) <= 1e-10
        its[eo] = (st0["iters"], st1["iters"])
        gpu_lib.op_destroy(op)
    print("full", its[False], "even-odd", its[True])
    assert its[True][0] < its[False][0] and its[True][1] < its[False][1]


def test_eo_error_paths(gpu_lib, cfg0):
    import torch

    dims, kappa, U = cfg0
    with pytest.raises(gpu_lib.EbicgError) as e:
        gpu_lib.op_create(synth.random_su3_links((3, 4, 4, 4), 0.3, 1), kappa, (3, 4, 4, 4), eo=True)
    assert e.value.status == -1
    V = synth.volume(dims)
    op = gpu_lib.op_create(U, kappa, dims, defl_capacity=4, eo=True)
    b = torch.from_numpy(synth.z2_source(V, 1)).to("cuda:0")
    x = torch.zeros_like(b)
    two_in = torch.zeros(2 * 12 * V, dtype=torch.complex128, device="cuda:0")
    two_out = torch.zeros_like(two_in)
    three_in = torch.zeros(3 * 12 * V, dtype=torch.complex128, device="cuda:0")
    with pytest.raises(gpu_lib.EbicgError) as e:
        gpu_lib.op_apply_schur_block(op, torch.zeros_like(three_in), three_in, 3)
    assert e.value.status == -1
    full = gpu_lib.op_create(U, kappa, dims)
    with pytest.raises(gpu_lib.EbicgError) as e:
        gpu_lib.op_apply_schur(full, x, b)
    assert e.value.status == -1
    with pytest.raises(gpu_lib.EbicgError) as e:
        gpu_lib.op_apply_schur_block(full, two_out, two_in, 2)
    assert e.value.status == -1
    gpu_lib.op_destroy(op)
    gpu_lib.op_destroy(full)


def test_eo_gamma5_form(gpu_lib, cfg0):
    """Dhat is gamma5-Hermitian as well (pinned in the oracle tests): the
    gamma5 form on the even system matches the oracle's eigBiCG on Dhat with
    rhat0 = gamma5 r0 (Gaussian source, x0 = 0)."""
    import torch

    dims, kappa, U = cfg0
    V = synth.volume(dims)
    Ve = V // 2
    A, Ad = _eo_ops(U, kappa, dims)
    b = synth.gaussian_spinor(V, 91)
    bhat = W.eo_prepare(U, b, kappa, dims).ravel()
    tol_e = 1e-10 * np.linalg.norm(b) / np.linalg.norm(bhat)
    g5 = W.apply_gamma5(bhat.reshape(Ve, 4, 3)).ravel()
    orc = K.eigbicg(A, Ad, bhat, np.zeros_like(bhat), 4, 16, tol_e, rhat0=g5)
    op = gpu_lib.op_create(U, kappa, dims, defl_capacity=8, eo=True)
    bt = torch.from_numpy(b).to("cuda:0")
    xt = torch.zeros_like(bt)
    st, ritz = gpu_lib.eigbicg_solve(op, bt, xt, nev=4, m=16, tol=1e-10, rhat=2)
    print(st["iters"], orc.iters, ritz, orc.lam)
    assert abs(st["iters"] - orc.iters) <= 1
    assert st["matvec_ddag"] == st["nev_added"]
    assert st["true_rel_resid"] <= 1e-10
    # with the gamma5 shadow the window matrix is real in exact arithmetic: its
    # eigenvalues come in conjugate pairs of equal modulus, and rounding decides
    # which member of a pair makes the nev cut, so either member matches
    rr, _ = K.ritz_residuals(A, Ad, orc.lam, orc.U, orc.Q)
    both = np.concatenate([ritz, np.conj(ritz)])
    for lam, res in zip(orc.lam, rr):
        assert np.min(np.abs(both - lam)) / abs(lam) < (1e-8 if res <= 1e-6 * abs(lam) else 1e-6)
    gpu_lib.op_destroy(op)


@pytest.mark.parametrize("inner,tol_err", [("fp32", 1e-8), ("bf16", 1e-8)])
def test_eo_mixed_precision(gpu_lib, cfg0, inner, tol_err):
    """FP32 and BF16-stored inner BiCGStab on Dhat inside FP64 refinement, with
    and without a deflation space: the full system's residual <= 1e-10 and the
    error against the dense FP64 solution of D x = b within cond(D) times it."""
    import torch

    dims, kappa, U = cfg0
    V = synth.volume(dims)
    Dm = W.dense_D(U, kappa, dims)
    op = gpu_lib.op_create(U, kappa, dims, defl_capacity=8, eo=True)
    for i in range(3):
        b = synth.z2_source(V, synth.rhs_seed(0, 20 + i))
        xd = np.linalg.solve(Dm, b.ravel())
        bt = torch.from_numpy(b).to("cuda:0")
        xt = torch.zeros_like(bt)
        if i == 1:  # grow a space, then solve deflated
            gpu_lib.eigbicg_solve(op, bt, torch.zeros_like(bt), nev=4, m=16, tol=1e-10)
        st = gpu_lib.deflated_bicg_solve(op, bt, xt, tol=1e-10, inner=inner)
        xg = xt.cpu().numpy().ravel()
        tr = np.linalg.norm(b.ravel() - Dm @ xg) / np.linalg.norm(b)
        err = np.linalg.norm(xg - xd) / np.linalg.norm(xd)
        print(inner, i, st["iters"], st["outer_steps"], tr, err)
        assert tr <= 1e-10 and st["true_rel_resid"] <= 1e-10
        assert err <= tol_err
        assert st["outer_steps"] >= 1
    gpu_lib.op_destroy(op)


@pytest.mark.parametrize("k", [2, 4, 16])
def test_schur_block_parity(gpu_lib, k):
    """Multi-RHS Dhat and Dhat^+ (one pass over the links for k sources) against
    the oracle column by column: FP64 at 1e-12; FP32 and BF16 storage against
    the oracle on the rounded inputs (links rounded too, so BF16 within a few
    units of 2^-9).  On an even-odd operator eb_op_apply_block applies the full D."""
    import torch

    dims, kappa = (4, 6, 4, 8), 0.122
    V = synth.volume(dims)
    U = synth.random_su3_links(dims, 0.3, 81)
    op = gpu_lib.op_create(U, kappa, dims, eo=True)
    par = W.parity(dims)
    psi = np.stack([synth.gaussian_spinor(V, 50 + c) for c in range(k)])
    x = torch.from_numpy(psi).to("cuda:0")
    for dag in (False, True):
        ref = np.stack([W.apply_Dhat(U, _even(psi[c], dims), kappa, dims, dagger=dag) for c in range(k)])
        scale = np.abs(ref).max()
        for prec, bound in (("fp64", 1e-12), ("fp32", 2e-6), ("bf16", 8 * 2.0**-9)):
            y = torch.full_like(x, 7.0)
            gpu_lib.op_apply_schur_block(op, y, x, k, dagger=dag, prec=prec)
            got = y.cpu().numpy().reshape(k, V, 4, 3)
            assert np.abs(got[:, par == 1]).max() == 0.0
            if prec == "fp64":
                r = ref
            else:
                dt = np.complex64 if prec == "fp32" else None
                if dt is not None:
                    pr = psi.astype(dt).astype(np.complex128)
                else:
                    pr = torch.view_as_complex(
                        torch.view_as_real(torch.from_numpy(psi)).to(torch.bfloat16).to(torch.float64)).numpy()
                r = np.stack([W.apply_Dhat(U, _even(pr[c], dims), kappa, dims, dagger=dag) for c in range(k)])
            err = np.abs(got[:, par == 0] - r).max() / scale
            print(k, dag, prec, err)
            assert err <= bound, (k, dag, prec, err)
    # the full D on the same operator
    y = torch.empty_like(x)
    gpu_lib.op_apply_block(op, y, x, k)
    ref = np.stack([W.apply_D(U, psi[c], kappa, dims) for c in range(k)])
    assert np.abs(y.cpu().numpy() - ref).max() / np.abs(ref).max() <= 1e-12
    gpu_lib.op_destroy(op)


@pytest.fixture(scope="module")
def eo_space8(gpu_lib, cfg0):
    """Even-odd operator on cfg0 with a space from two eigBiCG solves, 8 sources
    and their dense FP64 solutions of D x = b."""
    import torch

    dims, kappa, U = cfg0
    V = synth.volume(dims)
    op = gpu_lib.op_create(U, kappa, dims, defl_capacity=8, eo=True)
    for i in range(2):
        b = torch.from_numpy(synth.z2_source(V, synth.rhs_seed(0, i))).to("cuda:0")
        gpu_lib.eigbicg_solve(op, b, torch.zeros_like(b), nev=4, m=16, tol=1e-10)
    B = np.stack([synth.z2_source(V, synth.rhs_seed(0, 30 + i)) for i in range(8)])
    Dm = W.dense_D(U, kappa, dims)
    Xs = np.linalg.solve(Dm, B.reshape(8, -1).T).T
    return op, B, Xs, Dm


@pytest.mark.parametrize("inner,batch", [("fp64", 4), ("fp32", 8), ("bf16", 2), ("fp32", 0)])
def test_eo_batched_deflated_solves(gpu_lib, eo_space8, inner, batch):
    """Multi-RHS deflated solves on Dhat (per-column scalars, tolerances scaled
    per column by ||b|| / ||b_hat||): every column's full-system residual
    <= 1e-10 and its error against the dense FP64 solution <= 1e-8; the same
    sources one at a time take about as many iterations."""
    import torch

    op, B, Xs, Dm = eo_space8
    b = torch.from_numpy(B).to("cuda:0")
    x = torch.zeros_like(b)
    st = gpu_lib.deflated_bicg_solve(op, b, x, tol=1e-10, inner=inner, nrhs=8, batch=batch)
    X = x.cpu().numpy().reshape(8, -1)
    for c in range(8):
        tr = np.linalg.norm(B[c].ravel() - Dm @ X[c]) / np.linalg.norm(B[c])
        err = np.linalg.norm(X[c] - Xs[c]) / np.linalg.norm(Xs[c])
        assert tr <= 1e-10 and err <= 1e-8, (c, tr, err)
    assert st["true_rel_resid"] <= 1e-10
    x1 = torch.zeros_like(b)
    st1 = gpu_lib.deflated_bicg_solve(op, b, x1, tol=1e-10, inner=inner, nrhs=8, batch=1)
    print(f"{inner} batch {batch}: iters {st['iters']} (one at a time {st1['iters']}), outer {st['outer_steps']}")
    assert st["iters"] <= 1.5 * st1["iters"] + 8


def test_eo_batched_ragged_and_zero_column(gpu_lib, eo_space8):
    """5 right-hand sides with batch 4 on Dhat (a batch of 4, then one column
    alone), one of them zero, and a non-zero start: the zero column returns
    x = 0, the others reach the full-system residual 1e-10."""
    import torch

    op, B, Xs, Dm = eo_space8
    Bz = B[:5].copy()
    Bz[2] = 0
    b = torch.from_numpy(Bz).to("cuda:0")
    x = torch.full_like(b, 0.25)
    st = gpu_lib.deflated_bicg_solve(op, b, x, tol=1e-10, inner="fp32", nrhs=5, batch=4)
    X = x.cpu().numpy().reshape(5, -1)
    assert np.abs(X[2]).max() == 0
    for c in (0, 1, 3, 4):
        assert np.linalg.norm(Bz[c].ravel() - Dm @ X[c]) / np.linalg.norm(Bz[c]) <= 1e-10
    assert st["true_rel_resid"] <= 1e-10


def test_eo_full_size_batched(gpu_lib):
    """16^3 x 32, the benchmark's lattice, in the launch configuration the bench
    uses: the multi-RHS Dhat (k = 4, FP64) against the oracle at every even
    site, then four deflated solves batched (FP32 inner, batch 4; BF16 inner,
    batch chosen by the library), each column at the full system's 1e-10."""
    import torch

    dims, kappa = (16, 16, 16, 32), 0.122
    V = synth.volume(dims)
    U = synth.random_su3_links(dims, 0.3, synth.gauge_seed(1))
    op = gpu_lib.op_create(U, kappa, dims, defl_capacity=10, eo=True)
    psi = np.stack([synth.gaussian_spinor(V, 90 + c) for c in range(4)])
    x = torch.from_numpy(psi).to("cuda:0")
    y = torch.empty_like(x)
    gpu_lib.op_apply_schur_block(op, y, x, 4)
    got = y.cpu().numpy().reshape(4, V, 4, 3)[:, W.parity(dims) == 0]
    for c in range(4):
        ref = W.apply_Dhat(U, _even(psi[c], dims), kappa, dims)
        assert np.abs(got[c] - ref).max() / np.abs(ref).max() <= 1e-12
    b0 = torch.from_numpy(synth.z2_source(V, synth.rhs_seed(0, 0))).to("cuda:0")
    gpu_lib.eigbicg_solve(op, b0, torch.zeros_like(b0), nev=10, m=40, tol=1e-10)
    B = torch.from_numpy(np.stack([synth.z2_source(V, synth.rhs_seed(0, 40 + c)) for c in range(4)])).to("cuda:0")
    for inner, batch in (("fp32", 4), ("bf16", 0)):
        X = torch.zeros_like(B)
        st = gpu_lib.deflated_bicg_solve(op, B, X, tol=1e-10, inner=inner, nrhs=4, batch=batch)
        R = torch.empty_like(X)
        gpu_lib.op_apply_block(op, R, X, 4)
        for c in range(4):
            tr = float((B[c] - R[c]).norm() / B[c].norm())
            assert tr <= 1e-10, (inner, c, tr)
        print(inner, batch, st["iters"], st["outer_steps"], st["true_rel_resid"])
        assert st["true_rel_resid"] <= 1e-10
    gpu_lib.op_destroy(op)
