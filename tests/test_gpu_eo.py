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
    with pytest.raises(gpu_lib.EbicgError) as e:
        gpu_lib.op_apply_block(op, two_out, two_in, 2)
    assert e.value.status == -1
    full = gpu_lib.op_create(U, kappa, dims)
    with pytest.raises(gpu_lib.EbicgError) as e:
        gpu_lib.op_apply_schur(full, x, b)
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
