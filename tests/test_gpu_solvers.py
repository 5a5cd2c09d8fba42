"""GPU parity of eigBiCG, the incremental deflation space and deflated BiCGStab against the oracle."""
import numpy as np
import pytest

import synth
from oracle import krylov as K
from oracle import wilson as W

pytestmark = pytest.mark.gpu


def _ops(U, kappa, dims):
    V = synth.volume(dims)
    A = lambda v: W.apply_D(U, v.reshape(V, 4, 3), kappa, dims).ravel()
    Ad = lambda v: W.apply_Ddag(U, v.reshape(V, 4, 3), kappa, dims).ravel()
    return A, Ad


def _rel_match(a, b):
    """max over a of min_b |a - b| / |a| (nearest-neighbour relative distance)."""
    return max(np.min(np.abs(np.asarray(b) - v)) / abs(v) for v in a)


@pytest.fixture(scope="module")
def cfg0(gpu_lib):
    dims, kappa = (4, 4, 4, 4), 0.115
    U = synth.random_su3_links(dims, 0.3, synth.gauge_seed(0))
    return dims, kappa, U


def test_eigbicg_first_solve_parity(gpu_lib, cfg0):
    import torch

    dims, kappa, U = cfg0
    V = synth.volume(dims)
    A, Ad = _ops(U, kappa, dims)
    op = gpu_lib.op_create(U, kappa, dims, defl_capacity=16)
    b_np = synth.z2_source(V, synth.rhs_seed(0, 0))
    b = torch.from_numpy(b_np).to("cuda:0")
    x = torch.zeros_like(b)
    st, ritz = gpu_lib.eigbicg_solve(op, b, x, nev=4, m=16, tol=1e-10)
    orc = K.eigbicg(A, Ad, b_np.ravel(), np.zeros(12 * V, complex), 4, 16, 1e-10)
    print("gpu", st, ritz)
    print("oracle iters", orc.iters, orc.lam)
    assert abs(st["iters"] - orc.iters) <= 1
    assert st["window_restarts"] == len(orc.restarts)
    tr = np.linalg.norm(b_np.ravel() - A(x.cpu().numpy().ravel())) / np.linalg.norm(b_np)
    assert tr <= 1e-10
    assert _rel_match(ritz, orc.lam) < 1e-8 and _rel_match(orc.lam, ritz) < 1e-8
    xo = orc.x
    assert np.linalg.norm(x.cpu().numpy().ravel() - xo) / np.linalg.norm(xo) < 1e-8
    K_, H = gpu_lib.defl_info(op)
    assert K_ == 4


def test_incremental_parity_small_config(gpu_lib, cfg0):
    """4 eigBiCG solves then deflated BiCGStab (4^4, nev=4, m=16): the space matches the oracle's."""
    import torch

    dims, kappa, U = cfg0
    V = synth.volume(dims)
    A, Ad = _ops(U, kappa, dims)
    B = [synth.z2_source(V, synth.rhs_seed(0, i)) for i in range(6)]
    X0 = [np.zeros(12 * V, complex)] * 6
    xs_o, info_o, space_o = K.incremental_eigbicg(A, Ad, [b.ravel() for b in B], X0, 4, 16, 1e-10, n1=4)
    op = gpu_lib.op_create(U, kappa, dims, defl_capacity=16)
    for i, bnp in enumerate(B):
        b = torch.from_numpy(bnp).to("cuda:0")
        x = torch.zeros_like(b)
        if i < 4:
            st, ritz = gpu_lib.eigbicg_solve(op, b, x, nev=4, m=16, tol=1e-10)
            print(i, st["iters"], info_o[i]["iters"], ritz, info_o[i]["lam"])
            assert _rel_match(ritz, info_o[i]["lam"]) < 1e-8
        else:
            st = gpu_lib.deflated_bicg_solve(op, b, x, tol=1e-10)
            print(i, st["iters"], info_o[i]["iters"])
            assert abs(st["iters"] - info_o[i]["iters"]) <= max(2, 0.1 * info_o[i]["iters"])
        tr = np.linalg.norm(bnp.ravel() - A(x.cpu().numpy().ravel())) / np.linalg.norm(bnp)
        assert tr <= 1e-10
        assert st["true_rel_resid"] <= 1e-10
    K_, H = gpu_lib.defl_info(op)
    assert K_ == space_o.K == 16
    lam_g = np.linalg.eigvals(H)
    lam_o = np.linalg.eigvals(space_o.H)
    assert _rel_match(lam_g, lam_o) < 1e-7 and _rel_match(lam_o, lam_g) < 1e-7
    # Rayleigh-Ritz eigenpairs: values and residuals agree with the oracle's
    right = torch.zeros(16 * 12 * V, dtype=torch.complex128, device="cuda:0")
    left = torch.zeros_like(right)
    ev = gpu_lib.get_eigenpairs(op, 16, right, left)
    lam_rr, Ur, Ul = K.rayleigh_ritz(space_o)
    assert _rel_match(ev, lam_rr) < 1e-7
    R = right.cpu().numpy().reshape(16, -1).T
    L = left.cpu().numpy().reshape(16, -1).T
    assert np.allclose(np.linalg.norm(R, axis=0), 1)
    assert np.allclose(np.einsum("ij,ij->j", L.conj(), R), 1)
    rr_g, _ = K.ritz_residuals(A, Ad, ev, R, L)
    rr_o, _ = K.ritz_residuals(A, Ad, lam_rr, Ur, Ul)
    assert np.allclose(np.sort(rr_g), np.sort(rr_o), rtol=1e-5, atol=1e-9)


def test_mixed_precision_solve(gpu_lib, cfg0):
    import torch

    dims, kappa, U = cfg0
    V = synth.volume(dims)
    A, _ = _ops(U, kappa, dims)
    op = gpu_lib.op_create(U, kappa, dims)
    bnp = synth.z2_source(V, synth.rhs_seed(0, 9))
    b = torch.from_numpy(bnp).to("cuda:0")
    x = torch.zeros_like(b)
    st = gpu_lib.deflated_bicg_solve(op, b, x, tol=1e-10, inner="fp32", inner_tol=1e-5)
    tr = np.linalg.norm(bnp.ravel() - A(x.cpu().numpy().ravel())) / np.linalg.norm(bnp)
    print(st, tr)
    assert tr <= 1e-10 and st["outer_steps"] >= 1


@pytest.mark.parametrize("inner,inner_tol", [("fp32", 1e-5), ("bf16", 1e-2)])
def test_mixed_precision_error_vs_fp64_solution(gpu_lib, cfg0, inner, inner_tol):
    """FP32 / BF16 inner solves inside FP64 refinement: every solve reaches the
    FP64 true residual 1e-10, and the solution's error against the dense FP64
    solve is stated and bounded by cond(D) times the residual."""
    import torch

    dims, kappa, U = cfg0
    V = synth.volume(dims)
    A, _ = _ops(U, kappa, dims)
    D = W.dense_D(U, kappa, dims)
    op = gpu_lib.op_create(U, kappa, dims)
    for i in range(2):
        bnp = synth.z2_source(V, synth.rhs_seed(0, 20 + i))
        xs = np.linalg.solve(D, bnp.ravel())
        b = torch.from_numpy(bnp).to("cuda:0")
        x = torch.zeros_like(b)
        st = gpu_lib.deflated_bicg_solve(op, b, x, tol=1e-10, inner=inner, inner_tol=inner_tol)
        xg = x.cpu().numpy().ravel()
        tr = np.linalg.norm(bnp.ravel() - A(xg)) / np.linalg.norm(bnp)
        err = np.linalg.norm(xg - xs) / np.linalg.norm(xs)
        print(f"{inner}: iters {st['iters']} outer {st['outer_steps']} true resid {tr:.2e} error vs FP64 solve {err:.2e}")
        assert tr <= 1e-10 and st["true_rel_resid"] <= 1e-10
        assert st["outer_steps"] >= (3 if inner == "bf16" else 1)
        assert err <= 1e-8


@pytest.fixture(scope="module")
def space8(gpu_lib, cfg0):
    """cfg0 operator with a deflation space from two eigBiCG solves, and 8 sources."""
    import torch

    dims, kappa, U = cfg0
    V = synth.volume(dims)
    op = gpu_lib.op_create(U, kappa, dims, defl_capacity=8)
    for i in range(2):
        b = torch.from_numpy(synth.z2_source(V, synth.rhs_seed(0, i))).to("cuda:0")
        gpu_lib.eigbicg_solve(op, b, torch.zeros_like(b), nev=4, m=16, tol=1e-10)
    B = np.stack([synth.z2_source(V, synth.rhs_seed(0, 30 + i)) for i in range(8)])
    D = W.dense_D(U, kappa, dims)
    Xs = np.linalg.solve(D, B.reshape(8, -1).T).T
    return op, B, Xs


@pytest.mark.parametrize("inner,batch", [("fp64", 4), ("fp32", 8), ("bf16", 2), ("fp32", 0)])
def test_batched_deflated_solves(gpu_lib, cfg0, space8, inner, batch):
    """Multi-RHS deflated solves (k columns per iteration, per-column scalars):
    every column reaches the FP64 true residual 1e-10 and matches the dense
    FP64 solution; the same sources solved one at a time agree."""
    import torch

    dims, kappa, U = cfg0
    A, _ = _ops(U, kappa, dims)
    op, B, Xs = space8
    b = torch.from_numpy(B).to("cuda:0")
    x = torch.zeros_like(b)
    st = gpu_lib.deflated_bicg_solve(op, b, x, tol=1e-10, inner=inner, nrhs=8, batch=batch)
    X = x.cpu().numpy().reshape(8, -1)
    for c in range(8):
        tr = np.linalg.norm(B[c].ravel() - A(X[c])) / np.linalg.norm(B[c])
        err = np.linalg.norm(X[c] - Xs[c]) / np.linalg.norm(Xs[c])
        assert tr <= 1e-10 and err <= 1e-8, (c, tr, err)
    assert st["true_rel_resid"] <= 1e-10
    x1 = torch.zeros_like(b)
    st1 = gpu_lib.deflated_bicg_solve(op, b, x1, tol=1e-10, inner=inner, nrhs=8, batch=1)
    print(f"{inner} batch {batch}: iters {st['iters']} (one at a time {st1['iters']}), outer {st['outer_steps']}")
    assert st["iters"] <= 1.5 * st1["iters"] + 8


@pytest.mark.parametrize("inner", ["fp32", "fp64"])
def test_group_stats_sum_over_batches(gpu_lib, cfg0, inner):
    """One call on 6 sources in batches of 2 (one group of columns) reports the sums of
    iterations and refinement steps and the worst residual of three separate calls on
    2 sources each (no deflation space, so the batches are the same solves)."""
    import torch

    dims, kappa, U = cfg0
    V = synth.volume(dims)
    op = gpu_lib.op_create(U, kappa, dims)
    B = torch.from_numpy(np.stack([synth.z2_source(V, synth.rhs_seed(0, 60 + c)) for c in range(6)])).to("cuda:0")
    X = torch.zeros_like(B)
    st = gpu_lib.deflated_bicg_solve(op, B, X, tol=1e-10, inner=inner, nrhs=6, batch=2)
    parts = []
    for c in range(0, 6, 2):
        x = torch.zeros_like(B[c:c + 2])
        parts.append(gpu_lib.deflated_bicg_solve(op, B[c:c + 2].contiguous(), x, tol=1e-10, inner=inner, nrhs=2,
                                                 batch=2))
        assert torch.equal(x, X[c:c + 2])
    gpu_lib.op_destroy(op)
    print(inner, st, [p["outer_steps"] for p in parts])
    assert st["iters"] == sum(p["iters"] for p in parts)
    assert st["outer_steps"] == sum(p["outer_steps"] for p in parts)
    assert st["true_rel_resid"] == max(p["true_rel_resid"] for p in parts)
    assert st["matvec_d"] == sum(p["matvec_d"] for p in parts)


def test_batched_ragged_and_zero_column(gpu_lib, cfg0, space8):
    """5 right-hand sides with batch 4 (a batch of 4, then one column alone),
    one of them zero, and a non-zero start: the zero column returns x = 0."""
    import torch

    dims, kappa, U = cfg0
    A, _ = _ops(U, kappa, dims)
    op, B, Xs = space8
    Bz = B[:5].copy()
    Bz[2] = 0
    b = torch.from_numpy(Bz).to("cuda:0")
    x = torch.full_like(b, 0.25)
    st = gpu_lib.deflated_bicg_solve(op, b, x, tol=1e-10, inner="fp32", nrhs=5, batch=4)
    X = x.cpu().numpy().reshape(5, -1)
    assert np.abs(X[2]).max() == 0
    for c in (0, 1, 3, 4):
        assert np.linalg.norm(Bz[c].ravel() - A(X[c])) / np.linalg.norm(Bz[c]) <= 1e-10
    assert st["true_rel_resid"] <= 1e-10
    with pytest.raises(gpu_lib.EbicgError) as e:
        gpu_lib.deflated_bicg_solve(op, b, x, tol=1e-10, nrhs=5, batch=3)
    assert e.value.status == -1


def test_full_size_eigbicg_properties(gpu_lib):
    """16^3 x 32 (the benchmark operator), two eigBiCG solves: every true residual
    <= 1e-10; the accumulated space is biorthonormal (U_l^+ U_r = I) and the
    library's H equals U_l^+ A U_r recomputed from the returned vectors and the
    operator; its eigenvalues equal the Rayleigh-Ritz values returned."""
    import torch

    dims, kappa = (16, 16, 16, 32), 0.122
    V = synth.volume(dims)
    U = synth.random_su3_links(dims, 0.3, synth.gauge_seed(1))
    op = gpu_lib.op_create(U, kappa, dims, defl_capacity=20)
    for i in range(2):
        b = torch.from_numpy(synth.z2_source(V, synth.rhs_seed(0, i))).to("cuda:0")
        x = torch.zeros_like(b)
        st, ritz = gpu_lib.eigbicg_solve(op, b, x, nev=10, m=40, tol=1e-10)
        assert st["true_rel_resid"] <= 1e-10 and st["nev_added"] >= 1, st
    K, H = gpu_lib.defl_info(op)
    assert K >= 2
    R = torch.zeros((K, V, 4, 3), dtype=torch.complex128, device="cuda:0")
    L = torch.zeros_like(R)
    ev = gpu_lib.get_eigenpairs(op, K, R, L)
    Rm, Lm = R.reshape(K, -1), L.reshape(K, -1)
    G = (Lm.conj() @ Rm.T).cpu().numpy()
    assert np.abs(G - np.eye(K)).max() < 1e-10
    AR = torch.empty_like(R)
    for k in range(K):
        gpu_lib.op_apply(op, AR[k], R[k].contiguous())
    Hr = (Lm.conj() @ AR.reshape(K, -1).T).cpu().numpy()  # L^+ A R = diag(ev) for Rayleigh-Ritz vectors
    assert np.abs(Hr - np.diag(ev)).max() <= 1e-10 * np.abs(ev).max()
    assert np.allclose(np.sort_complex(np.linalg.eigvals(H)), np.sort_complex(ev), rtol=1e-9, atol=1e-12)


def test_error_paths(gpu_lib, cfg0):
    import torch

    dims, kappa, U = cfg0
    V = synth.volume(dims)
    op = gpu_lib.op_create(U, kappa, dims, defl_capacity=8)
    b = torch.from_numpy(synth.z2_source(V, 1)).to("cuda:0")
    x = torch.zeros_like(b)
    with pytest.raises(gpu_lib.EbicgError) as e:
        gpu_lib.eigbicg_solve(op, b, x, nev=4, m=8, tol=1e-10)
    assert e.value.status == -1
    # gamma5 shadow residual with a Z2 source and x0 = 0: (rhat0, r0) = 0 exactly
    with pytest.raises(gpu_lib.EbicgError) as e:
        gpu_lib.eigbicg_solve(op, b, x, nev=2, m=8, tol=1e-10, rhat=1)
    assert e.value.status == -3
    x.zero_()
    with pytest.raises(gpu_lib.EbicgError) as e:
        gpu_lib.deflated_bicg_solve(op, b, x, tol=1e-10, maxiter=2)
    assert e.value.status == -4
    assert e.value.stats["iters"] >= 1


def test_solves_are_deterministic(gpu_lib, cfg0):
    import torch

    dims, kappa, U = cfg0
    V = synth.volume(dims)
    outs = []
    for _ in range(2):
        op = gpu_lib.op_create(U, kappa, dims, defl_capacity=8)
        b = torch.from_numpy(synth.z2_source(V, 5)).to("cuda:0")
        x = torch.zeros_like(b)
        gpu_lib.eigbicg_solve(op, b, x, nev=4, m=16, tol=1e-10)
        x2 = torch.zeros_like(b)
        gpu_lib.deflated_bicg_solve(op, b, x2, tol=1e-10)
        outs.append((x.clone(), x2.clone()))
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])


def test_deflation_speedup_near_critical(gpu_lib):
    """Alg. Incremental eigBiCG pays off where the low spectrum separates: 4^4,
    eps = 1.0 links, kappa = 0.2379 (0.97 of the critical value of this
    configuration), 8 eigBiCG solves (nev 10, m 40), then deflated BiCGStab.
    The oracle needs about two thirds of the undeflated iterations; the library
    must match its deflated iteration counts within 10% and beat the
    undeflated counts by the same margin."""
    import torch

    dims, kappa = (4, 4, 4, 4), 0.2379
    V = synth.volume(dims)
    N = 12 * V
    U = synth.random_su3_links(dims, 1.0, 123)
    A, Ad = _ops(U, kappa, dims)
    B = [synth.z2_source(V, synth.rhs_seed(0, i)) for i in range(12)]
    _, info_o, _ = K.incremental_eigbicg(A, Ad, [b.ravel() for b in B], [np.zeros(N, complex)] * 12, 10, 40,
                                         1e-8, n1=8)
    defl_o = [d["iters"] for d in info_o[8:]]
    und_o = [K.bicgstab(A, b.ravel(), np.zeros(N, complex), 1e-8, 20000).iters for b in B[8:]]
    op = gpu_lib.op_create(U, kappa, dims, defl_capacity=80)
    defl_g, und_g = [], []
    for i, bnp in enumerate(B):
        b = torch.from_numpy(bnp).to("cuda:0")
        x = torch.zeros_like(b)
        if i < 8:
            gpu_lib.eigbicg_solve(op, b, x, nev=10, m=40, tol=1e-8, maxiter=20000)
        else:
            st = gpu_lib.deflated_bicg_solve(op, b, x, tol=1e-8, maxiter=20000)
            assert st["true_rel_resid"] <= 1e-8
            defl_g.append(st["iters"])
    gpu_lib.defl_reset(op)
    for bnp in B[8:]:
        b = torch.from_numpy(bnp).to("cuda:0")
        x = torch.zeros_like(b)
        und_g.append(gpu_lib.deflated_bicg_solve(op, b, x, tol=1e-8, maxiter=20000)["iters"])
    print("oracle deflated", defl_o, "undeflated", und_o)
    print("gpu    deflated", defl_g, "undeflated", und_g)
    assert np.mean(defl_o) <= 0.8 * np.mean(und_o)  # the premise: deflation helps here
    assert abs(np.mean(defl_g) - np.mean(defl_o)) <= 0.1 * np.mean(defl_o)
    assert np.mean(defl_g) <= 0.8 * np.mean(und_g)
    gpu_lib.op_destroy(op)


def test_windowed_vs_unrestarted_ritz_values(gpu_lib):
    """The analogue of the paper's Table 1: the lowest Ritz values of eigBiCG
    with a window of m = 40 (two restarts) against those of BiCG keeping every
    residual (window larger than the iteration count), on 8^4 with eps = 1.0
    links, kappa = 0.2 (100 iterations to 1e-8).  The un-restarted run is the
    oracle's; the library's un-restarted and windowed runs match the oracle's
    (1e-8), and the windowed values agree with the un-restarted ones to 5e-5
    relative (measured <= 1.5e-5)."""
    import torch

    dims, kappa = (8, 8, 8, 8), 0.2
    V = synth.volume(dims)
    U = synth.random_su3_links(dims, 1.0, 123)
    A, Ad = _ops(U, kappa, dims)
    b_np = synth.z2_source(V, synth.rhs_seed(0, 0))
    orc = K.eigbicg(A, Ad, b_np.ravel(), np.zeros(12 * V, complex), 5, 126, 1e-8)
    orc40 = K.eigbicg(A, Ad, b_np.ravel(), np.zeros(12 * V, complex), 5, 40, 1e-8)
    assert len(orc.restarts) == 0 and len(orc40.restarts) >= 2
    ritz = {}
    for m in (126, 40):
        op = gpu_lib.op_create(U, kappa, dims, defl_capacity=8)
        b = torch.from_numpy(b_np).to("cuda:0")
        st, r = gpu_lib.eigbicg_solve(op, b, torch.zeros_like(b), nev=5, m=m, tol=1e-8)
        ritz[m] = (st, r)
        gpu_lib.op_destroy(op)
    (s_u, r_u), (s_w, r_w) = ritz[126], ritz[40]
    print("oracle", orc.iters, orc.lam)
    print("unrestarted", s_u["iters"], r_u)
    print("windowed", s_w["iters"], s_w["window_restarts"], r_w)
    assert s_u["window_restarts"] == 0 and s_w["window_restarts"] >= 2
    assert abs(s_u["iters"] - orc.iters) <= 1 and abs(s_w["iters"] - orc.iters) <= 1
    assert _rel_match(r_u, orc.lam) < 1e-8 and _rel_match(orc.lam, r_u) < 1e-8
    assert _rel_match(r_w, orc40.lam) < 1e-8 and _rel_match(orc40.lam, r_w) < 1e-8
    # windowed against un-restarted (the Ritz pairs are not converged here:
    # residuals 0.12 - 0.19; the oracle's own two runs differ by <= 1.5e-5)
    assert _rel_match(r_w, orc.lam) < 5e-5 and _rel_match(orc.lam, r_w) < 5e-5


def test_deftol_restarts_match_oracle(gpu_lib, cfg0):
    """Deflated BiCGStab with DefTol > 0 (Alg. Incremental eigBiCG, step 3:
    re-deflate and restart whenever the residual falls below DefTol^k ||b||)
    after 4 eigBiCG solves: the restart count equals the oracle's, the
    iterations agree, and every solve reaches the true residual 1e-10."""
    import torch

    dims, kappa, U = cfg0
    V = synth.volume(dims)
    A, Ad = _ops(U, kappa, dims)
    B = [synth.z2_source(V, synth.rhs_seed(0, 50 + i)) for i in range(6)]
    X0 = [np.zeros(12 * V, complex)] * 6
    for deftol in (3e-3, 1e-3):
        xs_o, info_o, _ = K.incremental_eigbicg(A, Ad, [b.ravel() for b in B], X0, 4, 16, 1e-10, n1=4,
                                                deftol=deftol)
        op = gpu_lib.op_create(U, kappa, dims, defl_capacity=16)
        for i, bnp in enumerate(B):
            b = torch.from_numpy(bnp).to("cuda:0")
            x = torch.zeros_like(b)
            if i < 4:
                gpu_lib.eigbicg_solve(op, b, x, nev=4, m=16, tol=1e-10)
                continue
            st = gpu_lib.deflated_bicg_solve(op, b, x, tol=1e-10, deftol=deftol)
            io = info_o[i]
            print(deftol, i, st["iters"], io["iters"], st["defl_restarts"], io["defl_restarts"])
            assert st["defl_restarts"] == io["defl_restarts"] == 3
            assert abs(st["iters"] - io["iters"]) <= max(3, 0.1 * io["iters"])
            xg = x.cpu().numpy().ravel()
            assert np.linalg.norm(bnp.ravel() - A(xg)) / np.linalg.norm(bnp) <= 1e-10
            assert np.linalg.norm(xg - xs_o[i]) / np.linalg.norm(xs_o[i]) <= 1e-8
        gpu_lib.op_destroy(op)
