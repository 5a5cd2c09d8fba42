#!/usr/bin/env python3
"""Benchmark: incremental eigBiCG on one MI355X.

Workload (one "step" = the whole hot path over one batch of right-hand sides):
16^3 x 32 Wilson-Dirac operator, kappa = 0.122, SU(3) links exp(i 0.3 H)
(seeded), 24 Z2-noise sources resident in HBM.  The first 8 sources run
eigBiCG (nev = 10, m = 40), each growing the deflation space (up to 80
left/right pairs); the remaining 16 run deflated BiCGStab.  Every solve
reaches ||b - A x|| / ||b|| <= 1e-10 (checked in FP64 by the library).

Prints ONE JSON line on stdout: solves/s of the FP64 step, the dominant
kernel's roofline (achieved algorithmic GB/s from HIP events inside the
library, over the timed region), per-solve p50/p99 latency, and the CPU
oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E

# Algorithmic HBM bytes per lattice site and launch, in units of one FP64
# spinor (192 B/site): vectors each kernel must read or write once, links
# (4 x 9 complex = 576 B/site = 3 units) read once per stencil launch.
UNIT_BYTES_FP64 = 192
# the dominant step kernel of the workload (largest share of the step's kernel time)
ROOFLINE_CLASS = "bicg_matvec"
KERNEL_UNITS = {
    "bicg_matvec": 7,    # in p, phat; out Ap, A^+ phat; links (shared by D and D^+)
    "bicg_update_r": 6,  # in r, rhat, Ap, A^+ phat; out r, rhat
    "bicg_update_p": 8,  # in x, p, phat, r, rhat; out x, p, phat
    "stab_v": 6,         # in p, rhat; out v; links
    "stab_s": 3,         # in r, v; out s
    "stab_t": 5,         # in s; out t; links
    "stab_xr": 7,        # in x, p, s, t, rhat; out x, r
    "stab_p": 4,         # in r, p, v; out p
    "residual": 6,       # in x, b; out r; links
}

WORKLOADS = {
    # the incremental-eigBiCG workload: 16^3 x 32, 8 eigBiCG + 16 deflated solves
    "inc16x32": dict(dims=(16, 16, 16, 32), kappa=0.122, nrhs=24, n1=8, nev=10, m=40, tol=1e-10, cfg=1),
    # the small parity workload (4^4), for quick runs
    "inc4": dict(dims=(4, 4, 4, 4), kappa=0.115, nrhs=4, n1=4, nev=4, m=16, tol=1e-10, cfg=0),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def percentile(xs, q):
    import numpy as np

    return float(np.percentile(np.asarray(xs), q)) if xs else None


def run_step(eb, op, B, X, W, lat, iters, g5=False):
    """One pass of the workload.  g5: eigBiCG solves after the first in the
    gamma5-Hermitian form (the first, from x0 = 0 with a Z2 source, would have
    (gamma5 r0, r0) = 0)."""
    eb.defl_reset(op)
    for i, (b, x) in enumerate(zip(B, X)):
        x.zero_()
        t0 = time.perf_counter()
        if i < W["n1"]:
            st, _ = eb.eigbicg_solve(op, b, x, nev=W["nev"], m=W["m"], tol=W["tol"], maxiter=20000,
                                     rhat=2 if (g5 and i > 0) else 0)
        else:
            st = eb.deflated_bicg_solve(op, b, x, tol=W["tol"], maxiter=20000)
        lat.append(time.perf_counter() - t0)
        iters.append(st["iters"])
        if st["true_rel_resid"] > W["tol"]:
            raise RuntimeError(f"solve {i} missed the tolerance: {st}")


def run_mixed_step(eb, op, B, X, W, inner="bf16", inner_tol=1e-2):
    """The same pass with the deflated phase in lower precision: the n1
    eigBiCG solves in FP64 as in run_step, then the remaining right-hand sides
    in one call, batched by the library's autotuner, with `inner`-stored
    BiCGStab inside FP64 refinement to the same tolerance.  Returns seconds."""
    import torch

    eb.defl_reset(op)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(W["n1"]):
        X[i].zero_()
        st, _ = eb.eigbicg_solve(op, B[i], X[i], nev=W["nev"], m=W["m"], tol=W["tol"], maxiter=20000)
        if st["true_rel_resid"] > W["tol"]:
            raise RuntimeError(f"solve {i} missed the tolerance: {st}")
    Bd = torch.stack(B[W["n1"]:])
    Xd = torch.zeros_like(Bd)
    st = eb.deflated_bicg_solve(op, Bd, Xd, tol=W["tol"], maxiter=20000, nrhs=len(B) - W["n1"], batch=0,
                                inner=inner, inner_tol=inner_tol)
    torch.cuda.synchronize()
    if st["true_rel_resid"] > W["tol"]:
        raise RuntimeError(f"mixed deflated phase missed the tolerance: {st}")
    return time.perf_counter() - t0


def cpu_baseline(W, U, b_np, eig_iters, stab_iters, n_eig_it=5, n_stab_it=3):
    """The FP64 oracle on the host: a bounded sample, extrapolated to one step."""
    import numpy as np

    from oracle import krylov as K
    from oracle import wilson as Wl

    try:
        from threadpoolctl import threadpool_limits
    except Exception:  # pragma: no cover
        threadpool_limits = None
    dims, kappa = W["dims"], W["kappa"]
    V = int(np.prod(dims))
    A = lambda v: Wl.apply_D(U, v.reshape(V, 4, 3), kappa, dims).ravel()
    Ad = lambda v: Wl.apply_Ddag(U, v.reshape(V, 4, 3), kappa, dims).ravel()
    b = b_np.ravel()
    ctx = threadpool_limits(1) if threadpool_limits else None
    try:
        if ctx:
            ctx.__enter__()
        t0 = time.perf_counter()
        K.eigbicg(A, Ad, b, np.zeros_like(b), W["nev"], W["m"], W["tol"], maxiter=n_eig_it)
        t1 = time.perf_counter()
        K.bicgstab(A, b, np.zeros_like(b), W["tol"], maxiter=n_stab_it)
        t2 = time.perf_counter()
        A(b)
        t3 = time.perf_counter()
    finally:
        if ctx:
            ctx.__exit__(None, None, None)
    t_eig = (t1 - t0) / n_eig_it
    t_stab = (t2 - t1) / n_stab_it
    est = t_eig * eig_iters + t_stab * stab_iters
    return {
        "value": W["nrhs"] / est,
        "unit": "solves/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"oracle eigBiCG {n_eig_it} iterations and BiCGStab {n_stab_it} iterations on the same lattice "
                   f"and source ({t1 - t0:.1f} s + {t2 - t1:.1f} s, BLAS limited to 1 thread), extrapolated with the "
                   f"step's iteration counts ({eig_iters} eigBiCG + {stab_iters} BiCGStab)"),
        "seconds_per_eigbicg_iter": t_eig,
        "seconds_per_bicgstab_iter": t_stab,
        # one application of the oracle's D, in the GPU's byte model (960 B per site)
        "dslash_seconds": round(t3 - t2, 4),
        "dslash_GBps": round(960 * V / (t3 - t2) / 1e9, 3),
    }


def tune_untimed(eb, op, precs):
    """Run the library's batch autotuner (once per operator and precision, a
    setup step) outside the timed solves; returns its wall time per precision."""
    import torch

    out = {}
    for p in precs:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        eb.op_batch_tune(op, p)
        torch.cuda.synchronize()
        out[p] = round(time.perf_counter() - t0, 4)
    return out


def stencil_bytes(V, k, prec):
    """Algorithmic bytes of one k-column stencil launch: k inputs and k outputs
    of 12 complex per site, and the 4 x 9 complex links per site read once."""
    cb = {"fp64": 16, "fp32": 8, "bf16": 4}[prec]
    return V * cb * (24 * k + 36)


def multi_rhs_stencil(eb, op, V, precs=("fp64", "fp32", "bf16"), ks=(1, 2, 4, 8, 16), reps=5):
    """GB/s of the multi-RHS stencil (HIP events inside the library) per precision and k."""
    import torch

    out = {}
    for prec in precs:
        out[prec] = {}
        for k in ks:
            if prec == "bf16":
                x = torch.zeros(k * 24 * V, dtype=torch.bfloat16, device="cuda:0")
            else:
                x = torch.zeros(k * 12 * V, dtype={"fp64": torch.complex128, "fp32": torch.complex64}[prec],
                                device="cuda:0")
            y = torch.empty_like(x)
            eb.op_apply_block(op, y, x, k, prec=prec)
            torch.cuda.synchronize()
            eb.timing_enable(op, True)
            for _ in range(reps):
                eb.op_apply_block(op, y, x, k, prec=prec)
            torch.cuda.synchronize()
            n, ms = eb.timing_read(op)["bdslash"]
            eb.timing_enable(op, False)
            us = 1e3 * ms / n
            out[prec][k] = {"us": round(us, 2), "GBps": round(stencil_bytes(V, k, prec) / (us * 1e-6) / 1e9, 1)}
            del x, y
    return out


def large_lattice(eb, dims, kappa, nrhs, tol):
    """A lattice whose fields exceed the 256 MB Infinity Cache: multi-RHS stencil
    bandwidth, and mixed-precision batched solves (FP32 and BF16 storage in FP64
    refinement, batch size chosen by the library's timing) against plain FP64
    BiCGStab one right-hand side at a time.  No deflation space."""
    import numpy as np
    import torch

    import synth

    V = synth.volume(dims)
    t0 = time.perf_counter()
    U = synth.random_su3_links(dims, 0.3, synth.gauge_seed(2))
    log(f"[bench] {dims}: links generated in {time.perf_counter() - t0:.1f} s")
    op = eb.op_create(U, kappa, dims, bc_t=-1, defl_capacity=0)
    del U
    res = {"lattice": list(dims), "kappa": kappa, "stencil": multi_rhs_stencil(eb, op, V)}
    B = torch.stack([torch.from_numpy(synth.z2_source(V, synth.rhs_seed(2, i))) for i in range(nrhs)]).to("cuda:0")
    res["autotune_seconds"] = tune_untimed(eb, op, ("fp32", "bf16"))
    solves = {}
    for name, kw in [("fp64_one_at_a_time", dict(inner="fp64", batch=1)),
                     ("mixed_fp32_batched", dict(inner="fp32", inner_tol=1e-6, batch=0)),
                     ("mixed_bf16_batched", dict(inner="bf16", inner_tol=1e-2, batch=0))]:
        X = torch.zeros_like(B)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st = eb.deflated_bicg_solve(op, B, X, tol=tol, maxiter=20000, nrhs=nrhs, **kw)
        dt = time.perf_counter() - t1
        assert st["true_rel_resid"] <= tol, (name, st)
        solves[name] = {"solves_per_s": round(nrhs / dt, 3), "iters_per_rhs": round(st["iters"] / nrhs, 1),
                        "outer_steps": st["outer_steps"], "max_true_rel_resid": st["true_rel_resid"]}
        log(f"[bench] {dims} {name}: {solves[name]}")
    res["solves"] = solves
    res["nrhs"] = nrhs
    eb.op_destroy(op)
    del B, X
    torch.cuda.empty_cache()
    return res


def batching(eb, dims=(32, 32, 32, 64), kappa=0.123, nrhs=16, n1=4, nev=25, m=60, tol=1e-10):
    """Batching on 32^3 x 64: the multi-RHS stencil (FP32 and BF16 storage,
    k = 1, 4, 8, 16), the autotuner's choice of k and tile form, a deflation
    space of n1 * nev = 100 pairs grown by eigBiCG, and mixed-precision
    (complex64 inner, complex128 outer) batched deflated solves at k = 4, 8, 16
    and the tuned k.  The deflation of a batch is a tall-skinny complex GEMM
    pair on the matrix cores: C = U_l^+ R (K x N times N x k) and X += U_r C;
    its algorithmic bytes are 2 K N + 3 k N complex128 entries and its flops
    2 x 8 K N k."""
    import torch

    import synth

    V = synth.volume(dims)
    N = 12 * V
    t0 = time.perf_counter()
    U = synth.random_su3_links(dims, 0.3, synth.gauge_seed(3))
    log(f"[bench] {dims}: links generated in {time.perf_counter() - t0:.1f} s")
    op = eb.op_create(U, kappa, dims, bc_t=-1, defl_capacity=n1 * nev)
    del U
    res = {"lattice": list(dims), "kappa": kappa, "nrhs": nrhs}
    res["stencil"] = multi_rhs_stencil(eb, op, V, precs=("fp32", "bf16"), ks=(1, 4, 8, 16))
    res["autotune"] = {p: eb.op_batch_tune(op, p) for p in ("fp32", "bf16")}
    log(f"[bench] {dims} autotune: {res['autotune']}")
    grow = []
    for i in range(n1):
        b = torch.from_numpy(synth.z2_source(V, synth.rhs_seed(3, 100 + i))).to("cuda:0")
        x = torch.zeros_like(b)
        st, _ = eb.eigbicg_solve(op, b, x, nev, m, tol)
        assert st["true_rel_resid"] <= tol, st
        grow.append({"iters": st["iters"], "restarts": st["window_restarts"], "seconds": round(st["seconds"], 3)})
        log(f"[bench] {dims} eigBiCG {i}: {grow[-1]}")
        del b, x
    K = eb.defl_info(op)[0]
    res["eigbicg"] = {"nev": nev, "m": m, "solves": grow, "K": K}
    res["device_bytes_after_growth"] = eb.op_device_bytes(op)
    eb.op_trim(op)  # the windows of the eigBiCG phase: about 100 GB at this size
    res["device_bytes_trimmed"] = eb.op_device_bytes(op)
    B = torch.stack([torch.from_numpy(synth.z2_source(V, synth.rhs_seed(3, i))) for i in range(nrhs)]).to("cuda:0")
    solves = {}
    eb.timing_classes(op, ["proj"])
    for k in (4, 8, 16, 0):
        X = torch.zeros_like(B)
        eb.timing_enable(op, True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st = eb.deflated_bicg_solve(op, B, X, tol=tol, maxiter=20000, nrhs=nrhs, inner="fp32", inner_tol=1e-6,
                                    batch=k)
        dt = time.perf_counter() - t1
        n_proj, ms_proj = eb.timing_read(op)["proj"]
        eb.timing_enable(op, False)
        assert st["true_rel_resid"] <= tol, (k, st)
        kk = k if k else res["autotune"]["fp32"]["k"]
        nb = -(-nrhs // kk)
        gemm_bytes = nb * (2 * K * N + 3 * kk * N) * 16
        gemm_flops = nb * 2 * 8 * K * N * kk
        rec = {"solves_per_s": round(nrhs / dt, 3), "iters_per_rhs": round(st["iters"] / nrhs, 1),
               "outer_steps": st["outer_steps"], "max_true_rel_resid": st["true_rel_resid"],
               "deflation_gemm": {"launches": n_proj, "ms": round(ms_proj, 3),
                                  "GBps": round(gemm_bytes / (ms_proj * 1e-3) / 1e9, 1) if ms_proj else None,
                                  "TFLOPs_fp64": round(gemm_flops / (ms_proj * 1e-3) / 1e12, 2) if ms_proj else None}}
        solves[f"mixed_fp32_k{k}" if k else f"mixed_fp32_tuned_k{kk}"] = rec
        log(f"[bench] {dims} k={k}: {rec}")
        del X
    eb.timing_classes(op, None)
    # FP64 deflated BiCGStab one right-hand side at a time, on 4 of the sources
    X = torch.zeros_like(B[:4])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = eb.deflated_bicg_solve(op, B[:4].contiguous(), X, tol=tol, maxiter=20000, nrhs=4, batch=1)
    dt = time.perf_counter() - t1
    solves["fp64_one_at_a_time"] = {"solves_per_s": round(4 / dt, 3), "iters_per_rhs": round(st["iters"] / 4, 1),
                                    "max_true_rel_resid": st["true_rel_resid"]}
    res["solves"] = solves
    eb.op_destroy(op)
    del B, X
    torch.cuda.empty_cache()
    return res


# ---------------------------------------------------------------------------
# HBM traffic of the roofline kernel from rocprofv3 counters.
#   1. rocprofv3 --pmc FETCH_SIZE -d D1 -o run -- python3 bench.py --pmc-pass
#   2. rocprofv3 --pmc WRITE_SIZE -d D2 -o run -- python3 bench.py --pmc-pass
#   (--pmc-pass runs one eigBiCG solve of the workload, then a plain copy of
#   COPY_BYTES so the counters can be calibrated against a known size)
#   3. python3 bench.py --summarize-pmc D1/run_counter_collection.csv D2/run_counter_collection.csv
# writes profiles/pmc_<kernel>_<workload>.json.  The summary records a hash of
# the kernel sources; bench.py reports traffic only while the hash matches.
# ---------------------------------------------------------------------------
COPY_BYTES = 1 << 28
KERNEL_SOURCES = ["kernels.hip", "stencil.h", "kernel_util.h", "device_common.h", "kernels.h"]


def kernel_source_hash():
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_0911_2285_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def deflation_sweep(eb):
    """Deflation speed-up on small near-critical lattices with rough links (the
    analogue of the paper's Fig. 1): BiCGStab iterations per right-hand side
    after n1 = 8 eigBiCG solves, against the same sources undeflated.  The
    bench workload's eps = 0.3 links give a dense near-free low spectrum where
    80 vectors do not change the iteration count; eps = 1.0 near the critical
    kappa separates the low modes."""
    import numpy as np
    import torch

    import synth

    out = []
    for dims, kappa in [((4, 4, 4, 4), 0.2379), ((8, 8, 8, 8), 0.237)]:
        V = synth.volume(dims)
        U = synth.random_su3_links(dims, 1.0, 123)
        B = [torch.from_numpy(synth.z2_source(V, synth.rhs_seed(0, i))).to("cuda:0") for i in range(12)]
        und = None
        for nev, m in [(5, 40), (10, 40), (10, 100)]:
            op = eb.op_create(U, kappa, dims, bc_t=-1, defl_capacity=8 * nev)
            for i in range(8):
                eb.eigbicg_solve(op, B[i], torch.zeros_like(B[i]), nev=nev, m=m, tol=1e-8, maxiter=20000)
            defl = [eb.deflated_bicg_solve(op, B[i], torch.zeros_like(B[i]), tol=1e-8, maxiter=20000)["iters"]
                    for i in range(8, 12)]
            dt = None
            if (nev, m) == (10, 40):  # the same space with the DefTol restart (DefTol 1e-2)
                sts = [eb.deflated_bicg_solve(op, B[i], torch.zeros_like(B[i]), tol=1e-8, deftol=1e-2,
                                              maxiter=20000) for i in range(8, 12)]
                dt = {"deftol": 1e-2, "deflated_iters": [t["iters"] for t in sts],
                      "defl_restarts": [t["defl_restarts"] for t in sts]}
            if und is None:
                eb.defl_reset(op)
                und = [eb.deflated_bicg_solve(op, B[i], torch.zeros_like(B[i]), tol=1e-8, maxiter=20000)["iters"]
                       for i in range(8, 12)]
            eb.op_destroy(op)
            rec = {"lattice": list(dims), "eps": 1.0, "kappa": kappa, "nev": nev, "m": m, "n1": 8,
                   "deflated_iters": defl, "undeflated_iters": und,
                   "speedup": round(float(np.mean(und) / np.mean(defl)), 3)}
            if dt is not None:
                rec["with_deftol"] = dt
            out.append(rec)
    return out


def table1_analogue(eb):
    """Lowest Ritz values of eigBiCG with windows m = 20 and 40 against BiCG
    keeping every residual (m = 126 > the iteration count), as in the paper's
    Table 1, on 8^4 and 12^4 with eps = 1.0 links, kappa = 0.2, tol 1e-8."""
    import numpy as np
    import torch

    import synth

    out = []
    for dims in ((8, 8, 8, 8), (12, 12, 12, 12)):
        kappa = 0.2
        V = synth.volume(dims)
        U = synth.random_su3_links(dims, 1.0, 123)
        b = torch.from_numpy(synth.z2_source(V, synth.rhs_seed(0, 0))).to("cuda:0")
        runs = {}
        for m in (126, 40, 20):
            op = eb.op_create(U, kappa, dims, bc_t=-1, defl_capacity=8)
            st, r = eb.eigbicg_solve(op, b, torch.zeros_like(b), nev=5, m=m, tol=1e-8, maxiter=20000)
            eb.op_destroy(op)
            runs[m] = (st, np.asarray(r))
        ref = runs[126][1]
        rec = {"lattice": list(dims), "eps": 1.0, "kappa": kappa, "nev": 5,
               "unrestarted": {"iters": runs[126][0]["iters"], "restarts": runs[126][0]["window_restarts"],
                               "ritz": [[float(z.real), float(z.imag)] for z in ref]}}
        for m in (40, 20):
            st, r = runs[m]
            rec[f"m{m}"] = {"iters": st["iters"], "restarts": st["window_restarts"],
                            "ritz": [[float(z.real), float(z.imag)] for z in r],
                            "rel_diff_to_unrestarted": [float(np.min(np.abs(ref - z)) / abs(z)) for z in r]}
        out.append(rec)
    return out


SERVING_OPS = [  # (dims, kappa, share of the arrivals)
    ((8, 8, 8, 8), 0.11, 0.50),
    ((16, 16, 16, 32), 0.122, 0.35),
    ((24, 24, 24, 48), 0.123, 0.15),
]


def serving(eb, n_req=48, rel_rates=(0.25, 0.5, 1.0), slots=8, grow=4, nev=8, m=24, tol=1e-10, inner="bf16"):
    """Serving: a Poisson stream of Z2-source solve requests over three resident
    even-odd operators (8^4, 16^3 x 32, 24^3 x 48; arrival mix 50/35/15%).
    Each operator's first `grow` requests run eigBiCG and grow its deflation
    space; the rest are batched by its session (BF16-stored inner solves,
    FP64 refinement, `slots` columns; one burst with FP32 inner for
    comparison) with continuous admission.  A burst (every request at
    t = 0) gives the saturation throughput; Poisson streams at fractions of it
    give p50 / p99 latency (arrival to result) beside solves/s."""
    import numpy as np
    import torch

    import synth
    from paper_0911_2285_amd import serve

    specs = []
    for o, (dims, kappa, _) in enumerate(SERVING_OPS):
        U = synth.random_su3_links(dims, 0.3, synth.gauge_seed(4, o + 1))
        op = eb.op_create(U, kappa, dims, bc_t=-1, defl_capacity=grow * nev, eo=True)
        specs.append(serve.OperatorSpec(op, grow=grow, nev=nev, m=m, slots=slots))
    mix = [w for _, _, w in SERVING_OPS]
    _, which = serve.poisson_arrivals(n_req, 1.0, mix, seed=7)
    sources = []
    for i, o in enumerate(which):
        V = synth.volume(SERVING_OPS[o][0])
        sources.append(torch.from_numpy(synth.z2_source(V, synth.rhs_seed(int(o) + 1, i)).ravel()).pin_memory())
    budget = 64 << 30

    def run(arrivals, grow_now, graph=True, inner="fp32", hbm_budget=None):
        for sp in specs:
            sp.grow = grow if grow_now else 0
        srv = serve.Server(specs, inner=inner, tol=tol, hbm_budget=hbm_budget or budget, graph=graph)
        reqs = [serve.Request(i, int(o), float(t), sources[i]) for i, (t, o) in enumerate(zip(arrivals, which))]
        torch.cuda.synchronize()
        res = srv.run(reqs)
        torch.cuda.synchronize()
        assert len(res) == n_req and all(r.status == "EB_OK" for r in res), [r.status for r in res]
        assert all(r.stats["true_rel_resid"] <= tol for r in res)
        summ = serve.latency_summary(res, float(np.min(arrivals)))
        summ["per_operator_p50_ms"] = [round(1e3 * float(np.median([r.latency for r in res if r.op == o])), 3)
                                       if any(r.op == o for r in res) else None for o in range(len(specs))]
        summ["max_resident_bytes"] = srv.max_resident
        summ["deferred_admissions"] = srv.deferred
        srv.close()
        return res, summ

    out = {"operators": [{"dims": list(d), "kappa": k, "share": w, "even_odd": True} for d, k, w in SERVING_OPS],
           "requests": n_req, "slots": slots, "inner": inner, "tol": tol, "hbm_budget_bytes": budget,
           "growth": {"eigbicg_requests_per_operator": grow, "nev": nev, "m": m}}
    # 1. a burst with online growth of the spaces: the eigBiCG phase and then the sessions
    res, summ = run(np.zeros(n_req), True, inner=inner)
    out["burst_with_growth"] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in summ.items()}
    out["deflation_space_K"] = [eb.defl_info(sp.op)[0] for sp in specs]
    log(f"[bench] serving burst with growth: {out['burst_with_growth']}")
    # 2. a burst on the grown spaces: the saturation throughput of the sessions
    res, summ = run(np.zeros(n_req), False, inner=inner)
    sat = summ["solves_per_s"]
    out["burst"] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in summ.items()}
    log(f"[bench] serving burst: {out['burst']}")
    # the same burst with every chunk launched kernel by kernel (no hipGraph replay),
    # and with FP32-stored inner solves
    res, summ = run(np.zeros(n_req), False, graph=False, inner=inner)
    out["burst_direct_launches"] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in summ.items()}
    log(f"[bench] serving burst, direct launches: {out['burst_direct_launches']}")
    res, summ = run(np.zeros(n_req), False, inner="fp32")
    out["burst_fp32_inner"] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in summ.items()}
    log(f"[bench] serving burst, FP32 inner: {out['burst_fp32_inner']}")
    # 3. Poisson streams at fractions of the saturation rate
    out["poisson"] = []
    for f in rel_rates:
        t, _ = serve.poisson_arrivals(n_req, f * sat, mix, seed=7)
        res, summ = run(t, False, inner=inner)
        rec = {"rate_fraction": f, "arrival_rate_per_s": round(f * sat, 3)}
        rec.update({k: (round(v, 3) if isinstance(v, float) else v) for k, v in summ.items()})
        out["poisson"].append(rec)
        log(f"[bench] serving poisson {f}: {rec}")
    # 4. the saturation-rate stream under a memory budget that binds: what the
    # operators and sessions hold plus room for the b and x of four requests
    # of the largest operator; admissions wait for memory instead of failing
    probe = serve.Server(specs, inner=inner, tol=tol)
    resident = probe.resident_bytes()
    probe.close()
    tight = resident + 4 * 2 * 16 * max(sp.op.N for sp in specs)
    t, _ = serve.poisson_arrivals(n_req, sat, mix, seed=7)
    res, summ = run(t, False, inner=inner, hbm_budget=tight)
    rec = {"rate_fraction": 1.0, "hbm_budget_bytes": tight}
    rec.update({k: (round(v, 3) if isinstance(v, float) else v) for k, v in summ.items()})
    out["poisson_tight_budget"] = rec
    log(f"[bench] serving poisson under a tight budget: {rec}")
    for sp in specs:
        eb.op_destroy(sp.op)
    return out


def stencil_pass(dims=(32, 32, 32, 64), ks=(1, 16), reps=5, form=0):
    """For counter runs of the multi-RHS stencil: FP32 storage, k = 1 (LDS-staged
    form) and 16 columns (tile form `form`), `reps` launches each after one
    warm-up (unit links: the stencil's traffic does not depend on the link
    values), then the calibration copy."""
    import torch

    import synth
    from paper_0911_2285_amd import ebicg as eb

    V = synth.volume(dims)
    op = eb.op_create(synth.unit_links(dims), 0.12, dims, bc_t=-1)
    for k in ks:
        eb.op_batch_set_tile(op, "fp32", k, form if k > 1 else 1)
        x = torch.ones(k * 12 * V, dtype=torch.complex64, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(reps + 1):
            eb.op_apply_block(op, y, x, k, prec="fp32")
        torch.cuda.synchronize()
        del x, y
    src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    log(f"[bench] stencil pass done: V = {V}, k = {ks}, FP32, tile form 1 (k = 1) / {form} (k > 1)")


def proj_pass(dims=(16, 16, 16, 32), kappa=0.122, n1=8, nev=10, m=40, nrhs=16):
    """For counter runs of the deflation projections on the matrix cores: the
    headline lattice's space of n1 * nev pairs grown by eigBiCG (the absorb
    steps' Gram blocks), then nrhs right-hand sides deflated as one batch
    (C = U_l^+ R with K = 80, k = 16) and solved with FP32 inner BiCGStab."""
    import torch

    import synth
    from paper_0911_2285_amd import ebicg as eb

    V = synth.volume(dims)
    op = eb.op_create(synth.random_su3_links(dims, 0.3, synth.gauge_seed(1)), kappa, dims, bc_t=-1,
                      defl_capacity=n1 * nev)
    for i in range(n1):
        b = torch.from_numpy(synth.z2_source(V, synth.rhs_seed(0, i))).to("cuda:0")
        eb.eigbicg_solve(op, b, torch.zeros_like(b), nev, m, 1e-10)
    B = torch.stack([torch.from_numpy(synth.z2_source(V, synth.rhs_seed(0, n1 + i))) for i in range(nrhs)]).to("cuda:0")
    X = torch.zeros_like(B)
    st = eb.deflated_bicg_solve(op, B, X, tol=1e-10, nrhs=nrhs, batch=nrhs, inner="fp32", inner_tol=1e-6)
    torch.cuda.synchronize()
    log(f"[bench] proj pass done: K = {eb.defl_info(op)[0]}, batch of {nrhs}, residual {st['true_rel_resid']:.2e}")


def pmc_pass(workload):
    """One eigBiCG solve (its BiCG matvec launches are the roofline kernel), then a
    plain device copy of COPY_BYTES for the counter calibration."""
    import torch

    import synth
    from paper_0911_2285_amd import ebicg as eb

    W = WORKLOADS[workload]
    dims = W["dims"]
    V = synth.volume(dims)
    U = synth.random_su3_links(dims, 0.3, synth.gauge_seed(W["cfg"]))
    op = eb.op_create(U, W["kappa"], dims, bc_t=-1, defl_capacity=W["nev"])
    b = torch.from_numpy(synth.z2_source(V, synth.rhs_seed(0, 0))).to("cuda:0")
    eb.eigbicg_solve(op, b, torch.zeros_like(b), nev=W["nev"], m=W["m"], tol=W["tol"])
    src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log("[bench] pmc pass done")


def summarize_pmc(fetch_csv, write_csv, workload, kernel="k_bicg_matvec", cls="bicg_matvec"):
    import csv

    def per_dispatch(path, counter, match):
        vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(path))
                if r["Counter_Name"].startswith(counter) and match(r["Kernel_Name"])]
        return sum(vals) / len(vals), len(vals)

    def calibration(path, counter):
        # the pass ends with three device-to-device copies of COPY_BYTES (the runtime's blit kernel)
        rows = [r for r in csv.DictReader(open(path))
                if r["Counter_Name"].startswith(counter) and "copyBuffer" in r["Kernel_Name"]]
        rows.sort(key=lambda r: int(r["Dispatch_Id"]))
        vals = [float(r["Counter_Value"]) for r in rows[-3:]]
        return sum(vals) / len(vals)

    # the general form's launches (the template's gamma5 instance is another kernel)
    is_kernel = lambda n: kernel + "(" in n or kernel + "<false>(" in n
    f_k, n_f = per_dispatch(fetch_csv, "FETCH_SIZE", is_kernel)
    w_k, n_w = per_dispatch(write_csv, "WRITE_SIZE", is_kernel)
    f_c = calibration(fetch_csv, "FETCH_SIZE")
    w_c = calibration(write_csv, "WRITE_SIZE")
    fetch_scale = COPY_BYTES / (f_c * 1024.0)
    write_scale = COPY_BYTES / (w_c * 1024.0)
    traffic = f_k * 1024.0 * fetch_scale + w_k * 1024.0 * write_scale
    W = WORKLOADS[workload]
    V = 1
    for d in W["dims"]:
        V *= d
    out = {
        "kernel": kernel, "class": cls, "workload": workload, "source_hash": kernel_source_hash(),
        "dispatches": {"fetch": n_f, "write": n_w},
        "fetch_kib_per_dispatch": round(f_k, 1), "write_kib_per_dispatch": round(w_k, 1),
        "copy_calibration": {"bytes_read_and_written": COPY_BYTES, "fetch_kib": round(f_c, 1),
                             "write_kib": round(w_c, 1), "fetch_scale": round(fetch_scale, 4),
                             "write_scale": round(write_scale, 4)},
        "traffic_bytes_per_launch": round(traffic),
        "algorithmic_bytes_per_launch": KERNEL_UNITS[cls] * UNIT_BYTES_FP64 * V,
        "commands": [
            "rocprofv3 --pmc FETCH_SIZE -f csv -d gpurun_out/pmc_fetch -o run -- python3 bench.py --pmc-pass",
            "rocprofv3 --pmc WRITE_SIZE -f csv -d gpurun_out/pmc_write -o run -- python3 bench.py --pmc-pass",
            "python3 bench.py --summarize-pmc gpurun_out/pmc_fetch/run_counter_collection.csv "
            "gpurun_out/pmc_write/run_counter_collection.csv",
        ],
    }
    path = os.path.join(ROOT, "profiles", f"pmc_{cls}_{workload}.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


def measured_traffic(workload, cls):
    """Traffic per launch from the committed counter summary, if the kernel sources
    are unchanged since it was taken; else None."""
    path = os.path.join(ROOT, "profiles", f"pmc_{cls}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_hash") != kernel_source_hash():
        return None
    return rec["traffic_bytes_per_launch"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="inc16x32", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-timing", action="store_true", help="do not record per-kernel HIP events")
    ap.add_argument("--no-large", action="store_true", help="skip the 24^3 x 64 multi-RHS / precision section")
    ap.add_argument("--no-side", action="store_true",
                    help="skip the side records (multi-RHS table, gamma5 and even-odd forms, sweeps)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving (continuous batching) section")
    ap.add_argument("--no-batching", action="store_true", help="skip the 32^3 x 64 batching section")
    ap.add_argument("--batching-only", action="store_true", help="run only the 32^3 x 64 batching section")
    ap.add_argument("--serving-only", action="store_true", help="run only the serving section and print it")
    ap.add_argument("--proj-pass", action="store_true", help="deflation projections on the matrix cores, for --pmc")
    ap.add_argument("--stencil-pass", action="store_true", help="multi-RHS FP32 stencil launches for rocprofv3 --pmc")
    ap.add_argument("--stencil-form", type=int, default=0, help="tile form of the k > 1 launches of --stencil-pass")
    ap.add_argument("--pmc-pass", action="store_true", help="one eigBiCG solve and a calibration copy, for rocprofv3 --pmc")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/pmc_<kernel>_<workload>.json from two counter runs")
    args = ap.parse_args()
    if args.summarize_pmc:
        summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1], args.workload)
        return
    if args.pmc_pass:
        pmc_pass(args.workload)
        return
    if args.stencil_pass:
        stencil_pass(form=args.stencil_form)
        return
    if args.proj_pass:
        proj_pass()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {args.gpus} requested): the multi-GPU path is design-only",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_0911_2285_amd import ebicg as eb

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.serving_only:
        print(json.dumps({"serving": serving(eb)}), flush=True)
        return
    if args.batching_only:
        print(json.dumps({"batching": batching(eb)}), flush=True)
        return
    W = WORKLOADS[args.workload]
    dims = W["dims"]
    V = synth.volume(dims)
    dev = torch.device("cuda:0")
    log(f"[bench] workload {args.workload}: dims={dims} kappa={W['kappa']} nrhs={W['nrhs']} n1={W['n1']}")
    U = synth.random_su3_links(dims, 0.3, synth.gauge_seed(W["cfg"]))
    op = eb.op_create(U, W["kappa"], dims, bc_t=-1, defl_capacity=W["n1"] * W["nev"])
    B_np = [synth.z2_source(V, synth.rhs_seed(0, i)) for i in range(W["nrhs"])]
    B = [torch.from_numpy(b).to(dev) for b in B_np]
    X = [torch.zeros_like(b) for b in B]
    torch.cuda.synchronize()

    for w in range(args.warmup):
        lat, its = [], []
        run_step(eb, op, B, X, W, lat, its)
        log(f"[bench] warmup step {w}: {sum(lat):.3f} s, iterations {its}")

    # In the timed steps only the roofline kernel's launches carry HIP events
    # (each recorded launch costs two host-side event records); the per-kernel
    # table comes from one more, separately instrumented step below.
    if not args.no_timing:
        eb.timing_classes(op, [ROOFLINE_CLASS])
        eb.timing_enable(op, True)
    lat, its = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        run_step(eb, op, B, X, W, lat, its)
        log(f"[bench] step {k} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ktimes = eb.timing_read(op) if not args.no_timing else {}
    eb.timing_enable(op, False)
    # per-kernel table: one more step with every class instrumented (not timed)
    ktable = {}
    if not args.no_timing:
        eb.timing_classes(op, None)
        eb.timing_enable(op, True)
        run_step(eb, op, B, X, W, [], [])
        ktable = eb.timing_read(op)
        eb.timing_enable(op, False)

    n_solves = W["nrhs"] * args.steps
    value = n_solves / elapsed
    per_step_its = its[: W["nrhs"]]
    eig_its = sum(per_step_its[: W["n1"]])
    stab_its = sum(per_step_its[W["n1"]:])
    log(f"[bench] {n_solves} solves in {elapsed:.3f} s -> {value:.2f} solves/s; iterations/RHS {per_step_its}")

    # roofline of the dominant kernel: algorithmic bytes / average launch time
    roof = None
    kernels = {}
    for name, (n, ms) in ktable.items():
        if n == 0:
            continue
        rec = {"launches": n, "total_ms": round(ms, 3), "avg_us": round(1e3 * ms / n, 2)}
        if name in KERNEL_UNITS:
            bytes_per_launch = KERNEL_UNITS[name] * UNIT_BYTES_FP64 * V
            rec["GBps"] = round(bytes_per_launch / (ms / n * 1e-3) / 1e9, 1)
        kernels[name] = rec
    n_roof, ms_roof = ktimes.get(ROOFLINE_CLASS, (0, 0.0))
    # launches that did work: one BiCG matvec per eigBiCG iteration.  The host
    # queues iterations ahead of the convergence test, and the few launched
    # past it return at once; they are recorded too but do no work, so the
    # average is taken over the working launches (their ~1 us is included in
    # the total, which only lowers the figure).
    n_work = sum(sum(its[k * W["nrhs"]: k * W["nrhs"] + W["n1"]]) for k in range(args.steps))
    if n_roof:
        dom = ROOFLINE_CLASS
        bpl = KERNEL_UNITS[dom] * UNIT_BYTES_FP64 * V
        avg_us = 1e3 * ms_roof / min(n_roof, n_work) if n_work else 1e3 * ms_roof / n_roof
        ach = round(bpl / (avg_us * 1e-6) / 1e9, 1)
        roof = {
            "kernel": dom,
            "bound": "hbm",
            "achieved": ach,
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBPS, 4),
            "traffic": measured_traffic(args.workload, dom),
            "bytes_per_launch": bpl,
            "avg_launch_us": round(avg_us, 2),
            "launches": n_roof,
            "working_launches": n_work,
        }
        log(f"[bench] kernel times: {json.dumps(kernels)}")

    # deflated phase in mixed precision (FP32 inner, FP64 refinement) vs FP64,
    # with the space grown by the last step still in place
    extra = {}
    modes = {"fp64": dict(), "mixed_fp32_inner": dict(inner="fp32", inner_tol=1e-6),
             "mixed_bf16_inner": dict(inner="bf16", inner_tol=1e-2)}
    dt = {k: 0.0 for k in modes}
    mode_its = {k: [] for k in modes}
    for i in range(W["n1"], W["nrhs"]):
        for name, kw in modes.items():
            X[i].zero_()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            st = eb.deflated_bicg_solve(op, B[i], X[i], tol=W["tol"], maxiter=20000, **kw)
            dt[name] += time.perf_counter() - t1
            assert st["true_rel_resid"] <= W["tol"], (name, st)
            mode_its[name].append((st["iters"], st["outer_steps"]))
    nd = W["nrhs"] - W["n1"]
    extra["deflated_solves_per_s"] = {k: round(nd / dt[k], 3) for k in modes}
    extra["deflated_iters_outer"] = {k: mode_its[k][:4] for k in modes}
    # multi-RHS: the 16 deflated sources in batches (FP32 / BF16 inner, batch chosen by the library)
    nd = W["nrhs"] - W["n1"]
    Bd = torch.stack(B[W["n1"]:])
    extra["autotune_seconds"] = tune_untimed(eb, op, ("fp32", "bf16"))
    for name, kw in [("mixed_fp32_batched", dict(inner="fp32", inner_tol=1e-6)),
                     ("mixed_bf16_batched", dict(inner="bf16", inner_tol=1e-2))]:
        Xd = torch.zeros_like(Bd)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st = eb.deflated_bicg_solve(op, Bd, Xd, tol=W["tol"], maxiter=20000, nrhs=nd, batch=0, **kw)
        dt_b = time.perf_counter() - t1
        assert st["true_rel_resid"] <= W["tol"], (name, st)
        extra["deflated_solves_per_s"][name] = round(nd / dt_b, 3)
    # the batch autotuner's choice on this operator (k and tile form per precision)
    extra["autotune"] = {p: eb.op_batch_tune(op, p) for p in ("fp32", "bf16")}
    # the whole step with its deflated phase mixed (BF16 / FP32 inner, batched)
    # against the FP64 step above; every solve still at the FP64 true residual tol
    extra["mixed_step"] = {}
    for name, inner, itol in (("bf16_inner_batched", "bf16", 1e-2), ("fp32_inner_batched", "fp32", 1e-6)):
        dts = [run_mixed_step(eb, op, B, X, W, inner, itol) for _ in range(args.steps)]
        extra["mixed_step"][name] = {"solves_per_s": round(W["nrhs"] * len(dts) / sum(dts), 3),
                                     "ms_per_step": round(1e3 * sum(dts) / len(dts), 3)}
    extra["mixed_step"]["fp64_step_solves_per_s"] = round(value, 3)
    log(f"[bench] mixed step: {extra['mixed_step']}")
    # the side records (skipped with --no-side, e.g. to profile the headline workload alone)
    if not args.no_side:
        extra["multi_rhs_stencil"] = multi_rhs_stencil(eb, op, V)
        # the same step with eigBiCG solves 2..n1 in the gamma5-Hermitian form
        # (Sec. 4: one D per iteration, shadow vectors implicit)
        lat5, its5 = [], []
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        run_step(eb, op, B, X, W, lat5, its5, g5=True)
        torch.cuda.synchronize()
        dt5 = time.perf_counter() - t1
        n1 = W["n1"]
        last = slice((args.steps - 1) * W["nrhs"], args.steps * W["nrhs"])
        lat_g, its_g = lat[last], its[last]
        extra["gamma5_form"] = {
            "solves_per_s": round(W["nrhs"] / dt5, 3),
            "iters_per_rhs": its5,
            "eigbicg_ms_per_iter_solves_2_to_n1": {
                "general": round(1e3 * sum(lat_g[1:n1]) / sum(its_g[1:n1]), 4),
                "gamma5": round(1e3 * sum(lat5[1:n1]) / sum(its5[1:n1]), 4),
            },
        }
        log(f"[bench] gamma5 form: {extra['gamma5_form']}")
        # the same step on the even-odd (Schur) form: the paper's test matrices are
        # even-odd preconditioned; every solve still reaches ||b - D x|| <= tol ||b||
        op_eo = eb.op_create(U, W["kappa"], dims, bc_t=-1, defl_capacity=W["n1"] * W["nev"], eo=True)
        run_step(eb, op_eo, B, X, W, [], [])
        lat_e, its_e = [], []
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        run_step(eb, op_eo, B, X, W, lat_e, its_e)
        torch.cuda.synchronize()
        dt_e = time.perf_counter() - t1
        # its deflated solves with FP32 / BF16-stored inner BiCGStab in FP64 refinement
        eo_defl = {}
        for name, kw in [("fp64", dict()), ("mixed_fp32_inner", dict(inner="fp32", inner_tol=1e-6)),
                         ("mixed_bf16_inner", dict(inner="bf16", inner_tol=1e-2))]:
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            for i in range(W["n1"], W["nrhs"]):
                X[i].zero_()
                st = eb.deflated_bicg_solve(op_eo, B[i], X[i], tol=W["tol"], maxiter=20000, **kw)
                assert st["true_rel_resid"] <= W["tol"], (name, st)
            torch.cuda.synchronize()
            eo_defl[name] = round((W["nrhs"] - W["n1"]) / (time.perf_counter() - t2), 3)
        # and in batches (batch chosen by the library's autotuner, run before the timed solves)
        eo_tune = tune_untimed(eb, op_eo, ("fp64", "fp32", "bf16"))
        for name, kw in [("fp64_batched", dict()), ("mixed_fp32_batched", dict(inner="fp32", inner_tol=1e-6)),
                         ("mixed_bf16_batched", dict(inner="bf16", inner_tol=1e-2))]:
            Xd = torch.zeros_like(Bd)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            st = eb.deflated_bicg_solve(op_eo, Bd, Xd, tol=W["tol"], maxiter=20000, nrhs=nd, batch=0, **kw)
            torch.cuda.synchronize()
            assert st["true_rel_resid"] <= W["tol"], (name, st)
            eo_defl[name] = round(nd / (time.perf_counter() - t2), 3)
        eb.op_destroy(op_eo)
        extra["even_odd"] = {
            "solves_per_s": round(W["nrhs"] / dt_e, 3),
            "ms_per_step": round(1e3 * dt_e, 3),
            "iters_per_rhs": its_e,
            "p50_ms": round(1e3 * percentile(lat_e, 50), 3),
            "deflated_solves_per_s": eo_defl,
            "autotune_seconds": eo_tune,
        }
        log(f"[bench] even-odd form: {extra['even_odd']}")
        if not args.no_serving:
            extra["serving"] = serving(eb)
        extra["deflation_sweep"] = deflation_sweep(eb)
        extra["table1_analogue"] = table1_analogue(eb)
        log(f"[bench] deflation sweep: {extra['deflation_sweep']}")
    # undeflated FP64 BiCGStab on the same sources, for the deflation speed-up
    eb.defl_reset(op)
    plain_its = []
    for i in range(W["n1"], min(W["nrhs"], W["n1"] + 4)):
        X[i].zero_()
        st = eb.deflated_bicg_solve(op, B[i], X[i], tol=W["tol"], maxiter=20000)
        plain_its.append(st["iters"])
    extra["undeflated_bicgstab_iters"] = plain_its

    if not args.no_large:
        extra["large_lattice"] = large_lattice(eb, (24, 24, 24, 64), 0.123, 16, W["tol"])
    if not args.no_batching:
        extra["batching"] = batching(eb)

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample ...")
        cpu = cpu_baseline(W, U, B_np[0], eig_its, stab_its)
        log(f"[bench] cpu baseline {cpu['value']:.4g} solves/s")

    out = {
        "metric": "solves/s at 1e-10 rel. resid (mixed vs FP64), dslash HBM GB/s, p50/p99",
        "value": round(value, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"incremental eigBiCG, Wilson-Dirac {'x'.join(map(str, dims))}, kappa {W['kappa']}, "
                        f"eps 0.3 SU(3) links, {W['nrhs']} Z2 sources: {W['n1']} eigBiCG (nev {W['nev']}, "
                        f"m {W['m']}) + {W['nrhs'] - W['n1']} deflated BiCGStab, tol {W['tol']}",
            "lattice": list(dims),
            "nrhs": W["nrhs"],
            "parallelism": "single GPU",
        },
        "roofline": roof,
        "cpu_baseline": cpu,
        "dslash_GBps": roof["achieved"] if roof else None,
        "p50_ms": round(1e3 * percentile(lat, 50), 3),
        "p99_ms": round(1e3 * percentile(lat, 99), 3),
        "iters_per_rhs": per_step_its,
        "kernels": kernels,
        "kernels_note": "per-kernel HIP-event times from one extra step with every kernel class instrumented (averages include the launches queued past convergence, which return at once); "
                        "the timed steps instrument only the roofline kernel",
        **extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
