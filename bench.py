#!/usr/bin/env python3
"""Benchmark: incremental eigBiCG's deflated multi-RHS solves on one MI355X.

The bench line's workload (one "step" = the hot path over one batch of
right-hand sides): 32^3 x 64 Wilson-Dirac operator, kappa = 0.123, SU(3)
links exp(i 0.3 H) (seeded), a 100-pair left/right deflation space grown in
setup by 4 eigBiCG solves (nev = 25, m = 60), and per step 16 Z2-noise
sources resident in HBM solved by deflated BiCGStab in batches of k columns
(multi-RHS stencil; k and the tile form chosen by the library's autotuner in
setup), complex64 inner iterations inside complex128 iterative refinement.
Every solve reaches ||b - A x|| / ||b|| <= 1e-10, checked in FP64.

Prints ONE JSON line on stdout: solves/s of that step, the dominant kernel's
roofline (achieved algorithmic GB/s from HIP events inside the library over
the timed steps), FP64 comparators on the same GPU (plain BiCG, plain and
deflated BiCGStab), the CPU oracle timed on the host cores, and side records
(the 16^3 x 32 incremental eigBiCG step, serving, sweeps, 24^3 x 64).
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
# the dominant kernel of the 16^3 x 32 incremental step (a side record)
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
    "dslash1_march": 5,  # D on one FP64 column in the t-marching form: in; out; links
}

WORKLOADS = {
    # the incremental-eigBiCG workload: 16^3 x 32, 8 eigBiCG + 16 deflated solves
    "inc16x32": dict(dims=(16, 16, 16, 32), kappa=0.122, nrhs=24, n1=8, nev=10, m=40, tol=1e-10, cfg=1),
    # the small parity workload (4^4), for quick runs
    "inc4": dict(dims=(4, 4, 4, 4), kappa=0.115, nrhs=4, n1=4, nev=4, m=16, tol=1e-10, cfg=0),
    # the precision lattice, 24^3 x 64 (fields beyond the Infinity Cache): counters of its BiCG matvec
    "prec24x64": dict(dims=(24, 24, 24, 64), kappa=0.123, nrhs=32, n1=8, nev=10, m=40, tol=1e-10, cfg=2),
    # the bench line: 32^3 x 64 batched mixed-precision deflated solves (100 pairs)
    "batch32x64": dict(dims=(32, 32, 32, 64), kappa=0.123, nrhs=16, n1=4, nev=25, m=60, tol=1e-10, cfg=3,
                       inner="fp32", inner_tol=1e-6),
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
BATCH_SOURCES = ["batch.hip", "stencil.h", "kernel_util.h", "device_common.h", "kernels.h"]


def kernel_source_hash(cls="bicg_matvec"):
    import hashlib

    h = hashlib.sha256()
    for f in (BATCH_SOURCES if cls.startswith("bstab") or cls == "dslash1_march" else KERNEL_SOURCES):
        with open(os.path.join(ROOT, "paper_0911_2285_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def deflation_sweep(eb):
    """Deflation speed-up on small near-critical lattices with rough links (the
    analogue of the paper's Fig. 1): BiCGStab iterations per right-hand side
    after n1 = 8 eigBiCG solves for three (nev, m), and for (10, 40) after
    n1 = 2, 4, 8, 12 solves, against the same sources undeflated.  The
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
        # the n1 axis of Fig. 1: (nev, m) = (10, 40), the space after n1 = 2, 4, 8, 12
        # eigBiCG solves, each tried on the same four further sources
        B2 = [torch.from_numpy(synth.z2_source(V, synth.rhs_seed(0, i))).to("cuda:0") for i in range(12, 16)]
        op = eb.op_create(U, kappa, dims, bc_t=-1, defl_capacity=120)
        und2 = [eb.deflated_bicg_solve(op, b, torch.zeros_like(b), tol=1e-8, maxiter=20000)["iters"] for b in B2]
        axis = []
        for i in range(12):
            eb.eigbicg_solve(op, B[i], torch.zeros_like(B[i]), nev=10, m=40, tol=1e-8, maxiter=20000)
            if i + 1 in (2, 4, 8, 12):
                it = [eb.deflated_bicg_solve(op, b, torch.zeros_like(b), tol=1e-8, maxiter=20000)["iters"] for b in B2]
                axis.append({"n1": i + 1, "K": eb.defl_info(op)[0], "deflated_iters": it,
                             "speedup": round(float(np.mean(und2) / np.mean(it)), 3)})
        eb.op_destroy(op)
        out.append({"lattice": list(dims), "eps": 1.0, "kappa": kappa, "nev": 10, "m": 40,
                    "undeflated_iters": und2, "n1_axis": axis})
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
    """One pass of the workload's roofline kernel, then a plain device copy of
    COPY_BYTES for the counter calibration: for the incremental workloads one
    eigBiCG solve (its BiCG matvec launches) and three applications of D to one
    FP64 column in the t-marching form, for batch32x64 batched
    mixed-precision solves of the 16 sources at k = 2, 4, 8 and 16, each k in
    its tuned tile form (no deflation space, which does not change the passes)."""
    import torch

    import synth
    from paper_0911_2285_amd import ebicg as eb

    W = WORKLOADS[workload]
    if "inner" in W:
        dims = W["dims"]
        V = synth.volume(dims)
        op = eb.op_create(synth.random_su3_links(dims, 0.3, synth.gauge_seed(W["cfg"])), W["kappa"], dims, bc_t=-1)
        tuned = eb.op_batch_tune(op, W["inner"])
        B = torch.stack([torch.from_numpy(synth.z2_source(V, synth.rhs_seed(W["cfg"], i)))
                         for i in range(W["nrhs"])]).to("cuda:0")
        for kk in (2, 4, 8, 16):  # every k the tuner may pick, each in its tuned tile form
            X = torch.zeros_like(B)
            eb.deflated_bicg_solve(op, B, X, tol=W["tol"], maxiter=20000, nrhs=W["nrhs"], inner=W["inner"],
                                   inner_tol=W["inner_tol"], batch=kk)
            del X
        k = tuned["k"]
        del B
        src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] pmc pass done (batched, k = {k})")
        return
    dims = W["dims"]
    V = synth.volume(dims)
    U = synth.random_su3_links(dims, 0.3, synth.gauge_seed(W["cfg"]))
    op = eb.op_create(U, W["kappa"], dims, bc_t=-1, defl_capacity=W["nev"])
    eb.op_set_matvec_form(op, 1)  # the staged pair, whatever a timing under the profiler would pick
    b = torch.from_numpy(synth.z2_source(V, synth.rhs_seed(0, 0))).to("cuda:0")
    eb.eigbicg_solve(op, b, torch.zeros_like(b), nev=W["nev"], m=W["m"], tol=W["tol"])
    # the staged pair with one tile per block, the wider grid its timing may choose
    # (32768: the blocks whose sigma records fill a record region)
    op2 = eb.op_create(U, W["kappa"], dims, bc_t=-1, defl_capacity=W["nev"])
    eb.op_set_grid_cap(op2, 32768)
    eb.op_set_matvec_form(op2, 1)
    eb.eigbicg_solve(op2, b, torch.zeros_like(b), nev=W["nev"], m=W["m"], tol=W["tol"])
    eb.op_destroy(op2)
    # D on one FP64 column in the t-marching form (the one-at-a-time solver's stencil)
    eb.op_batch_set_tile(op, "fp64", 1, 6)
    y = torch.empty_like(b)
    for _ in range(3):
        eb.op_apply_block(op, y, b, 1)
    src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log("[bench] pmc pass done")


def _template_args(name, kernel):
    """Top-level template arguments of kernel<...> in a demangled kernel name."""
    i = name.find(kernel + "<")
    if i < 0:
        return None
    j, depth, args, cur = i + len(kernel) + 1, 1, [], ""
    while j < len(name) and depth:
        ch = name[j]
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
            if depth == 0:
                break
        if ch == "," and depth == 1:
            args.append(cur.strip())
            cur = ""
        else:
            cur += ch
        j += 1
    args.append(cur.strip())
    return args


def summarize_pmc(fetch_csv, write_csv, workload, kernel="k_bicg_matvec", cls="bicg_matvec"):
    import csv

    def rows_of(path, counter):
        return [r for r in csv.DictReader(open(_find_csv(path, "counter_collection.csv")))
                if r["Counter_Name"].startswith(counter)]

    def calibration(path, counter):
        # the pass ends with three device-to-device copies of COPY_BYTES (the runtime's blit kernel)
        rows = [r for r in rows_of(path, counter) if "copyBuffer" in r["Kernel_Name"]]
        rows.sort(key=lambda r: int(r["Dispatch_Id"]))
        vals = [float(r["Counter_Value"]) for r in rows[-3:]]
        return sum(vals) / len(vals)

    W = WORKLOADS[workload]
    V = 1
    for d in W["dims"]:
        V *= d
    f_c = calibration(fetch_csv, "FETCH_SIZE")
    w_c = calibration(write_csv, "WRITE_SIZE")
    fetch_scale = COPY_BYTES / (f_c * 1024.0)
    write_scale = COPY_BYTES / (w_c * 1024.0)
    out = {"kernel": kernel, "class": cls, "workload": workload, "source_hash": kernel_source_hash(cls)}
    if cls.startswith("bstab"):
        # batched pass: its kernel is k_bstab_* (or the t-marching k_bmarch with epilogue 1 for
        # v, 2 for t); the columns per batch k is the kernel's second template argument.  Per k,
        # the dispatches in which every column still iterates (WRITE_SIZE at its maximum; the
        # others skip stopped columns), matched between the two runs by their order.
        epi = {"bstab_v": "1", "bstab_t": "2"}.get(cls)

        def k_of(name):
            a = _template_args(name, kernel)
            if a is None:  # the variant that sums its producer's records itself (small grids)
                a = _template_args(name, kernel + "_f")
            if a is None and epi is not None:
                a = _template_args(name, "k_bmarch")
                if a is None or a[-1] != epi:
                    return None
            return int(a[1]) if a else None

        cb = CPLX_BYTES[W["inner"]]
        writes = 2 if cls == "bstab_xr" else 1  # spinors written per column
        links = 36 if cls in BATCH_STENCILS else 0
        fr, wr = rows_of(fetch_csv, "FETCH_SIZE"), rows_of(write_csv, "WRITE_SIZE")
        per_k = {}
        for kc in sorted({k_of(r["Kernel_Name"]) for r in wr} - {None}):
            wk = sorted((r for r in wr if k_of(r["Kernel_Name"]) == kc), key=lambda r: int(r["Dispatch_Id"]))
            fk = sorted((r for r in fr if k_of(r["Kernel_Name"]) == kc), key=lambda r: int(r["Dispatch_Id"]))
            wmax = max(float(r["Counter_Value"]) for r in wk)
            order = [i for i, r in enumerate(wk) if float(r["Counter_Value"]) >= 0.99 * wmax and i < len(fk)]
            f_k = sum(float(fk[i]["Counter_Value"]) for i in order) / len(order)
            w_k = sum(float(wk[i]["Counter_Value"]) for i in order) / len(order)
            traffic = f_k * 1024.0 * fetch_scale + w_k * 1024.0 * write_scale
            algo = V * (links + 12 * BATCH_COL_SPINORS[cls] * kc) * cb
            per_k[str(kc)] = {"dispatches": len(order), "fetch_kib_per_dispatch": round(f_k, 1),
                              "write_kib_per_dispatch": round(w_k, 1), "traffic_bytes_per_launch": round(traffic),
                              "algorithmic_bytes_per_launch": algo,
                              "traffic_over_algorithmic": round(traffic / algo, 3),
                              "expected_write_kib": V * 12 * writes * kc * cb / 1024.0}
        out["per_k"] = per_k
    else:
        # the general form's launches (the template's gamma5 instance is another kernel);
        # the one-column march: k_bmarch<double2, 1, -1, 0> (FP64, one column, D, no epilogue)
        def is_kernel(n):
            if cls == "dslash1_march":
                a = _template_args(n, kernel)
                return a is not None and "double" in a[0] and a[1:] == ["1", "-1", "0"]
            return kernel + "(" in n or kernel + "<false>(" in n
        # dispatches per grid size (the pass runs the BiCG matvec at the default grid and
        # with one tile per block); the top-level figures are the default grid's
        def by_grid(path, counter):
            g = {}
            for r in rows_of(path, counter):
                if is_kernel(r["Kernel_Name"]):
                    g.setdefault(int(r.get("Grid_Size") or 0), []).append(float(r["Counter_Value"]))
            return g

        fg, wg = by_grid(fetch_csv, "FETCH_SIZE"), by_grid(write_csv, "WRITE_SIZE")
        algo = KERNEL_UNITS[cls] * UNIT_BYTES_FP64 * V

        def figures(fv, wv):
            f_k, w_k = sum(fv) / len(fv), sum(wv) / len(wv)
            traffic = f_k * 1024.0 * fetch_scale + w_k * 1024.0 * write_scale
            return {"dispatches": {"fetch": len(fv), "write": len(wv)},
                    "fetch_kib_per_dispatch": round(f_k, 1), "write_kib_per_dispatch": round(w_k, 1),
                    "traffic_bytes_per_launch": round(traffic), "algorithmic_bytes_per_launch": algo,
                    "traffic_over_algorithmic": round(traffic / algo, 3)}

        grids = sorted(set(fg) & set(wg))
        out.update(figures(fg[grids[0]], wg[grids[0]]))
        if len(grids) > 1:
            out["by_grid_size"] = {str(gs): figures(fg[gs], wg[gs]) for gs in grids}
    out["copy_calibration"] = {"bytes_read_and_written": COPY_BYTES, "fetch_kib": round(f_c, 1),
                               "write_kib": round(w_c, 1), "fetch_scale": round(fetch_scale, 4),
                               "write_scale": round(write_scale, 4)}
    out["commands"] = [
        f"rocprofv3 --pmc FETCH_SIZE -f csv -d gpurun_out/pmc_fetch -o run -- python3 bench.py --pmc-pass "
        f"--workload {workload}",
        f"rocprofv3 --pmc WRITE_SIZE -f csv -d gpurun_out/pmc_write -o run -- python3 bench.py --pmc-pass "
        f"--workload {workload}",
        f"python3 bench.py --workload {workload} --summarize-pmc gpurun_out/pmc_fetch gpurun_out/pmc_write",
    ]
    path = os.path.join(ROOT, "profiles", f"pmc_{cls}_{workload}.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


def _find_csv(path, suffix):
    """path: a CSV file, or a rocprofv3 output directory searched for *suffix."""
    import glob

    if os.path.isfile(path):
        return path
    hits = sorted(glob.glob(os.path.join(path, "**", "*" + suffix), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {path}")
    return hits[-1]


def eigbicg_pass(eb, mode, workload="inc16x32"):
    """The eigBiCG gap workload for a kernel trace: the workload's lattice, nev and
    m (16^3 x 32: nev 10, m 40; 32^3 x 64: nev 25, m 60), tol 1e-10, FP64 window
    with the host or the device restart, or (fp32) the FP32 window with the device
    restart; one warm-up solve, three marker launches (D on a 2^4
    operator), two timed solves from an empty space, three more markers.  Prints
    iterations, restarts and ms per iteration."""
    import torch

    import synth

    W = WORKLOADS[workload]
    dims, kappa = W["dims"], W["kappa"]
    V = synth.volume(dims)
    U = synth.random_su3_links(dims, 0.3, synth.gauge_seed(W["cfg"]))
    op = eb.op_create(U, kappa, dims, bc_t=-1, defl_capacity=2 * W["nev"])
    del U
    mdims = (2, 2, 2, 2)
    mk = eb.op_create(synth.unit_links(mdims), 0.1, mdims)
    mb = torch.ones(16, 4, 3, dtype=torch.complex128, device="cuda:0")
    mo = torch.empty_like(mb)
    B = [torch.from_numpy(synth.z2_source(V, synth.rhs_seed(W["cfg"], i))).to("cuda:0") for i in range(3)]
    # fp32: the FP32 window with the device restart
    kw = dict(nev=W["nev"], m=W["m"], tol=1e-10, window="fp32" if mode == "fp32" else "fp64",
              device_eig=(mode != "host"))
    eb.eigbicg_solve(op, B[0], torch.zeros_like(B[0]), **kw)
    eb.defl_reset(op)
    torch.cuda.synchronize()
    for _ in range(3):
        eb.op_apply(mk, mo, mb)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = rst = 0
    for i in (1, 2):
        st, _ = eb.eigbicg_solve(op, B[i], torch.zeros_like(B[i]), **kw)
        its += st["iters"]
        rst += st["window_restarts"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for _ in range(3):
        eb.op_apply(mk, mo, mb)
    torch.cuda.synchronize()
    print(json.dumps({"workload": workload, "mode": mode, "iters": its, "restarts": rst,
                      "ms_per_iter": round(1e3 * dt / its, 4)}), flush=True)


GAP_CLASSES = [  # (label, kernel-name prefixes)
    ("BiCG step (matvec, r update, x/p update)", ("k_bicg_matvec", "k_bicg_update_r", "k_bicg_update_p")),
    ("window restart rotations (V and W, with the arrow dots)", ("k_combine<HIP_vector_type<double, 2u>, "
                                                                  "HIP_vector_type<double, 2u>, 20,",
                                                                  "k_rotate_mfma")),
    ("window eigenproblems on the device", ("k_window_pair", "k_window_restart", "k_window_final")),
    ("arrow vectors", ("k_arrow_vectors",)),
    ("final extraction and absorb (Ritz vectors, D and D^+ on them, Gram blocks, "
     "projections, residual)", ("k_combine", "k_gram", "k_dslash", "k_ts_", "k_residual", "k_to_soa",
                                "k_from_soa")),
    ("copies (scalar history to the host, coefficients to the device)", ("__amd_rocclr_copyBuffer",)),
]


def summarize_gap(trace_dirs, out_name, command, workload="inc16x32"):
    """profiles/<out_name>.md: where an eigBiCG iteration's time goes, from
    rocprofv3 kernel traces of `bench.py --eigbicg-pass MODE` (one directory per
    mode): the window between the marker launches, the time some kernel runs
    (union over streams), the idle rest, and the kernels by class."""
    import csv

    def kname(n):
        return n.replace("(anonymous namespace)::", "").replace("void ", "").replace("ebicg::", "").split("(")[0]

    W = WORKLOADS[workload]
    lat = "x".join(map(str, W["dims"][:3])) + " x " + str(W["dims"][3])
    out = [f"# eigBiCG iteration time at {lat}, attributed from kernel traces", "",
           "Command (repository root on the MI355X box, `export TMPDIR=/tmp` first), once per mode:", "",
           "```", command, "```", "",
           f"Each run: one warm-up solve, then two eigBiCG solves (nev {W['nev']}, m {W['m']}, tol 1e-10, "
           "FP64 window) "
           "between marker launches.  Window = first to last kernel between the markers; busy = the "
           "union of all kernels' intervals (the device restart runs on a side stream, overlapping the "
           "iterations); idle = window - busy.", ""]
    for mode, d in trace_dirs:
        rows = list(csv.DictReader(open(_find_csv(d, "kernel_trace.csv"))))
        rows.sort(key=lambda r: int(r["Start_Timestamp"]))
        dur = lambda r: int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        mk = [i for i, r in enumerate(rows) if kname(r["Kernel_Name"]).startswith("k_dslash") and dur(r) < 20000]
        groups = []
        for i in mk:
            if groups and i - groups[-1][-1] <= 3:
                groups[-1].append(i)
            else:
                groups.append([i])
        g = [x for x in groups if len(x) >= 3]
        win = rows[g[-2][-1] + 1:g[-1][0]]
        t0, t1 = int(win[0]["Start_Timestamp"]), int(win[-1]["End_Timestamp"])
        iv = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"])) for r in win)
        busy, (cs, ce) = 0, iv[0]
        for a, b in iv[1:]:
            if a > ce:
                busy += ce - cs
                cs, ce = a, b
            else:
                ce = max(ce, b)
        busy += ce - cs
        iters = sum(1 for r in win if kname(r["Kernel_Name"]).startswith("k_bicg_update_p"))
        cls = {lab: 0 for lab, _ in GAP_CLASSES}
        other = 0
        for r in win:
            n = kname(r["Kernel_Name"])
            for lab, pre in GAP_CLASSES:
                if any(n.startswith(p.replace("ebicg::", "")) for p in pre):
                    cls[lab] += dur(r)
                    break
            else:
                other += dur(r)
        us = lambda ns: ns / 1e3
        out += [f"## {mode} restart", "",
                f"Window {us(t1 - t0) / 1e3:.2f} ms for {iters} iterations: {us(t1 - t0) / iters:.1f} us per "
                f"iteration; some kernel running {us(busy) / 1e3:.2f} ms ({100 * busy / (t1 - t0):.1f} %), "
                f"idle {us(t1 - t0 - busy) / 1e3:.2f} ms ({us(t1 - t0 - busy) / iters:.1f} us per iteration).", "",
                "| class | total (ms) | us per iteration | share of the window |", "|---|---:|---:|---:|"]
        for lab, _ in GAP_CLASSES:
            if cls[lab]:
                out.append(f"| {lab} | {us(cls[lab]) / 1e3:.2f} | {us(cls[lab]) / iters:.1f} | "
                           f"{100 * cls[lab] / (t1 - t0):.1f} % |")
        if other:
            out.append(f"| other | {us(other) / 1e3:.2f} | {us(other) / iters:.1f} | {100 * other / (t1 - t0):.1f} % |")
        out.append("")
    path = os.path.join(ROOT, "profiles", out_name + ".md")
    with open(path, "w") as f:
        f.write("\n".join(out) + "\n")
    print("wrote", path)


def summarize_trace(prof_dir, bench_json, workload, out_name, command, top=20):
    """profiles/<out_name>.md from a rocprofv3 --kernel-trace --stats run of bench.py:
    the top kernels by total time from its kernel stats, launches longer than 5 us
    from its kernel trace, and the bench line's own per-class figures for comparison."""
    import csv

    stats = list(csv.DictReader(open(_find_csv(prof_dir, "kernel_stats.csv"))))
    trace = list(csv.DictReader(open(_find_csv(prof_dir, "kernel_trace.csv"))))
    dur = {}
    for r in trace:
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        dur.setdefault(r["Kernel_Name"], []).append(d)
    short = lambda n: n.replace("HIP_vector_type<double, 2u>", "f64").replace("HIP_vector_type<float, 2u>", "f32") \
        .replace("ebicg::bf16c", "bf16").replace("ebicg::(anonymous namespace)::", "").replace("void ", "") \
        .split("(")[0]
    rows = sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))[:top]
    line = None
    if bench_json and os.path.exists(bench_json):
        for ln in open(bench_json):
            ln = ln.strip()
            if ln.startswith("{"):
                line = json.loads(ln)
    out = [f"# Kernel trace: {workload} bench line", "",
           "Command (repository root on the MI355X box, `export TMPDIR=/tmp` first):", "", "```", command, "```", "",
           f"The first {top} kernels of the run's kernel stats by total time.  \"Long launches\" are those "
           "longer than 5 us in the kernel trace of the same run (launches queued past a batch's last "
           "stopped column return at once).", "",
           "| kernel | calls | avg (us) | min (us) | max (us) | total (ms) | % | long launches | long avg (us) |",
           "|---|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for r in rows:
        ds = [d for d in dur.get(r["Name"], []) if d > 5.0]
        out.append(f"| {short(r['Name'])} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                   f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                   f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.2f} | {len(ds)} | "
                   f"{(sum(ds) / len(ds) if ds else 0):.2f} |")
    if line and line.get("kernels", {}).get("batched"):
        out += ["", "The bench line printed by the same run (library HIP events over its timed steps; "
                "working launches = the columns' iterations / k, a lower bound):", "",
                "| class | launches | total (ms) | working launches | ms / working launch | algorithmic GB/s |",
                "|---|---:|---:|---:|---:|---:|"]
        for c, r in line["kernels"]["batched"].items():
            out.append(f"| {c} | {r['launches']} | {r['total_ms']} | {r['working_launches']} | "
                       f"{r['avg_launch_us'] / 1e3:.3f} | {r['achieved_GBps']} |")
        out += ["", f"value {line['value']} solves/s, roofline {json.dumps(line['roofline'])}"]
    path = os.path.join(ROOT, "profiles", out_name + ".md")
    with open(path, "w") as fh:
        fh.write("\n".join(out) + "\n")
    print(path)


def measured_traffic(workload, cls, k=None):
    """Traffic per launch from the committed counter summary, if the kernel sources
    are unchanged since it was taken (and, for a batched pass, it was taken at the
    same k); else None."""
    path = os.path.join(ROOT, "profiles", f"pmc_{cls}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_hash") != kernel_source_hash(cls):
        return None
    if "per_k" in rec:
        r = rec["per_k"].get(str(k))
        return r["traffic_bytes_per_launch"] if r else None
    return rec["traffic_bytes_per_launch"]


# ---------------------------------------------------------------------------
# The 16^3 x 32 incremental step (a side record: its fields sit in the 256 MB
# Infinity Cache, so its stencil rates are effective, not HBM, rates)
# ---------------------------------------------------------------------------
def eigbicg_modes(eb, op, B, W, n, modes=(("fp64", False), ("fp64", True), ("fp32", False), ("fp32", True))):
    """eigBiCG on the first n sources in each (window storage, device restart) mode,
    from an empty space each time, after one untimed solve of the mode:
    milliseconds per iteration, iterations, restarts."""
    import torch

    out = {}
    for window, dev in modes:
        # one untimed solve first: the mode's window buffers are allocated there
        eb.defl_reset(op)
        eb.eigbicg_solve(op, B[0], torch.zeros_like(B[0]), nev=W["nev"], m=W["m"], tol=W["tol"], maxiter=20000,
                         window=window, device_eig=dev)
        eb.defl_reset(op)
        its = rst = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(n):
            x = torch.zeros_like(B[i])
            st, _ = eb.eigbicg_solve(op, B[i], x, nev=W["nev"], m=W["m"], tol=W["tol"], maxiter=20000,
                                     window=window, device_eig=dev)
            assert st["true_rel_resid"] <= W["tol"], st
            its += st["iters"]
            rst += st["window_restarts"]
        dt = time.perf_counter() - t0
        out[f"{window}_window_{'device' if dev else 'host'}_restart"] = {
            "ms_per_iter": round(1e3 * dt / its, 4), "iters": its, "restarts": rst, "solves": n}
    eb.defl_reset(op)
    return out


def incremental_side(eb, W, steps, warmup, timing=True, full=True):
    """Solves/s of the FP64 incremental step (n1 eigBiCG + deflated BiCGStab),
    its dominant kernel's effective GB/s, the mixed-precision and batched
    variants of its deflated phase, and (full) the gamma5-Hermitian and
    even-odd forms of the same step."""
    import torch

    import synth

    dims = W["dims"]
    V = synth.volume(dims)
    dev = torch.device("cuda:0")
    U = synth.random_su3_links(dims, 0.3, synth.gauge_seed(W["cfg"]))
    op = eb.op_create(U, W["kappa"], dims, bc_t=-1, defl_capacity=W["n1"] * W["nev"])
    B = [torch.from_numpy(synth.z2_source(V, synth.rhs_seed(0, i))).to(dev) for i in range(W["nrhs"])]
    X = [torch.zeros_like(b) for b in B]
    for w in range(warmup):
        lat, its = [], []
        run_step(eb, op, B, X, W, lat, its)
    if timing:
        eb.timing_classes(op, [ROOFLINE_CLASS])
        eb.timing_enable(op, True)
    lat, its = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        run_step(eb, op, B, X, W, lat, its)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ktimes = eb.timing_read(op) if timing else {}
    eb.timing_enable(op, False)
    ktable = {}
    if timing:
        eb.timing_classes(op, None)
        eb.timing_enable(op, True)
        run_step(eb, op, B, X, W, [], [])
        ktable = eb.timing_read(op)
        eb.timing_enable(op, False)
    value = W["nrhs"] * steps / elapsed
    per_step_its = its[: W["nrhs"]]
    kernels = {}
    for name, (n, ms) in ktable.items():
        if n == 0:
            continue
        rec = {"launches": n, "total_ms": round(ms, 3), "avg_us": round(1e3 * ms / n, 2)}
        if name in KERNEL_UNITS:
            rec["effective_GBps"] = round(KERNEL_UNITS[name] * UNIT_BYTES_FP64 * V / (ms / n * 1e-3) / 1e9, 1)
        kernels[name] = rec
    n_roof, ms_roof = ktimes.get(ROOFLINE_CLASS, (0, 0.0))
    n_work = sum(sum(its[k * W["nrhs"]: k * W["nrhs"] + W["n1"]]) for k in range(steps))
    eff = None
    if n_roof and n_work:
        bpl = KERNEL_UNITS[ROOFLINE_CLASS] * UNIT_BYTES_FP64 * V
        avg_us = 1e3 * ms_roof / min(n_roof, n_work)
        eff = {"kernel": ROOFLINE_CLASS, "bytes_per_launch": bpl, "avg_launch_us": round(avg_us, 2),
               "effective_GBps": round(bpl / (avg_us * 1e-6) / 1e9, 1),
               "note": "16^3 x 32 FP64 fields (25 MB each) stay in the 256 MB Infinity Cache: an effective rate, "
                       "not an HBM rate",
               "traffic": measured_traffic("inc16x32", ROOFLINE_CLASS)}
    res = {"workload": f"incremental eigBiCG, {'x'.join(map(str, dims))}, kappa {W['kappa']}, {W['nrhs']} Z2 "
                       f"sources: {W['n1']} eigBiCG (nev {W['nev']}, m {W['m']}) + {W['nrhs'] - W['n1']} deflated "
                       f"BiCGStab, FP64, tol {W['tol']}",
           "solves_per_s": round(value, 3), "ms_per_step": round(1e3 * elapsed / steps, 3),
           "p50_ms": round(1e3 * percentile(lat, 50), 3), "p99_ms": round(1e3 * percentile(lat, 99), 3),
           "iters_per_rhs": per_step_its, "matvec_effective": eff, "kernels": kernels}
    # the deflated phase one at a time: FP64 and mixed precision
    modes = {"fp64": dict(), "mixed_fp32_inner": dict(inner="fp32", inner_tol=1e-6),
             "mixed_bf16_inner": dict(inner="bf16", inner_tol=1e-2)}
    dt = {k: 0.0 for k in modes}
    for i in range(W["n1"], W["nrhs"]):
        for name, kw in modes.items():
            X[i].zero_()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            st = eb.deflated_bicg_solve(op, B[i], X[i], tol=W["tol"], maxiter=20000, **kw)
            dt[name] += time.perf_counter() - t1
            assert st["true_rel_resid"] <= W["tol"], (name, st)
    nd = W["nrhs"] - W["n1"]
    res["deflated_solves_per_s"] = {k: round(nd / dt[k], 3) for k in modes}
    Bd = torch.stack(B[W["n1"]:])
    res["autotune_seconds"] = tune_untimed(eb, op, ("fp32", "bf16"))
    for name, kw in [("mixed_fp32_batched", dict(inner="fp32", inner_tol=1e-6)),
                     ("mixed_bf16_batched", dict(inner="bf16", inner_tol=1e-2))]:
        Xd = torch.zeros_like(Bd)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st = eb.deflated_bicg_solve(op, Bd, Xd, tol=W["tol"], maxiter=20000, nrhs=nd, batch=0, **kw)
        dt_b = time.perf_counter() - t1
        assert st["true_rel_resid"] <= W["tol"], (name, st)
        res["deflated_solves_per_s"][name] = round(nd / dt_b, 3)
    res["mixed_step"] = {}
    for name, inner, itol in (("bf16_inner_batched", "bf16", 1e-2), ("fp32_inner_batched", "fp32", 1e-6)):
        dts = [run_mixed_step(eb, op, B, X, W, inner, itol) for _ in range(max(1, min(steps, 2)))]
        res["mixed_step"][name] = {"solves_per_s": round(W["nrhs"] * len(dts) / sum(dts), 3),
                                   "ms_per_step": round(1e3 * sum(dts) / len(dts), 3)}
    res["eigbicg_modes"] = eigbicg_modes(eb, op, B, W, W["n1"])
    log(f"[bench] eigBiCG modes 16^3x32: {res['eigbicg_modes']}")
    if full:
        res["multi_rhs_stencil"] = multi_rhs_stencil(eb, op, V)
        lat5, its5 = [], []
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        run_step(eb, op, B, X, W, lat5, its5, g5=True)
        torch.cuda.synchronize()
        dt5 = time.perf_counter() - t1
        n1 = W["n1"]
        last = slice((steps - 1) * W["nrhs"], steps * W["nrhs"])
        lat_g, its_g = lat[last], its[last]
        res["gamma5_form"] = {
            "solves_per_s": round(W["nrhs"] / dt5, 3),
            "iters_per_rhs": its5,
            "eigbicg_ms_per_iter_solves_2_to_n1": {
                "general": round(1e3 * sum(lat_g[1:n1]) / sum(its_g[1:n1]), 4),
                "gamma5": round(1e3 * sum(lat5[1:n1]) / sum(its5[1:n1]), 4),
            },
        }
        op_eo = eb.op_create(U, W["kappa"], dims, bc_t=-1, defl_capacity=W["n1"] * W["nev"], eo=True)
        run_step(eb, op_eo, B, X, W, [], [])
        lat_e, its_e = [], []
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        run_step(eb, op_eo, B, X, W, lat_e, its_e)
        torch.cuda.synchronize()
        dt_e = time.perf_counter() - t1
        eo_tune = tune_untimed(eb, op_eo, ("fp64", "fp32", "bf16"))
        eo_defl = {}
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
        res["even_odd"] = {"solves_per_s": round(W["nrhs"] / dt_e, 3), "ms_per_step": round(1e3 * dt_e, 3),
                           "iters_per_rhs": its_e, "p50_ms": round(1e3 * percentile(lat_e, 50), 3),
                           "deflated_solves_per_s": eo_defl, "autotune_seconds": eo_tune}
    eb.defl_reset(op)
    plain = []
    for i in range(W["n1"], min(W["nrhs"], W["n1"] + 4)):
        X[i].zero_()
        plain.append(eb.deflated_bicg_solve(op, B[i], X[i], tol=W["tol"], maxiter=20000)["iters"])
    res["undeflated_bicgstab_iters"] = plain
    eb.op_destroy(op)
    del B, X
    torch.cuda.empty_cache()
    log(f"[bench] incremental 16^3x32 side record: {res['solves_per_s']} solves/s")
    return res


# ---------------------------------------------------------------------------
# The headline: 32^3 x 64 batched, mixed-precision, deflated solves
# ---------------------------------------------------------------------------
# Algorithmic bytes of the batched BiCGStab kernels, per site: complex entries
# per column (12 per spinor read or written once) and per launch (the 36 link
# entries, read once for all columns by the two stencils).
BATCH_COL_SPINORS = {"bstab_v": 3, "bstab_s": 3, "bstab_t": 2, "bstab_xr": 7, "bstab_p": 4}
BATCH_STENCILS = ("bstab_v", "bstab_t")
CPLX_BYTES = {"fp64": 16, "fp32": 8, "bf16": 4}


def batch_roofline(ktable, col_iters, k, V, prec):
    """Achieved algorithmic GB/s of each batched kernel class over the timed steps.

    A launch of class c moves 12 * BATCH_COL_SPINORS[c] complex entries per site
    for each column still iterating (stopped columns are skipped), plus the
    36 link entries per site for the stencils.  col_iters (the columns'
    iterations summed) counts the column passes of every class; the stencils'
    working launches are at least col_iters / k, and the link bytes are
    counted for that many (the launches queued past the last column's stop
    return at once).  Returns {class: record}."""
    cb = CPLX_BYTES[prec]
    n_work = -(-col_iters // k)
    out = {}
    for c, ncol in BATCH_COL_SPINORS.items():
        n, ms = ktable.get(c, (0, 0.0))
        if not n or not ms:
            continue
        total = col_iters * V * 12 * ncol * cb + (n_work * V * 36 * cb if c in BATCH_STENCILS else 0)
        out[c] = {"launches": n, "working_launches": n_work, "total_ms": round(ms, 3),
                  "bytes_per_launch": round(total / n_work), "avg_launch_us": round(1e3 * ms / n_work, 2),
                  "avg_us_all_launches": round(1e3 * ms / n, 2),
                  "achieved_GBps": round(total / (ms * 1e-3) / 1e9, 1)}
    return out


_CPU = {}


def _oracle_d_once(i):
    """Worker: one application of the oracle's D to source i (links inherited from the parent)."""
    import synth
    from oracle import wilson as Wl

    try:
        from threadpoolctl import threadpool_limits

        threadpool_limits(1)
    except Exception:  # pragma: no cover
        pass
    dims, kappa, U = _CPU["dims"], _CPU["kappa"], _CPU["U"]
    V = synth.volume(dims)
    b = synth.z2_source(V, synth.rhs_seed(3, i))
    t0 = time.perf_counter()
    Wl.apply_D(U, b, kappa, dims)
    return time.perf_counter() - t0


def oracle_dslash_parallel(U, dims, kappa):
    """One application of the oracle's D per host core in forked worker processes (before
    this process touches the GPU); returns (mean seconds, workers)."""
    import multiprocessing as mp

    try:
        ncpu = len(os.sched_getaffinity(0))
    except Exception:  # pragma: no cover
        ncpu = os.cpu_count() or 1
    nproc = max(1, min(16, ncpu))
    _CPU.update(dims=dims, kappa=kappa, U=U)
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(nproc) as pool:
        times = pool.map(_oracle_d_once, range(nproc))
    _CPU.clear()
    return sum(times) / len(times), nproc, time.perf_counter() - t0


def headline_batch(eb, W, U, args):
    """The workload of the bench line: 32^3 x 64, a 100-pair deflation space grown
    by eigBiCG (setup), then each step solves the 16 resident Z2 sources by
    deflated BiCGStab in batches (multi-RHS stencil, k and tile form chosen by
    the library's autotuner during setup), complex64 inner iterations inside
    complex128 refinement, every solve to ||b - A x|| <= 1e-10 ||b|| in FP64."""
    import torch

    import synth

    dims = W["dims"]
    V = synth.volume(dims)
    dev = torch.device("cuda:0")
    setup = {}
    op = eb.op_create(U, W["kappa"], dims, bc_t=-1, defl_capacity=W["n1"] * W["nev"])
    t0 = time.perf_counter()
    grow = []
    for i in range(W["n1"]):
        b = torch.from_numpy(synth.z2_source(V, synth.rhs_seed(W["cfg"], 100 + i))).to(dev)
        x = torch.zeros_like(b)
        st, _ = eb.eigbicg_solve(op, b, x, W["nev"], W["m"], W["tol"], maxiter=20000)
        assert st["true_rel_resid"] <= W["tol"], st
        grow.append({"iters": st["iters"], "restarts": st["window_restarts"], "seconds": round(st["seconds"], 3)})
        log(f"[bench] growth eigBiCG {i}: {grow[-1]}")
        del b, x
    setup["eigbicg_growth"] = {"nev": W["nev"], "m": W["m"], "solves": grow, "K": eb.defl_info(op)[0],
                               "seconds": round(time.perf_counter() - t0, 3)}
    setup["device_bytes_after_growth"] = eb.op_device_bytes(op)
    eb.op_trim(op)  # the eigBiCG windows and absorb buffers
    setup["device_bytes_trimmed"] = eb.op_device_bytes(op)
    # (FP64 too: its k = 1 entry is the stencil form of the one-at-a-time FP64 comparator)
    setup["autotune_seconds"] = tune_untimed(eb, op, (W["inner"], "bf16", "fp64"))
    tune = {p: eb.op_batch_tune(op, p) for p in (W["inner"], "bf16")}
    setup["autotune"] = tune
    k = tune[W["inner"]]["k"]
    log(f"[bench] autotuner: k = {k}, forms {tune[W['inner']]['stage']}")
    nrhs = W["nrhs"]
    B = torch.stack([torch.from_numpy(synth.z2_source(V, synth.rhs_seed(W["cfg"], i))) for i in range(nrhs)]).to(dev)
    X = torch.zeros_like(B)

    def step():
        X.zero_()
        st = eb.deflated_bicg_solve(op, B, X, tol=W["tol"], maxiter=20000, nrhs=nrhs, inner=W["inner"],
                                    inner_tol=W["inner_tol"], batch=0)
        if st["true_rel_resid"] > W["tol"]:
            raise RuntimeError(f"a solve missed the tolerance: {st}")
        return st

    for w in range(args.warmup):
        step()
        log(f"[bench] warmup step {w} done")
    timing = not args.no_timing
    if timing:
        eb.timing_classes(op, None)
        eb.timing_enable(op, True)
    lat, sts = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        t1 = time.perf_counter()
        sts.append(step())
        lat.append(time.perf_counter() - t1)
        log(f"[bench] step {i}: {lat[-1]:.3f} s, {sts[-1]['iters'] / nrhs:.1f} iterations per source")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ktable = eb.timing_read(op) if timing else {}
    eb.timing_enable(op, False)
    col_iters = sum(s["iters"] for s in sts)
    kern = batch_roofline(ktable, col_iters, k, V, W["inner"])
    others = {n: {"launches": c, "total_ms": round(ms, 3)} for n, (c, ms) in ktable.items()
              if c and n not in kern}
    total_ms = sum(ms for _, ms in ktable.values())
    dom = max(kern, key=lambda c: kern[c]["total_ms"]) if kern else None
    roof = None
    if dom:
        rk = kern[dom]
        roof = {"kernel": dom, "bound": "hbm", "achieved": rk["achieved_GBps"], "peak": HBM_PEAK_GBPS,
                "unit": "GB/s", "frac": round(rk["achieved_GBps"] / HBM_PEAK_GBPS, 4),
                "traffic": measured_traffic("batch32x64", dom, k),
                "bytes_per_launch": rk["bytes_per_launch"], "avg_launch_us": rk["avg_launch_us"],
                "launches": rk["launches"], "working_launches": rk["working_launches"],
                "share_of_kernel_time": round(rk["total_ms"] / total_ms, 4) if total_ms else None}
    value = nrhs * args.steps / elapsed
    st0 = sts[0]
    head = {"value": value, "elapsed": elapsed, "lat": lat, "k": k, "roofline": roof,
            "kernels": {"batched": kern, "other": others},
            "iters_per_rhs": round(st0["iters"] / nrhs, 1), "outer_steps": st0["outer_steps"],
            "max_true_rel_resid": max(s["true_rel_resid"] for s in sts),
            "matvec_d_per_rhs": round(st0["matvec_d"] / nrhs, 1), "setup": setup}
    # the same sources on the same GPU: FP64 deflated BiCGStab, plain (undeflated)
    # FP64 BiCG and BiCGStab, BF16-stored inner, one at a time / batched
    comp = {"mixed_fp32_batched_deflated": {"solves_per_s": round(value, 3), "k": k,
                                            "iters_per_rhs": head["iters_per_rhs"]}}
    nc = 4

    def run(name, o, n, **kw):
        Xc = torch.zeros_like(B[:n])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st = eb.deflated_bicg_solve(o, B[:n].contiguous(), Xc, tol=W["tol"], maxiter=20000, nrhs=n, **kw)
        dt = time.perf_counter() - t1
        assert st["true_rel_resid"] <= W["tol"], (name, st)
        comp[name] = {"solves_per_s": round(n / dt, 3), "iters_per_rhs": round(st["iters"] / n, 1),
                      "max_true_rel_resid": st["true_rel_resid"]}
        log(f"[bench] {name}: {comp[name]}")
        del Xc

    run("mixed_bf16_batched_deflated", op, nrhs, inner="bf16", inner_tol=1e-2, batch=0)
    run("fp64_bicgstab_deflated", op, nc, batch=1)
    eb.op_trim(op)  # the batch buffers (reallocated on use): room for an FP64 window at this size
    op2 = eb.op_create(U, W["kappa"], dims, bc_t=-1, defl_capacity=0)  # no deflation space
    tune_untimed(eb, op2, (W["inner"], "fp64"))  # as for op: the tuning is setup, not part of a solve
    # eigBiCG at this size with the FP64 window and host restarts against the device
    # restart and the FP32 window (no space to absorb into: the solves alone)
    head["eigbicg_modes"] = None
    if not args.no_side:  # (a profiled run of the headline leaves them out)
        gsrc = [torch.from_numpy(synth.z2_source(V, synth.rhs_seed(W["cfg"], 100))).to(dev)]
        head["eigbicg_modes"] = eigbicg_modes(eb, op2, gsrc, W, 1)
        log(f"[bench] eigBiCG modes {dims}: {head['eigbicg_modes']}")
        eb.op_trim(op2)
        del gsrc
    run("fp64_bicg_plain", op2, nc, method=1)
    run("fp64_bicgstab_plain", op2, nc, batch=1)
    run("mixed_fp32_batched_plain", op2, nrhs, inner=W["inner"], inner_tol=W["inner_tol"], batch=0)
    eb.op_destroy(op2)
    head["comparators"] = comp
    head["speedup_vs_fp64_bicg_plain"] = round(value / comp["fp64_bicg_plain"]["solves_per_s"], 3)
    head["speedup_vs_fp64_bicgstab_deflated"] = round(value / comp["fp64_bicgstab_deflated"]["solves_per_s"], 3)
    head["fp64_bicgstab_iters_per_rhs"] = comp["fp64_bicgstab_deflated"]["iters_per_rhs"]
    head["multi_rhs_stencil"] = multi_rhs_stencil(eb, op, V, precs=("fp32", "bf16"), ks=(1, 4, 8, 16))
    eb.op_destroy(op)
    del B, X
    torch.cuda.empty_cache()
    return head


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="batch32x64", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-timing", action="store_true", help="do not record per-kernel HIP events")
    ap.add_argument("--no-large", action="store_true", help="skip the 24^3 x 64 precision section")
    ap.add_argument("--no-side", action="store_true", help="the headline workload only (e.g. to profile it)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving (continuous batching) section")
    ap.add_argument("--serving-only", action="store_true", help="run only the serving section and print it")
    ap.add_argument("--proj-pass", action="store_true", help="deflation projections on the matrix cores, for --pmc")
    ap.add_argument("--stencil-pass", action="store_true", help="multi-RHS FP32 stencil launches for rocprofv3 --pmc")
    ap.add_argument("--stencil-form", type=int, default=0, help="tile form of the k > 1 launches of --stencil-pass")
    ap.add_argument("--pmc-pass", action="store_true",
                    help="one pass of the workload's roofline kernel and a calibration copy, for rocprofv3 --pmc")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/pmc_<kernel>_<workload>.json from two counter runs")
    ap.add_argument("--eigbicg-pass", choices=("host", "device", "fp32"),
                    help="two eigBiCG solves between marker launches, for rocprofv3 --kernel-trace")
    ap.add_argument("--eigbicg-workload", default="inc16x32", choices=sorted(WORKLOADS),
                    help="lattice, nev and m of --eigbicg-pass and --summarize-gap")
    ap.add_argument("--summarize-gap", nargs=4, metavar=("HOST_TRACE_DIR", "DEVICE_TRACE_DIR", "NAME", "COMMAND"),
                    help="write profiles/NAME.md from the kernel traces of --eigbicg-pass host / device")
    ap.add_argument("--summarize-trace", nargs=4, metavar=("PROF_DIR", "BENCH_JSON", "NAME", "COMMAND"),
                    help="write profiles/NAME.md from a rocprofv3 --kernel-trace --stats run of bench.py")
    args = ap.parse_args()
    if args.summarize_trace:
        d, bj, name, cmd = args.summarize_trace
        summarize_trace(d, bj, args.workload, name, cmd)
        return
    if args.summarize_pmc:
        if args.workload == "batch32x64":  # the two passes that take the most time
            for kern, cls in (("k_bstab_v", "bstab_v"), ("k_bstab_xr", "bstab_xr")):
                summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1], args.workload, kernel=kern, cls=cls)
        else:
            summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1], args.workload)
            summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1], args.workload, kernel="k_bmarch",
                          cls="dslash1_march")
        return
    if args.summarize_gap:
        h, d, name, cmd = args.summarize_gap
        summarize_gap([("host", h), ("device", d)], name, cmd, args.eigbicg_workload)
        return
    if args.pmc_pass:
        pmc_pass(args.workload)
        return
    if args.eigbicg_pass:
        from paper_0911_2285_amd import ebicg as eb

        eigbicg_pass(eb, args.eigbicg_pass, args.eigbicg_workload)
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
    W = WORKLOADS[args.workload]
    if "inner" not in W:
        print("the bench line runs the batch32x64 workload; the incremental workloads are side records",
              file=sys.stderr)
        sys.exit(2)

    import synth

    dims = W["dims"]
    log(f"[bench] workload {args.workload}: dims={dims} kappa={W['kappa']} nrhs={W['nrhs']}")
    t0 = time.perf_counter()
    U = synth.random_su3_links(dims, 0.3, synth.gauge_seed(W["cfg"]))
    log(f"[bench] links generated in {time.perf_counter() - t0:.1f} s")
    # the CPU oracle leg runs first, in forked workers, before this process touches the GPU
    cpu_d = None
    if not args.no_cpu_baseline and not args.serving_only:
        log("[bench] timing the CPU oracle (one D application per host core) ...")
        cpu_d = oracle_dslash_parallel(U, dims, W["kappa"])
        log(f"[bench] oracle D: {cpu_d[0]:.2f} s per application, {cpu_d[1]} workers")

    import torch

    from paper_0911_2285_amd import ebicg as eb

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.serving_only:
        print(json.dumps({"serving": serving(eb)}), flush=True)
        return
    head = headline_batch(eb, W, U, args)
    del U
    V = synth.volume(dims)
    extra = {}
    if not args.no_side:
        extra["incremental_16x32"] = incremental_side(eb, WORKLOADS["inc16x32"], max(1, min(args.steps, 2)), 1)
        if not args.no_serving:
            extra["serving"] = serving(eb)
        extra["deflation_sweep"] = deflation_sweep(eb)
        extra["table1_analogue"] = table1_analogue(eb)
        if not args.no_large:
            extra["large_lattice"] = large_lattice(eb, (24, 24, 24, 64), 0.123, 16, W["tol"])

    cpu = None
    if cpu_d:
        t_d, nproc, wall = cpu_d
        # the oracle's deflated FP64 BiCGStab solve: 2 D per iteration at the GPU's FP64
        # iteration count, plus the initial and final residuals
        d_per_solve = 2 * head["fp64_bicgstab_iters_per_rhs"] + 2
        cpu = {"value": round(nproc / (t_d * d_per_solve), 6), "unit": "solves/s", "cores": nproc, "kind": "oracle",
               "sample": (f"one application of the oracle's D on the {'x'.join(map(str, dims))} lattice in each of "
                          f"{nproc} forked worker processes, one per host core (1 thread each; {t_d:.2f} s per "
                          f"application, {wall:.1f} s wall); a deflated FP64 BiCGStab solve of the oracle is costed "
                          f"at {d_per_solve:.0f} D applications (2 per iteration at the GPU's FP64 iteration count "
                          f"plus two residuals), its vector operations and deflation projections not counted, so "
                          f"this is an upper bound on the oracle's rate"),
               "dslash_seconds": round(t_d, 3), "dslash_GBps_per_core": round(960 * V / t_d / 1e9, 3)}

    lat = head["lat"]
    out = {
        "metric": "solves/s at 1e-10 rel. resid (mixed vs FP64), dslash HBM GB/s, p50/p99",
        "value": round(head["value"], 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * head["elapsed"] / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 inner / c128 outer",
        "data": "synthetic",
        "config": {
            "workload": (f"batched mixed-precision deflated solves, Wilson-Dirac {'x'.join(map(str, dims))}, "
                         f"kappa {W['kappa']}, eps 0.3 SU(3) links, {W['nrhs']} Z2 sources per step, "
                         f"{W['n1'] * W['nev']}-pair deflation space grown by {W['n1']} eigBiCG solves "
                         f"(nev {W['nev']}, m {W['m']}) in setup, multi-RHS BiCGStab with autotuned k "
                         f"({head['k']}) and tile form, complex64 inner / complex128 refinement, tol {W['tol']}"),
            "lattice": list(dims),
            "nrhs": W["nrhs"],
            "k": head["k"],
            "deflation_pairs": W["n1"] * W["nev"],
            "parallelism": "single GPU",
        },
        "roofline": head["roofline"],
        "cpu_baseline": cpu,
        # the batched solve's dslash: the v stencil pass (D on k columns with its dots)
        "dslash_GBps": head["kernels"]["batched"].get("bstab_v", {}).get("achieved_GBps"),
        "p50_ms": round(1e3 * percentile(lat, 50), 3),
        "p99_ms": round(1e3 * percentile(lat, 99), 3),
        "latency_note": "p50/p99 of the step (16 solves in one batched call, all finishing together); per-request "
                        "latency under continuous batching is in serving",
        "iters_per_rhs": head["iters_per_rhs"],
        "outer_steps": head["outer_steps"],
        "max_true_rel_resid": head["max_true_rel_resid"],
        "comparators": head["comparators"],
        "speedup_vs_fp64_bicg_plain": head["speedup_vs_fp64_bicg_plain"],
        "speedup_vs_fp64_bicgstab_deflated": head["speedup_vs_fp64_bicgstab_deflated"],
        "kernels": head["kernels"],
        "setup": head["setup"],
        "multi_rhs_stencil": head["multi_rhs_stencil"],
        "eigbicg_modes": head["eigbicg_modes"],
        **extra,
    }
    print(json.dumps(out), flush=True)

if __name__ == "__main__":
    main()
