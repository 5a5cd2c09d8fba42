"""Write the oracle's first eigBiCG solve of the 16^3 x 32 incremental workload.

Alg. eigBiCG with Alg. BiCG-eigen (Sec. 2) on the Wilson-Dirac operator,
16^3 x 32 lattice, kappa = 0.122, eps = 0.3 links (gauge seed 1001), the
first Z2 source of operator 0, x0 = 0, nev = 10, m = 40, tol = 1e-10.  The
run takes several CPU minutes, so the GPU parity test reads its result from
tests/golden/cfg1_eigbicg_16x16x16x32.json instead of repeating it.

Only the oracle and the seeded input generators are called here.

    python tests/golden/make_cfg1_eigbicg.py
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import krylov as K  # noqa: E402
from oracle import wilson as W  # noqa: E402

DIMS, KAPPA, EPS = (16, 16, 16, 32), 0.122, 0.3
NEV, M, TOL = 10, 40, 1e-10
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cfg1_eigbicg_16x16x16x32.json")
N_SAMPLES = 96


def main():
    t0 = time.time()
    V = synth.volume(DIMS)
    U = synth.random_su3_links(DIMS, EPS, synth.gauge_seed(1))
    A = lambda v: W.apply_D(U, v.reshape(V, 4, 3), KAPPA, DIMS).ravel()
    Ad = lambda v: W.apply_Ddag(U, v.reshape(V, 4, 3), KAPPA, DIMS).ravel()
    b = synth.z2_source(V, synth.rhs_seed(0, 0)).ravel()
    res = K.eigbicg(A, Ad, b, np.zeros_like(b), NEV, M, TOL)
    x = res.x
    true_rel = float(np.linalg.norm(b - A(x)) / np.linalg.norm(b))
    # Ritz residuals of the returned pairs: ||A u - theta u|| / ||u|| and
    # ||A^+ q - conj(theta) q|| / ||q||
    right, left = [], []
    for i, th in enumerate(res.lam):
        u, q = res.U[:, i], res.Q[:, i]
        right.append(float(np.linalg.norm(A(u) - th * u) / np.linalg.norm(u)))
        left.append(float(np.linalg.norm(Ad(q) - np.conj(th) * q) / np.linalg.norm(q)))
    rng = np.random.default_rng(12345)
    idx = np.sort(rng.choice(x.size, N_SAMPLES, replace=False))
    out = {
        "what": "oracle eigBiCG (Alg. eigBiCG with Alg. BiCG-eigen), first solve of the 16^3x32 incremental workload",
        "dims": list(DIMS), "kappa": KAPPA, "eps": EPS, "gauge_seed": synth.gauge_seed(1),
        "rhs_seed": synth.rhs_seed(0, 0), "nev": NEV, "m": M, "tol": TOL, "bc_t": -1,
        "iters": int(res.iters), "restarts": len(res.restarts), "converged": bool(res.converged),
        "true_rel_resid": true_rel,
        "ritz": [[float(z.real), float(z.imag)] for z in res.lam],
        "ritz_res_right": right, "ritz_res_left": left,
        "x_norm": float(np.linalg.norm(x)),
        "x_sample_index": [int(i) for i in idx],
        "x_sample": [[float(x[i].real), float(x[i].imag)] for i in idx],
        "cpu_seconds": round(time.time() - t0, 1),
    }
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {OUT}: {res.iters} iterations, {len(res.restarts)} restarts, true residual {true_rel:.2e}, "
          f"{out['cpu_seconds']} s")


if __name__ == "__main__":
    main()
