"""Write the oracle's runs of the Table 1 analogue on 12^4.

Table 1 of the paper compares the lowest Ritz values of eigBiCG with a
limited window against those of BiCG that keeps every residual.  The
analogue here: Alg. eigBiCG with Alg. BiCG-eigen (Sec. 2) on the
Wilson-Dirac operator, 12^4 lattice, kappa = 0.2, eps = 1.0 links (seed
123), antiperiodic in t, the first Z2 source of operator 0, x0 = 0, nev = 5,
tol = 1e-8, windows m = 126 (larger than the iteration count: no restart),
40 and 20.  For each run: iterations, restarts, the nev returned Ritz values
and their right / left Ritz residuals, and the solution at sampled entries.
The three runs take about a CPU minute; the GPU test reads them from
tests/golden/table1_12x12x12x12.json.

Only the oracle and the seeded input generators are called here.

    python tests/golden/make_table1_12x4.py
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

DIMS, KAPPA, EPS, GAUGE_SEED = (12, 12, 12, 12), 0.2, 1.0, 123
NEV, TOL, WINDOWS = 5, 1e-8, (126, 40, 20)
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "table1_12x12x12x12.json")
N_SAMPLES = 64


def main():
    t0 = time.time()
    V = synth.volume(DIMS)
    U = synth.random_su3_links(DIMS, EPS, GAUGE_SEED)
    A = lambda v: W.apply_D(U, v.reshape(V, 4, 3), KAPPA, DIMS).ravel()
    Ad = lambda v: W.apply_Ddag(U, v.reshape(V, 4, 3), KAPPA, DIMS).ravel()
    b = synth.z2_source(V, synth.rhs_seed(0, 0)).ravel()
    rng = np.random.default_rng(4321)
    idx = np.sort(rng.choice(b.size, N_SAMPLES, replace=False))
    runs = {}
    for m in WINDOWS:
        res = K.eigbicg(A, Ad, b, np.zeros_like(b), NEV, m, TOL)
        x = res.x
        right = [float(np.linalg.norm(A(res.U[:, i]) - th * res.U[:, i]) / np.linalg.norm(res.U[:, i]))
                 for i, th in enumerate(res.lam)]
        left = [float(np.linalg.norm(Ad(res.Q[:, i]) - np.conj(th) * res.Q[:, i]) / np.linalg.norm(res.Q[:, i]))
                for i, th in enumerate(res.lam)]
        runs[str(m)] = {
            "iters": int(res.iters), "restarts": len(res.restarts), "converged": bool(res.converged),
            "true_rel_resid": float(np.linalg.norm(b - A(x)) / np.linalg.norm(b)),
            "ritz": [[float(z.real), float(z.imag)] for z in res.lam],
            "ritz_res_right": right, "ritz_res_left": left,
            "x_sample": [[float(z.real), float(z.imag)] for z in x[idx]],
        }
        print(f"m {m}: {res.iters} iterations, {len(res.restarts)} restarts, "
              f"{time.time() - t0:.0f} s", flush=True)
    out = {
        "what": "oracle eigBiCG on 12^4 (the Table 1 analogue): windows 126 (no restart), 40, 20",
        "dims": list(DIMS), "kappa": KAPPA, "eps": EPS, "gauge_seed": GAUGE_SEED, "bc_t": -1,
        "rhs_seed": synth.rhs_seed(0, 0), "nev": NEV, "tol": TOL,
        "x_sample_index": [int(i) for i in idx], "runs": runs,
        "generator": "tests/golden/make_table1_12x4.py (oracle only)",
    }
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", OUT, f"in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
