"""FP64 CPU oracle for incremental eigBiCG -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import anything from this package.  The product path (the
HIP library and its Python binding) never calls it and shares no code with
it; the two meet only at the seeded inputs of ``synth``.

Everything here is plain NumPy/SciPy in complex128, written for a reader who
checks it against the paper by eye:

* ``wilson``   -- the Wilson-Dirac operator D, its adjoint, gamma matrices and
                  a dense builder (the operator of the paper's tests, Sec. 3).
* ``eig``      -- eig(C) with left/right vectors and the sort criterion of the
                  paper's conventions (Sec. 1, end).
* ``krylov``   -- BiCG / eigBiCG (Alg. eigBiCG), the window restart
                  (Alg. BiCG-eigen), the incremental driver (Alg. Incremental
                  eigBiCG), deflated BiCGStab with the DefTol restart (Sec. 2,
                  text after the listings), and the final Rayleigh-Ritz.

Parity status: every function is pinned by ``tests/test_oracle_*.py``
(closed forms, invariants, dense LAPACK, textbook reductions).  The paper's
Table 1 values and Fig. 1 speed-up need gauge configurations that are not
available; they are context only ("parity unpinned" for those numbers, not
for any function).
"""
