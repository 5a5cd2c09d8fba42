"""The BiCG matvec pair (D p with the partials of (phat, D p), and D^+ phat; the
products of every iteration of Alg. eigBiCG and of plain BiCG) in its
t-marching form (eb_op_set_matvec_form(op, 6): the D and D^+ units of one box
and chunk of time slices on one XCD together) against the oracle and against
the LDS-staged form (1):

* 8^4 (boxes of 8 x 8 x 8 sites): eigBiCG (nev 5, m 24) in both forms against
  the oracle's run (iterations +-1, restart count, true residual in the
  oracle's D, the nev - 2 Ritz values of smallest modulus to 1e-8 relative)
  and the two forms against each other (solutions to 1e-9); the
  gamma5-Hermitian form (rhat = 2, D units only, sigma from gamma5 p);
  deflated BiCG (method 1) against the oracle's bicg (iterations +-1,
  solution to 1e-8);
* 16^3 x 32, the first eigBiCG solve of the incremental workload in the
  t-marching form against the oracle's stored run
  (tests/golden/cfg1_eigbicg_16x16x16x32.json), as the staged form is in
  test_gpu_fullsize.py;
* the knob's error paths (values other than -1, 1, 6; the even-odd operator).
"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import krylov as K
from oracle import wilson as W

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _ops(U, kappa, dims):
    V = synth.volume(dims)
    A = lambda v: W.apply_D(U, v.reshape(V, 4, 3), kappa, dims).ravel()
    Ad = lambda v: W.apply_Ddag(U, v.reshape(V, 4, 3), kappa, dims).ravel()
    return A, Ad


def _rel_match(a, b):
    return max(np.min(np.abs(np.asarray(b) - v)) / abs(v) for v in a)


def _smallest(lam, p):
    return sorted(np.asarray(lam), key=abs)[:p]


@pytest.fixture(scope="module")
def lat8():
    dims, kappa = (8, 8, 8, 8), 0.12
    U = synth.random_su3_links(dims, 0.3, synth.gauge_seed(5))
    return dims, kappa, U


def test_eigbicg_matvec_forms_match_oracle(gpu_lib, lat8):
    import torch

    dims, kappa, U = lat8
    V = synth.volume(dims)
    A, Ad = _ops(U, kappa, dims)
    b_np = synth.z2_source(V, synth.rhs_seed(5, 3))
    orc = K.eigbicg(A, Ad, b_np.ravel(), np.zeros(12 * V, complex), 5, 24, 1e-10)
    xs = {}
    for form in (6, 1):
        op = gpu_lib.op_create(U, kappa, dims, defl_capacity=5)
        gpu_lib.op_set_matvec_form(op, form)
        b = torch.from_numpy(b_np).to("cuda:0")
        x = torch.zeros_like(b)
        st, ritz = gpu_lib.eigbicg_solve(op, b, x, nev=5, m=24, tol=1e-10)
        assert gpu_lib.op_get_matvec_form(op)[0] == form
        gpu_lib.op_destroy(op)
        xs[form] = x.cpu().numpy().ravel()
        tr = np.linalg.norm(b_np.ravel() - A(xs[form])) / np.linalg.norm(b_np)
        err = _rel_match(_smallest(orc.lam, 3), ritz)
        print(f"8^4 eigBiCG matvec form {form}: {st['iters']} it ({orc.iters}), {st['window_restarts']} restarts "
              f"({len(orc.restarts)}), residual {tr:.1e}, 3 smallest Ritz values vs oracle {err:.1e}", flush=True)
        assert abs(st["iters"] - orc.iters) <= 1 and st["window_restarts"] == len(orc.restarts)
        assert tr <= 1e-10 and err < 1e-8
    d = np.linalg.norm(xs[6] - xs[1]) / np.linalg.norm(xs[1])
    print(f"  solutions of the two forms differ by {d:.1e}")
    assert d < 1e-9


def test_eigbicg_gamma5_form_march_matvec(gpu_lib, lat8):
    """rhat = 2: gamma5 p is the left vector; sigma from the input at the site."""
    import torch

    dims, kappa, U = lat8
    V = synth.volume(dims)
    A, Ad = _ops(U, kappa, dims)
    b_np = synth.gaussian_spinor(V, 31)
    orc = K.eigbicg(A, Ad, b_np.ravel(), np.zeros(12 * V, complex), 5, 24, 1e-10,
                    rhat0=W.apply_gamma5(b_np.reshape(V, 4, 3)).ravel())
    op = gpu_lib.op_create(U, kappa, dims, defl_capacity=5)
    gpu_lib.op_set_matvec_form(op, 6)
    b = torch.from_numpy(b_np).to("cuda:0")
    x = torch.zeros_like(b)
    st, ritz = gpu_lib.eigbicg_solve(op, b, x, nev=5, m=24, tol=1e-10, rhat=2)
    gpu_lib.op_destroy(op)
    tr = np.linalg.norm(b_np.ravel() - A(x.cpu().numpy().ravel())) / np.linalg.norm(b_np)
    print(f"8^4 gamma5 form, matvec form 6: {st['iters']} it ({orc.iters}), residual {tr:.1e}")
    assert abs(st["iters"] - orc.iters) <= 1 and tr <= 1e-10


def test_bicg_march_matvec_matches_oracle(gpu_lib, lat8):
    import torch

    dims, kappa, U = lat8
    V = synth.volume(dims)
    A, Ad = _ops(U, kappa, dims)
    b_np = synth.z2_source(V, synth.rhs_seed(5, 4))
    xo, its, _ = K.bicg(A, Ad, b_np.ravel(), np.zeros(12 * V, complex), 1e-10)
    op = gpu_lib.op_create(U, kappa, dims)
    gpu_lib.op_set_matvec_form(op, 6)
    b = torch.from_numpy(b_np).to("cuda:0")
    x = torch.zeros_like(b)
    st = gpu_lib.deflated_bicg_solve(op, b, x, tol=1e-10, method=1)
    gpu_lib.op_destroy(op)
    xg = x.cpu().numpy().ravel()
    err = np.linalg.norm(xg - xo) / np.linalg.norm(xo)
    print(f"8^4 BiCG, matvec form 6: {st['iters']} it ({its}), solution vs oracle {err:.1e}")
    assert abs(st["iters"] - its) <= 1 and err < 1e-8


def test_eigbicg_16x32_march_matvec_matches_oracle(gpu_lib):
    import torch

    with open(os.path.join(GOLDEN, "cfg1_eigbicg_16x16x16x32.json")) as f:
        g = json.load(f)
    dims, kappa = tuple(g["dims"]), g["kappa"]
    V = synth.volume(dims)
    U = synth.random_su3_links(dims, g["eps"], g["gauge_seed"])
    b_np = synth.z2_source(V, g["rhs_seed"])
    op = gpu_lib.op_create(U, kappa, dims, bc_t=g["bc_t"], defl_capacity=g["nev"])
    gpu_lib.op_set_matvec_form(op, 6)
    b = torch.from_numpy(b_np).to("cuda:0")
    x = torch.zeros_like(b)
    st, ritz = gpu_lib.eigbicg_solve(op, b, x, nev=g["nev"], m=g["m"], tol=g["tol"])
    gpu_lib.op_destroy(op)
    A, _ = _ops(U, kappa, dims)
    xg = x.cpu().numpy().ravel()
    tr = np.linalg.norm(b_np.ravel() - A(xg)) / np.linalg.norm(b_np)
    idx = np.asarray(g["x_sample_index"])
    xs = np.asarray(g["x_sample"]) @ np.array([1, 1j])
    err = np.linalg.norm(xg[idx] - xs) / np.linalg.norm(xs)
    lam = np.asarray(g["ritz"]) @ np.array([1, 1j])
    print(f"16^3x32 eigBiCG, matvec form 6: {st['iters']} it ({g['iters']}), {st['window_restarts']} restarts "
          f"({g['restarts']}), residual {tr:.1e}, solution at samples {err:.1e}, Ritz {_rel_match(lam, ritz):.1e}")
    assert abs(st["iters"] - g["iters"]) <= 1 and st["window_restarts"] == g["restarts"]
    assert tr <= 1e-10 and err < 1e-8
    assert _rel_match(lam, ritz) < 1e-6 and _rel_match(ritz, lam) < 1e-6


def test_matvec_form_errors(gpu_lib, lat8):
    dims, kappa, U = lat8
    op = gpu_lib.op_create(U, kappa, dims)
    for bad in (0, 2, 7, -2):
        with pytest.raises(RuntimeError):
            gpu_lib.op_set_matvec_form(op, bad)
    gpu_lib.op_set_matvec_form(op, -1)
    assert gpu_lib.op_get_matvec_form(op)[0] == -1
    gpu_lib.op_destroy(op)
    eo = gpu_lib.op_create(U, kappa, dims, eo=True)
    with pytest.raises(RuntimeError):
        gpu_lib.op_set_matvec_form(eo, 6)
    assert gpu_lib.op_get_matvec_form(eo)[0] == 1
    gpu_lib.op_destroy(eo)
