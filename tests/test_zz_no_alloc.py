"""The allocation-free entry point eb_op_apply_noalloc against eb_op_apply (FP64).

Both run the same kernels, so their outputs agree bit for bit; the
allocation-free call must not grow the operator's device buffers, must keep
working when the next call is on a smaller lattice (the shared staging array
keeps the previous call's contents), and must refuse a lattice beyond its
staging array.
"""
import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _apply_noalloc(eb, op, out, inp, dagger):
    rc = eb.lib().eb_op_apply_noalloc(op.handle, ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(inp.data_ptr()),
                                      int(dagger), eb._stream(None))
    return rc


def test_noalloc_apply_matches_apply_on_two_calls(gpu_lib):
    import torch

    eb = gpu_lib
    for dims, seed in (((8, 8, 8, 8), 11), ((4, 4, 4, 6), 12)):  # the second call on a smaller input
        V = synth.volume(dims)
        U = synth.random_su3_links(dims, 0.3, synth.gauge_seed(seed))
        op = eb.op_create(U, 0.12, dims)
        psi = torch.from_numpy(synth.gaussian_spinor(V, seed)).to("cuda:0")
        for dagger in (0, 1):
            y0 = torch.full_like(psi, float("nan"))
            before = eb.op_device_bytes(op)
            assert _apply_noalloc(eb, op, y0, psi, dagger) == 0, eb._last_error()
            torch.cuda.synchronize()
            assert eb.op_device_bytes(op) == before  # nothing allocated for this operator
            y1 = torch.empty_like(psi)
            (eb.op_apply_dagger if dagger else eb.op_apply)(op, y1, psi)
            torch.cuda.synchronize()
            assert torch.isfinite(y0).all()
            assert torch.equal(y0, y1), f"{dims} dagger={dagger}: max diff {(y0 - y1).abs().max().item()}"
        eb.op_destroy(op)


def test_noalloc_apply_rejects_too_large_lattice(gpu_lib):
    import torch

    eb = gpu_lib
    dims = (16, 16, 16, 34)  # 139264 sites > 131072
    V = synth.volume(dims)
    op = eb.op_create(synth.unit_links(dims), 0.12, dims)
    x = torch.zeros(V, 4, 3, dtype=torch.complex128, device="cuda:0")
    y = torch.zeros_like(x)
    rc = _apply_noalloc(eb, op, y, x, 0)
    assert rc == -1 and "too large" in eb._last_error()
    eb.op_destroy(op)
