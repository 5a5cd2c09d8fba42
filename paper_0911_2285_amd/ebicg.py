"""Python binding of libebicg.so (include/ebicg.h): argument marshalling only.

Every step of the solver runs in the HIP library; this module checks tensor
shapes, dtypes and devices, passes raw pointers and the current torch HIP
stream, and turns status codes into exceptions.  It raises if the built
library is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libebicg.so")

EB_OK = 0
# kernel classes of eb_timing_read (include/ebicg.h)
KERNEL_CLASSES = ["bicg_matvec", "bicg_update_r", "bicg_update_p", "stab_v", "stab_s", "stab_t", "stab_xr", "stab_p",
                  "rotate", "residual", "proj", "dslash", "bstab_v", "bstab_s", "bstab_t", "bstab_xr", "bstab_p",
                  "bdslash"]
STATUS = {
    0: "EB_OK",
    -1: "EB_ERR_INVALID",
    -2: "EB_ERR_OOM",
    -3: "EB_ERR_BREAKDOWN",
    -4: "EB_ERR_NOT_CONVERGED",
    -5: "EB_ERR_HIP",
    -6: "EB_ERR_EIG",
    -7: "EB_ERR_CAPACITY",
}
PREC = {"fp64": 0, "fp32": 1, "bf16": 2}


class EbicgError(RuntimeError):
    def __init__(self, status, msg, stats=None):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
        self.stats = stats


class _EigParams(ctypes.Structure):
    _fields_ = [
        ("nev", ctypes.c_int32),
        ("m", ctypes.c_int32),
        ("tol", ctypes.c_double),
        ("maxiter", ctypes.c_int32),
        ("rhat", ctypes.c_int32),
        ("window", ctypes.c_int32),
        ("device_eig", ctypes.c_int32),
        ("sort", ctypes.c_int32),
    ]


class _SolveParams(ctypes.Structure):
    _fields_ = [
        ("tol", ctypes.c_double),
        ("deftol", ctypes.c_double),
        ("maxiter", ctypes.c_int32),
        ("method", ctypes.c_int32),
        ("inner", ctypes.c_int32),
        ("inner_tol", ctypes.c_double),
        ("nrhs", ctypes.c_int32),
        ("batch", ctypes.c_int32),
    ]


class _Stats(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int32),
        ("matvec_d", ctypes.c_int32),
        ("matvec_ddag", ctypes.c_int32),
        ("window_restarts", ctypes.c_int32),
        ("defl_restarts", ctypes.c_int32),
        ("breakdown_restarts", ctypes.c_int32),
        ("outer_steps", ctypes.c_int32),
        ("nev_added", ctypes.c_int32),
        ("true_rel_resid", ctypes.c_double),
        ("rec_rel_resid", ctypes.c_double),
        ("seconds", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class _SessionParams(ctypes.Structure):
    _fields_ = [
        ("slots", ctypes.c_int32),
        ("inner", ctypes.c_int32),
        ("tol", ctypes.c_double),
        ("inner_tol", ctypes.c_double),
        ("maxiter", ctypes.c_int32),
        ("chunk", ctypes.c_int32),
        ("graph", ctypes.c_int32),
    ]


_lib = None

# (name, restype, argtypes) of every symbol declared in include/ebicg.h
_P = ctypes.c_void_p
_SIGNATURES = [
    ("eb_op_create", ctypes.c_int, [_P, ctypes.c_double, _P, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(_P)]),
    ("eb_op_create_eo", ctypes.c_int, [_P, ctypes.c_double, _P, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(_P)]),
    ("eb_op_destroy", ctypes.c_int, [_P]),
    ("eb_op_apply", ctypes.c_int, [_P, _P, _P, ctypes.c_int, _P]),
    ("eb_op_apply_dagger", ctypes.c_int, [_P, _P, _P, ctypes.c_int, _P]),
    ("eb_op_apply_noalloc", ctypes.c_int, [_P, _P, _P, ctypes.c_int32, _P]),
    ("eb_op_apply_schur", ctypes.c_int, [_P, _P, _P, ctypes.c_int32, _P]),
    ("eb_op_apply_block", ctypes.c_int, [_P, _P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int, _P]),
    ("eb_op_apply_schur_block", ctypes.c_int, [_P, _P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int, _P]),
    ("eb_eigbicg_solve", ctypes.c_int, [_P, _P, _P, ctypes.POINTER(_EigParams), _P, ctypes.POINTER(_Stats), _P]),
    ("eb_deflated_bicg_solve", ctypes.c_int, [_P, _P, _P, ctypes.POINTER(_SolveParams), ctypes.POINTER(_Stats), _P]),
    ("eb_get_eigenpairs", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32), _P, _P, _P, _P]),
    ("eb_defl_info", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32), _P]),
    ("eb_defl_reset", ctypes.c_int, [_P]),
    ("eb_small_eig", ctypes.c_int, [ctypes.c_int32, _P, _P, _P, _P]),
    ("eb_small_eig_device", ctypes.c_int, [ctypes.c_int32, _P, _P, _P, _P]),
    ("eb_timing_enable", ctypes.c_int, [_P, ctypes.c_int32]),
    ("eb_timing_classes", ctypes.c_int, [_P, ctypes.c_uint32]),
    ("eb_timing_read", ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                                      ctypes.POINTER(ctypes.c_double)]),
    ("eb_session_create", ctypes.c_int, [_P, ctypes.POINTER(_SessionParams), _P, ctypes.POINTER(_P)]),
    ("eb_session_destroy", ctypes.c_int, [_P]),
    ("eb_session_admit", ctypes.c_int, [_P, _P, _P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32)]),
    ("eb_session_step", ctypes.c_int, [_P]),
    ("eb_session_ready", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32)]),
    ("eb_session_poll", ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P, ctypes.POINTER(ctypes.c_int32)]),
    ("eb_session_info", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_uint64)]),
    ("eb_op_device_bytes", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_uint64)]),
    ("eb_op_trim", ctypes.c_int, [_P, _P]),
    ("eb_op_set_grid_cap", ctypes.c_int, [_P, ctypes.c_int32]),
    ("eb_op_batch_tune", ctypes.c_int, [_P, ctypes.c_int, _P, ctypes.POINTER(ctypes.c_int32), _P, _P]),
    ("eb_op_batch_set_tile", ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int32, ctypes.c_int32]),
    ("eb_op_set_matvec_form", ctypes.c_int, [_P, ctypes.c_int32]),
    ("eb_op_get_matvec_form", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32), _P]),
    ("eb_last_error", None, [ctypes.c_char_p, ctypes.c_size_t]),
    ("eb_version", ctypes.c_char_p, []),
]
SYMBOLS = [n for n, _, _ in _SIGNATURES]


def lib():
    """Load libebicg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_0911_2285_amd.build` first")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _last_error():
    buf = ctypes.create_string_buffer(1024)
    lib().eb_last_error(buf, 1024)
    return buf.value.decode(errors="replace")


def _check(status, stats=None):
    if status != EB_OK:
        raise EbicgError(status, _last_error(), stats)


def _stream(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_ptr(t, numel, dtype, name):
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA/HIP tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous() or t.numel() != numel:
        raise ValueError(f"{name} must be contiguous with {numel} elements, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


def version():
    return lib().eb_version().decode()


def small_eig(C):
    """[y, z, lambda] of the library's host eigensolver (eig(C) of the paper's conventions)."""
    C = np.ascontiguousarray(C, dtype=np.complex128)
    n = C.shape[0]
    lam = np.zeros(n, np.complex128)
    y = np.zeros((n, n), np.complex128)
    z = np.zeros((n, n), np.complex128)
    _check(lib().eb_small_eig(n, C.ctypes.data, lam.ctypes.data, y.ctypes.data, z.ctypes.data))
    return y, z, lam


def small_eig_device(C):
    """The same eigenproblem solved by the library's one-workgroup device solver."""
    C = np.ascontiguousarray(C, dtype=np.complex128)
    n = C.shape[0]
    lam = np.zeros(n, np.complex128)
    y = np.zeros((n, n), np.complex128)
    z = np.zeros((n, n), np.complex128)
    _check(lib().eb_small_eig_device(n, C.ctypes.data, lam.ctypes.data, y.ctypes.data, z.ctypes.data))
    return y, z, lam


@dataclass
class Operator:
    """An eb_op: the Wilson-Dirac operator on one gauge field plus its deflation space."""

    handle: ctypes.c_void_p
    dims: tuple
    kappa: float
    V: int

    @property
    def N(self):
        return 12 * self.V

    def __del__(self):
        try:
            op_destroy(self)
        except Exception:
            pass


def op_create(gauge, kappa, dims, bc_t=-1, defl_capacity=0, eo=False):
    """gauge: complex128 array [4][V][3][3] on the host.  eo: solves run on the
    even-odd (Schur) form (eb_op_create_eo); vectors stay full-lattice canonical."""
    dims = tuple(int(d) for d in dims)
    V = int(np.prod(dims))
    g = np.ascontiguousarray(gauge, dtype=np.complex128)
    if g.size != 36 * V:
        raise ValueError(f"gauge must have 36*V = {36 * V} complex entries")
    d = (ctypes.c_int32 * 4)(*dims)
    h = ctypes.c_void_p()
    create = lib().eb_op_create_eo if eo else lib().eb_op_create
    _check(create(g.ctypes.data, float(kappa), d, int(bc_t), int(defl_capacity), ctypes.byref(h)))
    return Operator(h, dims, float(kappa), V)


def op_destroy(op):
    if op.handle and op.handle.value:
        _check(lib().eb_op_destroy(op.handle))
        op.handle = ctypes.c_void_p()


def _spinor_ptr(op, t, prec, name):
    """Device pointer of a canonical spinor: complex128 (fp64), complex64 (fp32),
    or bfloat16 pairs (re, im) with 2 N elements (bf16)."""
    import torch

    if prec == "bf16":
        return _dev_ptr(t, 2 * op.N, torch.bfloat16, name)
    return _dev_ptr(t, op.N, {"fp64": torch.complex128, "fp32": torch.complex64}[prec], name)


def op_apply(op, out, inp, prec="fp64", stream=None):
    """out = D inp (device tensors in the canonical [V][4][3] layout)."""
    _check(lib().eb_op_apply(op.handle, _spinor_ptr(op, out, prec, "out"), _spinor_ptr(op, inp, prec, "in"),
                             PREC[prec], _stream(stream)))


def op_apply_dagger(op, out, inp, prec="fp64", stream=None):
    """out = D^+ inp."""
    _check(lib().eb_op_apply_dagger(op.handle, _spinor_ptr(op, out, prec, "out"), _spinor_ptr(op, inp, prec, "in"),
                                    PREC[prec], _stream(stream)))


def op_apply_noalloc(op, out, inp, dagger=False, stream=None):
    """out = D inp (or D^+) in FP64 without any device allocation (the library's fixed
    per-GPU staging array; V <= 131072)."""
    _check(lib().eb_op_apply_noalloc(op.handle, _spinor_ptr(op, out, "fp64", "out"),
                                     _spinor_ptr(op, inp, "fp64", "in"), int(bool(dagger)), _stream(stream)))


def op_apply_schur(op, out, inp, dagger=False, stream=None):
    """out = Dhat inp_e (or Dhat^+) for an even-odd operator; full-lattice FP64
    canonical tensors, odd sites of inp ignored and of out zero."""
    _check(lib().eb_op_apply_schur(op.handle, _spinor_ptr(op, out, "fp64", "out"), _spinor_ptr(op, inp, "fp64", "in"),
                                   int(bool(dagger)), _stream(stream)))


def op_apply_schur_block(op, out, inp, k, dagger=False, prec="fp64", stream=None):
    """out_i = Dhat inp_i (or Dhat^+) for k full-lattice FP64 canonical spinors
    back to back (even-odd operator); prec is the storage of the pass."""
    import torch

    _check(lib().eb_op_apply_schur_block(op.handle, _dev_ptr(out, op.N * k, torch.complex128, "out"),
                                         _dev_ptr(inp, op.N * k, torch.complex128, "in"), int(k),
                                         int(bool(dagger)), PREC[prec], _stream(stream)))


def op_apply_block(op, out, inp, k, dagger=False, prec="fp64", stream=None):
    """out_i = D inp_i (or D^+) for k spinors back to back, one pass over the links."""
    import torch

    if prec == "bf16":
        po, pi = _dev_ptr(out, 2 * op.N * k, torch.bfloat16, "out"), _dev_ptr(inp, 2 * op.N * k, torch.bfloat16, "in")
    else:
        dt = {"fp64": torch.complex128, "fp32": torch.complex64}[prec]
        po, pi = _dev_ptr(out, op.N * k, dt, "out"), _dev_ptr(inp, op.N * k, dt, "in")
    _check(lib().eb_op_apply_block(op.handle, po, pi, int(k), int(bool(dagger)), PREC[prec], _stream(stream)))


SORT = {"SM": 0, "SR": 1, "LM": 2}


def eigbicg_solve(op, b, x, nev, m, tol, maxiter=10000, rhat=0, window="fp64", device_eig=False, sort="SM",
                  stream=None):
    """One eigBiCG solve that grows the deflation space; returns (stats, ritz values).

    rhat: 0 -> rhat_0 = r_0; 1 -> gamma5 r_0; 2 -> the gamma5-Hermitian form
    (shadow vectors implicit, one D per iteration).  window: "fp64" or "fp32"
    storage of the window vectors; device_eig: the window eigenproblems on the GPU.
    sort: the pairs kept and returned, "SM" smallest |lambda|, "SR" smallest real
    part, "LM" largest |lambda| (or the eb_sort value)."""
    import torch

    srt = SORT[sort] if isinstance(sort, str) else int(sort)
    p = _EigParams(int(nev), int(m), float(tol), int(maxiter), int(rhat), PREC[window], int(bool(device_eig)), srt)
    st = _Stats()
    ritz = np.zeros(int(nev), np.complex128)
    rc = lib().eb_eigbicg_solve(
        op.handle,
        _dev_ptr(b, op.N, torch.complex128, "b"),
        _dev_ptr(x, op.N, torch.complex128, "x"),
        ctypes.byref(p),
        ritz.ctypes.data,
        ctypes.byref(st),
        _stream(stream),
    )
    _check(rc, st.as_dict())
    return st.as_dict(), ritz


def deflated_bicg_solve(op, b, x, tol, deftol=0.0, maxiter=10000, method=0, inner="fp64", inner_tol=0.0, nrhs=1,
                        batch=1, stream=None):
    """Deflated BiCGStab (method 0) or two-sided BiCG (method 1, FP64 only) solve(s); b, x hold nrhs
    spinors back to back.  batch: columns per
    multi-RHS iteration (1, 2, 4, 8, 16; 0 = the library's timed choice).  Returns stats."""
    import torch

    p = _SolveParams(float(tol), float(deftol), int(maxiter), int(method), PREC[inner], float(inner_tol), int(nrhs),
                     int(batch))
    st = _Stats()
    rc = lib().eb_deflated_bicg_solve(
        op.handle,
        _dev_ptr(b, op.N * nrhs, torch.complex128, "b"),
        _dev_ptr(x, op.N * nrhs, torch.complex128, "x"),
        ctypes.byref(p),
        ctypes.byref(st),
        _stream(stream),
    )
    _check(rc, st.as_dict())
    return st.as_dict()


def get_eigenpairs(op, k, right=None, left=None, stream=None):
    """Rayleigh-Ritz eigenpairs of the deflation space; returns the eigenvalues."""
    import torch

    kk = ctypes.c_int32(int(k))
    ev = np.zeros(int(k), np.complex128)
    rp = _dev_ptr(right, op.N * k, torch.complex128, "right") if right is not None else None
    lp = _dev_ptr(left, op.N * k, torch.complex128, "left") if left is not None else None
    _check(lib().eb_get_eigenpairs(op.handle, ctypes.byref(kk), ev.ctypes.data, rp, lp, _stream(stream)))
    return ev[: kk.value]


def defl_info(op):
    """(K, H) of the deflation space; H = U_l^+ A U_r as a K x K numpy array."""
    K = ctypes.c_int32(0)
    _check(lib().eb_defl_info(op.handle, ctypes.byref(K), None))
    H = np.zeros((K.value, K.value), np.complex128)
    _check(lib().eb_defl_info(op.handle, ctypes.byref(K), H.ctypes.data if K.value else None))
    return K.value, H


def defl_reset(op):
    _check(lib().eb_defl_reset(op.handle))


def timing_enable(op, enable=True):
    """Start (and reset) or stop per-kernel HIP-event timing inside the library's solves."""
    _check(lib().eb_timing_enable(op.handle, int(bool(enable))))


def timing_classes(op, names=None):
    """Record only these kernel classes while timing is enabled (None: all)."""
    mask = 0xFFFFFFFF if names is None else sum(1 << KERNEL_CLASSES.index(n) for n in names)
    _check(lib().eb_timing_classes(op.handle, mask))


def timing_read(op):
    """{kernel class: (launches, total ms)} since the last timing_enable."""
    out = {}
    for k, name in enumerate(KERNEL_CLASSES):
        n = ctypes.c_int64(0)
        ms = ctypes.c_double(0)
        _check(lib().eb_timing_read(op.handle, k, ctypes.byref(n), ctypes.byref(ms)))
        out[name] = (n.value, ms.value)
    return out


def op_device_bytes(op):
    """Device bytes the operator holds (links, deflation space, work buffers)."""
    n = ctypes.c_uint64(0)
    _check(lib().eb_op_device_bytes(op.handle, ctypes.byref(n)))
    return n.value


def op_set_grid_cap(op, max_blocks):
    """Cap the grid of the reducing stencil kernels (0 restores the default of 1024 blocks); with a
    small cap every block loops over several site tiles, the path large lattices take."""
    _check(lib().eb_op_set_grid_cap(op.handle, int(max_blocks)))


def op_trim(op, stream=None):
    """Release the operator's work buffers (not its links or deflation space)."""
    _check(lib().eb_op_trim(op.handle, _stream(stream)))


TILE_FORMS = 7  # EB_TILE_FORMS


def op_batch_tune(op, prec="fp32", stream=None):
    """The batch autotuner's choice for one precision: {"k": best k, "stage": {k: tile form},
    "ms_per_rhs": {k: [global reads, LDS-staged, bricks 8x8x4x4, 8x8x8x8, 4x4x4x4, unfenced,
    t-marching]}} (0 for a form the operator does not admit; runs the tuner once per operator
    and precision)."""
    kb = ctypes.c_int32(0)
    stage = np.zeros(5, np.int32)
    ms = np.zeros(5 * TILE_FORMS, np.float64)
    _check(lib().eb_op_batch_tune(op.handle, PREC[prec], _stream(stream), ctypes.byref(kb), stage.ctypes.data,
                                  ms.ctypes.data))
    ks = [1, 2, 4, 8, 16]
    F = TILE_FORMS
    return {"k": kb.value, "stage": {k: int(stage[i]) for i, k in enumerate(ks)},
            "ms_per_rhs": {k: [float(v) for v in ms[F * i: F * i + F]] for i, k in enumerate(ks)}}


def op_set_matvec_form(op, form):
    """Form of the BiCG matvec pair (eigBiCG, deflated BiCG): 1 LDS-staged tiles, 6
    t-marching units, -1 time both at the next solve."""
    _check(lib().eb_op_set_matvec_form(op.handle, int(form)))


def op_get_matvec_form(op):
    """(form in use, {1: ms, 6: ms} measured by the choice)."""
    f = ctypes.c_int32(0)
    ms = np.zeros(2, np.float64)
    _check(lib().eb_op_get_matvec_form(op.handle, ctypes.byref(f), ms.ctypes.data))
    return f.value, {1: float(ms[0]), 6: float(ms[1])}


def op_batch_set_tile(op, prec, k, stage):
    """Force the tile form of the batched stencil for (prec, k): 0 global reads, 1 LDS-staged,
    2 / 3 / 4 global reads in bricks, 5 global reads without fences between hops, 6 t-marching
    boxes (full-lattice operators; the box must hold a whole number of blocks for k), -1
    built-in rule.  For k = 1 it also picks the one-at-a-time solver's stencil form (6, or 1
    for any other form)."""
    _check(lib().eb_op_batch_set_tile(op.handle, PREC[prec], int(k), int(stage)))


class Session:
    """An eb_session: continuous batching of deflated solves on one operator.

    admit() reserves a slot (host only); step() harvests the chunk in flight,
    starts admitted requests and launches the next chunk; poll() returns the
    finished requests as (tag, status name, stats dict)."""

    def __init__(self, op, slots=8, inner="fp32", tol=1e-10, inner_tol=0.0, maxiter=20000, chunk=8, graph=True,
                 stream=None):
        import torch

        self.op = op
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        p = _SessionParams(int(slots), PREC[inner], float(tol), float(inner_tol), int(maxiter), int(chunk),
                           int(bool(graph)))
        self.handle = ctypes.c_void_p()
        _check(lib().eb_session_create(op.handle, ctypes.byref(p), _stream(self.stream), ctypes.byref(self.handle)))
        self.slots = int(slots)
        self._tags = np.zeros(self.slots, np.int64)
        self._status = np.zeros(self.slots, np.int32)
        self._stats = (_Stats * self.slots)()

    def admit(self, b, x, tag):
        """Reserve a slot for solving A x = b (device FP64 canonical spinors, x holds x0);
        returns the slot, or None when every slot is busy."""
        import torch

        slot = ctypes.c_int32(-1)
        rc = lib().eb_session_admit(self.handle, _dev_ptr(b, self.op.N, torch.complex128, "b"),
                                    _dev_ptr(x, self.op.N, torch.complex128, "x"), int(tag), ctypes.byref(slot))
        if rc == -7:
            return None
        _check(rc)
        return slot.value

    def step(self):
        _check(lib().eb_session_step(self.handle))

    def ready(self):
        """True when step() would not wait for the chunk in flight."""
        r = ctypes.c_int32(0)
        _check(lib().eb_session_ready(self.handle, ctypes.byref(r)))
        return bool(r.value)

    def poll(self):
        n = ctypes.c_int32(0)
        _check(lib().eb_session_poll(self.handle, self.slots, self._tags.ctypes.data, self._status.ctypes.data,
                                     self._stats, ctypes.byref(n)))
        return [(int(self._tags[i]), STATUS.get(int(self._status[i]), int(self._status[i])), self._stats[i].as_dict())
                for i in range(n.value)]

    def info(self):
        """{free, busy, done, device_bytes}."""
        f, b, d = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
        nb = ctypes.c_uint64(0)
        _check(lib().eb_session_info(self.handle, ctypes.byref(f), ctypes.byref(b), ctypes.byref(d),
                                     ctypes.byref(nb)))
        return {"free": f.value, "busy": b.value, "done": d.value, "device_bytes": nb.value}

    def close(self):
        if self.handle and self.handle.value:
            _check(lib().eb_session_destroy(self.handle))
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
