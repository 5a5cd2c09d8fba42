"""The C-ABI library loads and exports every declared symbol; host-only calls work without a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle.eig import eig as oracle_eig

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ebicg.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(eb_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def eb():
    from paper_0911_2285_amd import ebicg

    if not os.path.exists(ebicg.LIB_PATH):
        pytest.fail("libebicg.so is not built (run __graft_entry__.build())")
    ebicg.lib()
    return ebicg


def test_header_declares_the_boundary():
    names = _declared()
    for must in ["eb_op_create", "eb_op_apply", "eb_op_apply_dagger", "eb_eigbicg_solve", "eb_deflated_bicg_solve",
                 "eb_get_eigenpairs"]:
        assert must in names


def test_library_exports_every_declared_symbol(eb):
    L = eb.lib()
    for name in _declared():
        assert hasattr(L, name), name
    assert set(_declared()) == set(eb.SYMBOLS)
    assert "gfx950" in eb.version()


def _header_structs():
    """Field (C type, name) lists of the header's typedef'd parameter structs."""
    txt = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    out = {}
    for body, name in re.findall(r"typedef struct \{(.*?)\}\s*(eb_[a-z_]+)\s*;", txt, flags=re.S):
        out[name] = [tuple(f.split()) for f in body.split(";") if f.strip()]
    return out


def test_binding_structs_match_the_header():
    """The ctypes mirrors of the parameter and statistics structs have the header's
    fields, in its order, with the same widths (a field added to one side only
    would shift every later field)."""
    from paper_0911_2285_amd import ebicg

    ctype = {"int32_t": ctypes.c_int32, "double": ctypes.c_double, "eb_prec": ctypes.c_int32,
             "uint64_t": ctypes.c_uint64, "int64_t": ctypes.c_int64}
    mirrors = {"eb_eig_params": ebicg._EigParams, "eb_solve_params": ebicg._SolveParams, "eb_stats": ebicg._Stats,
               "eb_session_params": ebicg._SessionParams}
    structs = _header_structs()
    assert set(mirrors) <= set(structs)
    for name, cls in mirrors.items():
        fields = structs[name]
        assert [f[1] for f in fields] == [f[0] for f in cls._fields_], name
        for (ct, fname), (_, pyt) in zip(fields, cls._fields_):
            assert ctypes.sizeof(ctype[ct]) == ctypes.sizeof(pyt), (name, fname)


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (7, 2), (16, 3), (40, 4), (64, 5)])
def test_small_eig_matches_lapack(eb, n, seed):
    rng = np.random.default_rng(seed)
    C = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    y, z, lam = eb.small_eig(C)
    yr, zr, lr = oracle_eig(C)
    assert np.abs(lam - lr).max() <= 1e-12 * max(1, np.abs(lr).max())
    assert np.abs(C @ y - y * lam).max() < 1e-12 * max(1, np.abs(C).max()) * n
    assert np.abs(z.conj().T @ C - lam[:, None] * z.conj().T).max() < 1e-12 * max(1, np.abs(C).max()) * n
    assert np.abs(np.diag(z.conj().T @ y) - 1).max() < 1e-12
    assert np.allclose(np.linalg.norm(y, axis=0), 1)
    # vectors agree with LAPACK's up to a unit phase
    for i in range(n):
        ph = np.vdot(yr[:, i], y[:, i])
        assert abs(abs(ph) - 1) < 1e-8
        assert np.linalg.norm(y[:, i] - ph * yr[:, i]) < 1e-8


def test_small_eig_structured(eb):
    """Tridiagonal + arrow (the restarted window matrix), real with conjugate pairs, diagonal ties."""
    rng = np.random.default_rng(9)
    n = 40
    T = np.diag(rng.standard_normal(n) + 0.1j * rng.standard_normal(n)) + np.diag(rng.standard_normal(n - 1), 1)
    T += np.diag(rng.standard_normal(n - 1), -1)
    T[20, :20] = rng.standard_normal(20)
    T[:20, 20] = rng.standard_normal(20)
    D = np.diag([3.0, 1.0, 2.0, 1.0, 2.0 + 0.5j, 2.0 - 0.5j]).astype(complex)
    R = rng.standard_normal((30, 30)).astype(complex)
    for C in (T.astype(complex), D, R):
        y, z, lam = eb.small_eig(C)
        _, _, lr = oracle_eig(C)
        assert np.abs(lam - lr).max() < 1e-12 * max(1, np.abs(lr).max())
        assert np.abs(C @ y - y * lam).max() < 1e-11 * max(1, np.abs(C).max())


def test_invalid_arguments_are_rejected_on_the_host(eb):
    import ctypes

    U = np.zeros((4, 16, 3, 3), np.complex128)
    h = ctypes.c_void_p()
    dims = (ctypes.c_int32 * 4)(1, 2, 2, 4)
    rc = eb.lib().eb_op_create(U.ctypes.data, 0.1, dims, -1, 0, ctypes.byref(h))
    assert rc == -1
    buf = ctypes.create_string_buffer(256)
    eb.lib().eb_last_error(buf, 256)
    assert b">= 2" in buf.value
    dims = (ctypes.c_int32 * 4)(2, 2, 2, 2)
    assert eb.lib().eb_op_create(U.ctypes.data, float("nan"), dims, -1, 0, ctypes.byref(h)) == -1
    assert eb.lib().eb_op_create(U.ctypes.data, 0.1, dims, 0, 0, ctypes.byref(h)) == -1
    assert eb.lib().eb_op_create(None, 0.1, dims, -1, 0, ctypes.byref(h)) == -1


def test_session_and_tuning_calls_reject_null_handles_on_the_host(eb):
    """The serving and autotuning entry points validate their arguments before
    touching a device: null handles and null outputs give EB_ERR_INVALID with a
    message, and destroying a null session is a no-op."""
    import ctypes

    L = eb.lib()
    n = ctypes.c_int32(0)
    r = ctypes.c_int32(0)
    nb = ctypes.c_uint64(0)
    params = eb._SessionParams(4, 1, 1e-10, 0.0, 100, 8, 1)
    out = ctypes.c_void_p()
    assert L.eb_session_create(None, ctypes.byref(params), None, ctypes.byref(out)) == -1
    assert L.eb_session_admit(None, None, None, 0, None) == -1
    assert L.eb_session_step(None) == -1
    assert L.eb_session_ready(None, ctypes.byref(r)) == -1
    assert L.eb_session_poll(None, 0, None, None, None, ctypes.byref(n)) == -1
    assert L.eb_session_info(None, None, None, None, None) == -1
    assert L.eb_session_destroy(None) == 0
    assert L.eb_op_device_bytes(None, ctypes.byref(nb)) == -1
    assert L.eb_op_trim(None, None) == -1
    assert L.eb_op_batch_set_tile(None, 1, 4, 0) == -1
    assert L.eb_op_batch_tune(None, 1, None, ctypes.byref(n), None, None) == -1
    assert L.eb_op_set_grid_cap(None, 4) == -1
    buf = ctypes.create_string_buffer(256)
    L.eb_last_error(buf, 256)
    assert buf.value  # the last call left a message
