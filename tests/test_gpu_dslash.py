"""GPU parity of D and D^+ (through the C ABI) against the FP64 oracle."""
import numpy as np
import pytest

import synth
from oracle import wilson as W

pytestmark = pytest.mark.gpu


def _setup(gpu_lib, dims, kappa, bc_t=-1, seed=1000, eps=0.3):
    import torch

    U = synth.random_su3_links(dims, eps, seed)
    op = gpu_lib.op_create(U, kappa, dims, bc_t=bc_t)
    return U, op, torch.device("cuda:0")


@pytest.mark.parametrize(
    "dims,bc_t",
    [((2, 2, 2, 2), -1), ((4, 4, 4, 4), -1), ((4, 4, 4, 4), 1), ((3, 4, 2, 6), -1), ((8, 8, 8, 8), -1),
     ((6, 2, 10, 4), 1)],
)
def test_dslash_fp64_parity(gpu_lib, dims, bc_t):
    import torch

    kappa = 0.122
    U, op, dev = _setup(gpu_lib, dims, kappa, bc_t)
    V = synth.volume(dims)
    psi = synth.gaussian_spinor(V, 7)
    x = torch.from_numpy(psi).to(dev)
    for dag in (False, True):
        y = torch.empty_like(x)
        (gpu_lib.op_apply_dagger if dag else gpu_lib.op_apply)(op, y, x)
        ref = (W.apply_Ddag if dag else W.apply_D)(U, psi, kappa, dims, bc_t=bc_t)
        err = np.abs(y.cpu().numpy() - ref).max() / np.abs(ref).max()
        print(f"dims={dims} bc={bc_t} dagger={dag}: max rel err {err:.2e}")
        assert err <= 1e-12


def test_dslash_free_field_plane_wave(gpu_lib):
    """U = 1: a plane wave is an eigenvector with the closed-form eigenvalue."""
    import torch

    dims = (4, 4, 4, 8)
    kappa = 0.1
    V = synth.volume(dims)
    op = gpu_lib.op_create(synth.unit_links(dims), kappa, dims, bc_t=-1)
    p = np.array([2 * np.pi / 4, 0.0, 2 * np.pi * 3 / 4, np.pi * 3 / 8])
    g = W.gammas()
    ev, evec = np.linalg.eigh(sum(g[mu] * np.sin(p[mu]) for mu in range(4)))
    c = np.stack(W.site_coords(np.arange(V), dims), axis=1)
    psi = np.exp(1j * (c @ p))[:, None, None] * evec[:, 0][None, :, None] * np.array([1.0, 0.5j, -0.25])[None, None, :]
    lam = 1 - 2 * kappa * np.cos(p).sum() + 2j * kappa * ev[0]
    x = torch.from_numpy(psi).to("cuda:0")
    y = torch.empty_like(x)
    gpu_lib.op_apply(op, y, x)
    assert np.abs(y.cpu().numpy() - lam * psi).max() < 1e-14


def test_dslash_fp32_error(gpu_lib):
    import torch

    dims, kappa = (8, 8, 4, 8), 0.122
    U, op, dev = _setup(gpu_lib, dims, kappa)
    V = synth.volume(dims)
    psi = synth.gaussian_spinor(V, 3)
    x = torch.from_numpy(psi.astype(np.complex64)).to(dev)
    y = torch.empty_like(x)
    gpu_lib.op_apply(op, y, x, prec="fp32")
    ref = W.apply_D(U, psi.astype(np.complex64).astype(np.complex128), kappa, dims)
    err = np.abs(y.cpu().numpy() - ref).max() / np.abs(ref).max()
    print(f"fp32 dslash max rel err vs FP64 oracle: {err:.2e}")
    assert err < 5e-7


def test_dslash_bf16_error(gpu_lib):
    """BF16-stored links and spinors, FP32 arithmetic: error against the FP64
    oracle applied to the same (rounded) input.  Links and the output are
    rounded to 8 significant bits (relative 2^-9), so the bound is a few 2^-9
    of the largest entry."""
    import torch

    dims, kappa = (8, 4, 4, 8), 0.122
    U, op, dev = _setup(gpu_lib, dims, kappa)
    V = synth.volume(dims)
    psi = synth.gaussian_spinor(V, 5)
    x = torch.view_as_real(torch.from_numpy(psi)).to(torch.bfloat16).contiguous().to(dev)
    psi_r = torch.view_as_complex(x.cpu().to(torch.float64)).numpy()
    for dag in (False, True):
        y = torch.empty_like(x)
        (gpu_lib.op_apply_dagger if dag else gpu_lib.op_apply)(op, y, x, prec="bf16")
        got = torch.view_as_complex(y.cpu().to(torch.float64)).numpy()
        ref = (W.apply_Ddag if dag else W.apply_D)(U, psi_r, kappa, dims)
        err = np.abs(got - ref).max() / np.abs(ref).max()
        print(f"bf16 dslash dagger={dag}: max rel err vs FP64 oracle {err:.2e}")
        assert 1e-5 < err < 4 * 2.0**-9


def test_dslash_full_size_sampled(gpu_lib):
    """16^3 x 32 (the incremental-eigBiCG workload): sampled sites against the per-site oracle."""
    import torch

    dims, kappa = (16, 16, 16, 32), 0.122
    U, op, dev = _setup(gpu_lib, dims, kappa, seed=synth.gauge_seed(1))
    V = synth.volume(dims)
    psi = synth.z2_source(V, synth.rhs_seed(0, 3))
    x = torch.from_numpy(psi).to(dev)
    rng = np.random.default_rng(0)
    sites = np.concatenate([[0, 15, 16 * 16 * 16 - 1, V - 1, V - 16 * 16 * 16], rng.integers(0, V, 60)])
    for dag in (False, True):
        y = torch.empty_like(x)
        (gpu_lib.op_apply_dagger if dag else gpu_lib.op_apply)(op, y, x)
        got = y.cpu().numpy()[sites]
        ref = W.apply_D_sites(U, psi, kappa, dims, sites, dagger=dag)
        err = np.abs(got - ref).max() / np.abs(ref).max()
        assert err <= 1e-12, err


@pytest.fixture(scope="module")
def lattice_24x64(gpu_lib):
    """24^3 x 64 (the precision / batching lattice: fields beyond the Infinity Cache)."""
    dims, kappa = (24, 24, 24, 64), 0.123
    U = synth.random_su3_links(dims, 0.3, synth.gauge_seed(2))
    op = gpu_lib.op_create(U, kappa, dims)
    return dims, kappa, U, op


def _sample_sites(dims, n=48, seed=0):
    V = synth.volume(dims)
    plane = dims[0] * dims[1] * dims[2]
    rng = np.random.default_rng(seed)
    # corners of the lattice and of the t boundary, tile boundaries, then random sites
    fixed = [0, dims[0] - 1, plane - 1, V - 1, V - plane, 255, 256, 511]
    return np.concatenate([fixed, rng.integers(0, V, n)])


def test_dslash_24x64_sampled(gpu_lib, lattice_24x64):
    """FP64 D and D^+ on 24^3 x 64 at sampled sites against the per-site oracle (1e-12)."""
    import torch

    dims, kappa, U, op = lattice_24x64
    V = synth.volume(dims)
    psi = synth.gaussian_spinor(V, 11)
    x = torch.from_numpy(psi).to("cuda:0")
    sites = _sample_sites(dims)
    for dag in (False, True):
        y = torch.empty_like(x)
        (gpu_lib.op_apply_dagger if dag else gpu_lib.op_apply)(op, y, x)
        got = y.cpu().numpy()[sites]
        ref = W.apply_D_sites(U, psi, kappa, dims, sites, dagger=dag)
        err = np.abs(got - ref).max() / np.abs(ref).max()
        print(f"24^3x64 dagger={dag}: sampled max rel err {err:.2e}")
        assert err <= 1e-12, err


def _boundary_sites(dims, n=32, seed=0):
    """Sites on the t slices where chunks of 8, 16 and 32 slices meet and on the
    z planes where boxes of 8 meet, at random x, y; then random sites."""
    lx, ly, lz, lt = dims
    rng = np.random.default_rng(seed)
    ts = sorted({t % lt for c in (8, 16, 32) for t in range(0, lt, c) for t in (t - 1, t)})
    zs = sorted({z % lz for z in range(0, lz, 8) for z in (z - 1, z)})
    fixed = [W.site_index(int(rng.integers(lx)), int(rng.integers(ly)), z, t, dims) for t in ts for z in zs]
    return np.concatenate([fixed, rng.integers(0, synth.volume(dims), n)])


def _one_column_march_fp64(gpu_lib, op, U, dims, kappa, seed):
    """FP64 D and D^+ with one column in the t-marching form (8-slice chunks at
    24^3 x 64, 16-slice chunks at 32^3 x 64, boxes of 8 z planes) and in the
    LDS-staged form, at the chunk- and box-boundary sites, against the per-site
    oracle (1e-12)."""
    import torch

    V = synth.volume(dims)
    psi = synth.gaussian_spinor(V, seed)
    x = torch.from_numpy(psi).to("cuda:0")
    sites = _boundary_sites(dims, seed=seed)
    for dag in (False, True):
        ref = W.apply_D_sites(U, psi, kappa, dims, sites, dagger=dag)
        for stage in (6, 1):
            gpu_lib.op_batch_set_tile(op, "fp64", 1, stage)
            y = torch.empty_like(x)
            gpu_lib.op_apply_block(op, y, x, 1, dagger=dag)
            err = np.abs(y.cpu().numpy()[sites] - ref).max() / np.abs(ref).max()
            print(f"{dims} one column FP64 form {stage} dagger={dag}: {len(sites)} sites, max rel err {err:.2e}")
            assert err <= 1e-12, (stage, dag, err)
    gpu_lib.op_batch_set_tile(op, "fp64", 1, -1)


def test_one_column_march_fp64_24x64_sampled(gpu_lib, lattice_24x64):
    dims, kappa, U, op = lattice_24x64
    _one_column_march_fp64(gpu_lib, op, U, dims, kappa, 13)


def test_dslash_block_24x64_sampled(gpu_lib, lattice_24x64):
    """FP32 multi-RHS stencil (k = 4) on 24^3 x 64: every column at sampled sites
    against the oracle on the rounded inputs; timing of the block stencil class."""
    import torch

    dims, kappa, U, op = lattice_24x64
    V = synth.volume(dims)
    k = 4
    psi = np.stack([synth.z2_source(V, synth.rhs_seed(2, c)) for c in range(k)]).astype(np.complex64)
    x = torch.from_numpy(psi).to("cuda:0")
    y = torch.empty_like(x)
    gpu_lib.timing_classes(op, ["bdslash"])
    gpu_lib.timing_enable(op, True)
    gpu_lib.op_apply_block(op, y, x, k, prec="fp32")
    n, ms = gpu_lib.timing_read(op)["bdslash"]
    assert n == 1 and ms > 0 and gpu_lib.timing_read(op)["dslash"][0] == 0
    gpu_lib.timing_enable(op, False)
    gpu_lib.timing_classes(op, None)
    sites = _sample_sites(dims, n=24, seed=1)
    got = y.cpu().numpy()
    for c in range(k):
        ref = W.apply_D_sites(U, psi[c].astype(np.complex128), kappa, dims, sites)
        err = np.abs(got[c][sites] - ref).max() / np.abs(ref).max()
        assert err < 5e-7, (c, err)


def test_gamma5_hermiticity_on_gpu(gpu_lib):
    """gamma5 D gamma5 = D^+ and <y, D x> = <D^+ y, x> at a size the dense oracle cannot hold."""
    import torch

    dims, kappa = (8, 8, 8, 16), 0.122
    U, op, dev = _setup(gpu_lib, dims, kappa, seed=4)
    V = synth.volume(dims)
    x = torch.from_numpy(synth.gaussian_spinor(V, 1)).to(dev)
    yv = torch.from_numpy(synth.gaussian_spinor(V, 2)).to(dev)
    g5 = torch.tensor([1, 1, -1, -1], dtype=torch.complex128, device=dev)[None, :, None]
    Dx = torch.empty_like(x)
    gpu_lib.op_apply(op, Dx, (g5 * x).contiguous())
    Ddx = torch.empty_like(x)
    gpu_lib.op_apply_dagger(op, Ddx, x)
    assert (g5 * Dx - Ddx).abs().max().item() < 1e-13
    Dx2 = torch.empty_like(x)
    gpu_lib.op_apply(op, Dx2, x)
    Ddy = torch.empty_like(x)
    gpu_lib.op_apply_dagger(op, Ddy, yv)
    a = torch.vdot(yv.flatten(), Dx2.flatten()).item()
    b = torch.vdot(Ddy.flatten(), x.flatten()).item()
    assert abs(a - b) <= 1e-12 * abs(a)


def test_dslash_deterministic(gpu_lib):
    import torch

    dims, kappa = (8, 8, 8, 8), 0.12
    U, op, dev = _setup(gpu_lib, dims, kappa)
    x = torch.from_numpy(synth.gaussian_spinor(synth.volume(dims), 9)).to(dev)
    y1, y2 = torch.empty_like(x), torch.empty_like(x)
    gpu_lib.op_apply(op, y1, x)
    gpu_lib.op_apply(op, y2, x)
    assert torch.equal(y1, y2)


@pytest.mark.parametrize("k", [2, 4, 16])
def test_dslash_block_parity(gpu_lib, k):
    """Multi-RHS stencil (one pass over the links for k sources) against the
    oracle column by column: FP64 at 1e-12; FP32 and BF16 storage against the
    oracle on the rounded inputs."""
    import torch

    dims, kappa = (4, 6, 4, 8), 0.122
    U, op, dev = _setup(gpu_lib, dims, kappa)
    V = synth.volume(dims)
    psi = np.stack([synth.gaussian_spinor(V, 40 + c) for c in range(k)])
    for dag in (False, True):
        f = W.apply_Ddag if dag else W.apply_D
        ref = np.stack([f(U, psi[c], kappa, dims) for c in range(k)])
        x = torch.from_numpy(psi).to(dev)
        y = torch.empty_like(x)
        gpu_lib.op_apply_block(op, y, x, k, dagger=dag)
        err = np.abs(y.cpu().numpy() - ref).max() / np.abs(ref).max()
        assert err <= 1e-12, (k, dag, err)
        x32 = x.to(torch.complex64)
        y32 = torch.empty_like(x32)
        gpu_lib.op_apply_block(op, y32, x32, k, dagger=dag, prec="fp32")
        ref32 = np.stack([f(U, psi[c].astype(np.complex64).astype(np.complex128), kappa, dims) for c in range(k)])
        assert np.abs(y32.cpu().numpy() - ref32).max() / np.abs(ref32).max() < 5e-7
        xb = torch.view_as_real(x).to(torch.bfloat16).contiguous()
        yb = torch.empty_like(xb)
        gpu_lib.op_apply_block(op, yb, xb, k, dagger=dag, prec="bf16")
        psib = torch.view_as_complex(xb.cpu().to(torch.float64)).numpy()
        refb = np.stack([f(U, psib[c], kappa, dims) for c in range(k)])
        got = torch.view_as_complex(yb.cpu().to(torch.float64)).numpy()
        assert np.abs(got - refb).max() / np.abs(refb).max() < 4 * 2.0**-9
    with pytest.raises(gpu_lib.EbicgError):
        gpu_lib.op_apply_block(op, torch.empty(3 * 12 * V, dtype=torch.complex128, device=dev),
                               torch.zeros(3 * 12 * V, dtype=torch.complex128, device=dev), 3)


@pytest.mark.parametrize("eo", [False, True])
def test_block_tile_forms_and_tuner(gpu_lib, eo):
    """Every tile form of the multi-RHS stencil (global reads in site order,
    LDS-staged tile, global reads in 8x8x4x4, 8x8x8x8 and 4x4x4x4 bricks,
    unfenced global reads, t-marching boxes; the even-odd hop has the first
    two), forced per precision and k, against
    the oracle: FP64 at 1e-12 (D, or Dhat for an even-odd operator), FP32 / BF16
    storage against the first form within their rounding; forms the operator
    does not admit are rejected; then the autotuner's table names a form per k
    and a best k."""
    import torch

    dims, kappa = (8, 8, 8, 8), 0.122
    V = synth.volume(dims)
    U = synth.random_su3_links(dims, 0.3, 91)
    op = gpu_lib.op_create(U, kappa, dims, eo=eo)
    par = W.parity(dims)
    forms = (0, 1) if eo else (0, 1, 2, 3, 4, 5, 6)
    for k in (2, 16):
        psi = np.stack([synth.gaussian_spinor(V, 70 + c) for c in range(k)])
        x = torch.from_numpy(psi).to("cuda:0")
        if eo:
            ref = np.stack([W.apply_Dhat(U, psi[c][par == 0], kappa, dims) for c in range(k)])
        else:
            ref = np.stack([W.apply_D(U, psi[c], kappa, dims) for c in range(k)])
        scale = np.abs(ref).max()
        for prec, bound in (("fp64", 1e-12), ("fp32", 2e-6), ("bf16", 8 * 2.0**-9)):
            outs = []
            for stage in forms:
                gpu_lib.op_batch_set_tile(op, prec, k, stage)
                if eo:
                    y = torch.full_like(x, 7.0)
                    gpu_lib.op_apply_schur_block(op, y, x, k, prec=prec)
                    got = y.cpu().numpy().reshape(k, V, 4, 3)
                    assert np.abs(got[:, par == 1]).max() == 0.0
                    got = got[:, par == 0]
                elif prec == "bf16":
                    xb = torch.view_as_real(x).to(torch.bfloat16).contiguous()
                    yb = torch.empty_like(xb)
                    gpu_lib.op_apply_block(op, yb, xb, k, prec="bf16")
                    got = torch.view_as_complex(yb.cpu().to(torch.float64)).numpy().reshape(k, V, 4, 3)
                else:
                    xx = x if prec == "fp64" else x.to(torch.complex64)
                    y = torch.empty_like(xx)
                    gpu_lib.op_apply_block(op, y, xx, k, prec=prec)
                    got = y.cpu().numpy().astype(np.complex128).reshape(k, V, 4, 3)
                outs.append(got)
                if prec == "fp64":
                    err = np.abs(got - ref).max() / scale
                    assert err <= 1e-12, (k, stage, err)
            d = max(np.abs(o - outs[0]).max() / scale for o in outs[1:])
            print(f"eo={eo} k={k} {prec}: largest difference between tile forms {d:.2e}")
            assert d <= bound, (k, prec, d)
            gpu_lib.op_batch_set_tile(op, prec, k, -1)
    for bad in ((3, 1), (4, 2) if eo else (4, 7), (4, 6) if eo else (4, -2)):
        with pytest.raises(gpu_lib.EbicgError):
            gpu_lib.op_batch_set_tile(op, "fp32", *bad)
    odd = gpu_lib.op_create(synth.random_su3_links((4, 4, 4, 8), 0.3, 92), kappa, (4, 4, 4, 8))
    with pytest.raises(gpu_lib.EbicgError):
        gpu_lib.op_batch_set_tile(odd, "fp32", 4, 2)  # the 8-wide brick does not divide Lx = 4
    with pytest.raises(gpu_lib.EbicgError):
        gpu_lib.op_batch_set_tile(odd, "fp32", 2, 6)  # a 4 x 4 x 4 box of 2 columns is half a block
    gpu_lib.op_batch_set_tile(odd, "fp32", 4, 4)
    gpu_lib.op_batch_set_tile(odd, "fp32", 4, 6)
    for prec in ("fp32", "bf16"):
        t = gpu_lib.op_batch_tune(op, prec)
        print(prec, t)
        assert t["k"] in (1, 2, 4, 8, 16)
        assert all(s in forms for s in t["stage"].values())
        for kk, ms in t["ms_per_rhs"].items():
            # one column: the two forms of the one-at-a-time solver (staged, t-marching)
            timed = tuple(f for f in (1, 6) if f in forms) if kk == 1 else forms
            assert all(ms[f] > 0 for f in timed) and all(ms[f] == 0 for f in range(7) if f not in timed)
            assert ms[t["stage"][kk]] == min(ms[f] for f in timed)


def test_block_tile_forms_full_size_sampled(gpu_lib):
    """16^3 x 32 (the incremental-eigBiCG lattice), FP64 multi-RHS stencil with
    k = 16 in every tile form (the bricks cover the lattice in several bricks
    per dimension): sampled sites of every column against the per-site
    oracle at 1e-12."""
    import torch

    dims, kappa = (16, 16, 16, 32), 0.122
    U, op, dev = _setup(gpu_lib, dims, kappa, seed=synth.gauge_seed(1))
    V = synth.volume(dims)
    k = 16
    psi = np.stack([synth.z2_source(V, synth.rhs_seed(0, 200 + c)) for c in range(k)])
    x = torch.from_numpy(psi).to(dev)
    sites = _sample_sites(dims, n=12)
    refs = [W.apply_D_sites(U, psi[c], kappa, dims, sites) for c in range(k)]
    scale = max(np.abs(r).max() for r in refs)
    for stage in (0, 1, 2, 3, 4, 5, 6):
        gpu_lib.op_batch_set_tile(op, "fp64", k, stage)
        y = torch.empty_like(x)
        gpu_lib.op_apply_block(op, y, x, k)
        got = y.cpu().numpy().reshape(k, V, 4, 3)
        err = max(np.abs(got[c][sites] - refs[c]).max() for c in range(k)) / scale
        print(f"tile form {stage}: {err:.2e}")
        assert err <= 1e-12, (stage, err)


def test_dslash_block_32x64_sampled(gpu_lib):
    """32^3 x 64 (the batching lattice), FP32 storage, k = 16 columns: the
    8x8x8x8 bricks, form 0, the unfenced form and the t-marching boxes, at sampled
    sites of every column against the per-site oracle on the rounded input
    (FP32 rounding bound 5e-7 of the largest entry); then FP64 with one column
    in the t-marching and the staged form at the chunk and box boundaries."""
    import torch

    dims, kappa = (32, 32, 32, 64), 0.123
    V = synth.volume(dims)
    U = synth.random_su3_links(dims, 0.3, synth.gauge_seed(3))
    op = gpu_lib.op_create(U, kappa, dims)
    k = 16
    psi = np.stack([synth.z2_source(V, synth.rhs_seed(3, 300 + c)) for c in range(k)]).astype(np.complex64)
    x = torch.from_numpy(psi).to("cuda:0")
    sites = _sample_sites(dims, n=10, seed=3)
    U32 = U.astype(np.complex64).astype(np.complex128)
    refs = [W.apply_D_sites(U32, psi[c].astype(np.complex128), kappa, dims, sites) for c in range(k)]
    scale = max(np.abs(r).max() for r in refs)
    for stage in (3, 0, 5, 6):
        gpu_lib.op_batch_set_tile(op, "fp32", k, stage)
        y = torch.empty_like(x)
        gpu_lib.op_apply_block(op, y, x, k, prec="fp32")
        got = y.cpu().numpy().reshape(k, V, 4, 3)
        err = max(np.abs(got[c][sites] - refs[c]).max() for c in range(k)) / scale
        print(f"32^3 x 64, tile form {stage}: {err:.2e}")
        assert err <= 5e-7, (stage, err)
    del x, y
    _one_column_march_fp64(gpu_lib, op, U, dims, kappa, 14)
    gpu_lib.op_destroy(op)
