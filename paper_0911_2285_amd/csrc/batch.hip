// Multi-RHS kernels: the Wilson-Dirac stencil and the BiCGStab passes over a
// batch of KC right-hand sides.
//
// Batch layout: KC spinors interleaved as the fastest index, element
// (component c, site s, column col) at (c V + s) KC + col.  Thread u of a
// launch works on column u % KC of site u / KC: the KC lanes of one site read
// the same link addresses, which the memory pipeline merges into one request,
// so a link is fetched from HBM once for KC sources (links are 60% of a
// single-RHS dslash's bytes); spinor accesses of a wavefront stay contiguous.
//
// Every column is an independent BiCGStab recurrence (Alg. Incremental
// eigBiCG, step 3, without DefTol): its own scalars in the history at index
// j KC + col, its own stop flag in KrylovState[col], and per-column
// reductions (block_partial_cols / sum_partials).  A column that has stopped
// is skipped by every later kernel; the others continue.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_common.h"
#include "kernel_util.h"
#include "kernels.h"
#include "slot.h"
#include "stencil.h"

namespace ebicg {
namespace {

template <int N>
__device__ __forceinline__ double pick(const double (&v)[N], int i) {
  double r = 0.0;
#pragma unroll
  for (int k = 0; k < N; ++k)
    if (k == i) r = v[k];
  return r;
}

__device__ __forceinline__ bool col_active(const KrylovState *K, int col, int j) {
  return !(K[col].stopped && j > K[col].stop_at);
}

// Tile form of the batched stencils: STG = true stages each block's tile of
// kBlock / KC sites in LDS (stencil.h), false reads every neighbour from
// global memory.  Staging pays when a tile holds many sites or the entries
// are small; the default (stage < 0 at launch) is the rule measured on
// MI355X: stage for one column at every precision and for BF16 at every
// batch size.  The batch autotuner times both forms per precision and k.
template <typename S, int KC>
constexpr bool kStage = KC == 1 || std::is_same<S, bf16c>::value;
// (staged, fenced) for a tile form: form 1 (or the rule) stages in LDS;
// form 5 reads globally without fences between the hops; the rest read
// globally with one hop's loads in flight at a time.
template <typename S, int KC, typename F>
void dispatch_stage(int stage, F &&f) {
  if (stage < 0 ? kStage<S, KC> : stage == 1)
    f(std::true_type{}, std::true_type{});
  else if (stage == 5)
    f(std::false_type{}, std::false_type{});
  else
    f(std::false_type{}, std::true_type{});
}
// Site order of the global-read form.  Linear order puts a site's
// t-neighbour Lx Ly Lz sites back in the traversal; with k columns of 12
// entries per site that distance outgrows an XCD's L2 at large k (32^3 x 64,
// FP32, k = 16: 48 MB), and the neighbour reads miss.  Visiting the lattice
// brick after brick (bx x by x bz x bt sites, x fastest inside a brick and
// across bricks) keeps most neighbours of the sites in flight inside the
// brick.  At k >= 4 a site's k entries of one component fill a whole cache
// line, so bricks narrower than Lx cost no coalescing.
struct Brick {
  int bx, by, bz, bt;  // bx = 0: linear order
};
inline Brick brick_of(int stage) {
  switch (stage) {
    case 2: return Brick{8, 8, 4, 4};
    case 3: return Brick{8, 8, 8, 8};
    case 4: return Brick{4, 4, 4, 4};
    default: return Brick{0, 0, 0, 0};
  }
}
__device__ __forceinline__ int brick_site(int q, const Geom &g, Brick b) {
  if (b.bx == 0) return q;
  const int bsize = b.bx * b.by * b.bz * b.bt;
  int k = q / bsize, r = q - k * bsize;
  const int nbx = g.lx / b.bx, nby = g.ly / b.by, nbz = g.lz / b.bz;
  const int ix = k % nbx;
  k /= nbx;
  const int iy = k % nby;
  k /= nby;
  const int iz = k % nbz, it = k / nbz;
  const int xx = r % b.bx;
  r /= b.bx;
  const int yy = r % b.by;
  r /= b.by;
  const int zz = r % b.bz, tt = r / b.bz;
  return (ix * b.bx + xx) + g.lx * ((iy * b.by + yy) + g.ly * ((iz * b.bz + zz) + g.lz * (it * b.bt + tt)));
}

template <typename S, int KC, int SF, bool STG, bool FENCE>
__global__ void __launch_bounds__(kBlock)
    k_bdslash(S *__restrict__ out, const S *__restrict__ in, const S *__restrict__ U, Geom g, double kappa, Brick bk) {
  using R = typename Store<S>::R;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const R k = R(kappa);
  if constexpr (STG) {
    __shared__ S tile[12 * kBlock];
    constexpr int spt = kBlock / KC;  // sites per tile
    const int ntiles = (g.V + spt - 1) / spt, col = threadIdx.x % KC;
    for (int T = lb; T < ntiles; T += gridDim.x) {
      const int s0 = T * spt, s = s0 + threadIdx.x / KC;
      __syncthreads();
      stage_tile<S, KC>(tile, in, s0, g.V);
      __syncthreads();
      if (s >= g.V) continue;
      cx<R> acc[12];
      hopping_t<SF, S>(acc, TileSrc<S, KC>{in + col, tile + col, s0, g.V}, U, g, s);
#pragma unroll
      for (int c = 0; c < 12; ++c)
        Store<S>::st(out, (size_t(c) * g.V + s) * KC + col,
                     Store<S>::ld(tile, size_t(c) * kBlock + threadIdx.x) - k * acc[c]);
    }
  } else {
    const size_t n = size_t(g.V) * KC;
    for (size_t u = size_t(lb) * kBlock + threadIdx.x; u < n; u += size_t(gridDim.x) * kBlock) {
      const int s = brick_site(int(u / KC), g, bk), col = int(u % KC);
      cx<R> acc[12];
      hopping<SF, S, KC, FENCE>(acc, in + col, U, g, s);
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        const size_t i = (size_t(c) * g.V + s) * KC + col;
        Store<S>::st(out, i, Store<S>::ld(in, i) - k * acc[c]);
      }
    }
  }
}

// ---- tile form 6: t-marching ---------------------------------------------------
// A unit of work is a box of rx x ry x rz sites (x fastest) times a chunk of
// tc consecutive time slices.  Its threads, one per (site of the box,
// column) with the columns fastest, walk the chunk in t.  A thread keeps its
// site's spinor at the current and the next slice at hand (registers; the
// current one in the block's LDS for FP64), so the t hops read no
// neighbour: the forward hop projects the next slice, and the backward hop
// of slice t + 1 (U_t^+ times the projection of slice t) is formed while
// slice t is at hand and carried to the next step.  The
// x, y, z neighbours come from global memory; the threads of one box step
// through the same slices together, so those reads hit the slices the box
// itself has just loaded into L2 and only the box's faces come from beyond
// it.  The blocks of one unit are consecutive in the XCD-remapped order, so
// a unit runs on one XCD (at 32^3 x 64 each XCD holds one box).
struct March {
  int rx, ry, rz, tc;  // rx = 0: the form does not fit the lattice and k
};
constexpr int kMarchForm = kMarchTile;
// Largest divisor of n not above cap.
inline int divisor_below(int n, int cap) {
  for (int d = cap < n ? cap : n; d > 1; --d)
    if (n % d == 0) return d;
  return 1;
}
// Box and chunk for k columns.  The box caps are the fastest measured on
// MI355X at 32^3 x 64 (FP32): 16 x 16 x 8 sites for k = 16, 32 x 16 x 8 for
// k = 2 .. 8, 32 x 32 x 8 for one column; each extent is the largest divisor
// of the lattice extent within its cap.  A box must hold a whole number of
// blocks; chunks are cut from the full t extent until the launch has at least
// 512 blocks (two per CU), but no shorter than 8 slices: a chunk re-reads the
// slice before it, and at 24^3 x 64 (FP64, one column) 8-slice chunks on 432
// blocks beat 4-slice chunks on 864 (264 against 286 us).  The records of the
// reducing variants (three per column and block) must fit one region.
inline March march_shape(const Geom &g, int kc) {
  const int cy = kc == 1 ? 32 : 16, cx = kc >= 16 ? 16 : 32;
  March m{divisor_below(g.lx, cx), divisor_below(g.ly, cy), divisor_below(g.lz, 8), g.lt};
  const long long box = (long long)m.rx * m.ry * m.rz;
  if ((box * kc) % kBlock != 0) return March{};
  auto blocks = [&](int tc) { return (long long)g.V / tc * kc / kBlock; };
  while (m.tc % 2 == 0 && m.tc > 8 && blocks(m.tc) < 512) m.tc /= 2;
  if (blocks(m.tc) * kc * 3 > (long long)kRegion) return March{};
  return m;
}
inline int march_blocks(const Geom &g, int kc, const March &m) { return int((long long)g.V / m.tc * kc / kBlock); }
// Records (blocks) a batched stencil pass of tile form `stage` writes with nv
// partials per column: what its consumer sums.
inline int stencil_records(const Geom &g, int kc, int nv, int stage) {
  return stage == kMarchForm ? march_blocks(g, kc, march_shape(g, kc)) : batch_stencil_grid(g.V, kc, nv);
}

// One thread's walk of the t-marching form: site (x, y, z) of its box, column
// col, through the slices of chunk `chunk`: out = in - kappa hop at every
// slice, and epi(c, i, o, in_c) for each of the 12 components (i the entry's
// index, o the output, in_c the input at the site).  FP64: the spinor of the
// current slice waits in the block's LDS (cbuf: [12][kBlock], each thread its
// own column) instead of registers, which keeps the walk's live state within
// the registers of two waves per SIMD.
template <typename S, int KC, int SF, typename Epi>
__device__ __forceinline__ void march_walk(S *__restrict__ out, const S *__restrict__ in, const S *__restrict__ U,
                                           const Geom &g, typename Store<S>::R k, const March &m, int x, int y, int z,
                                           int col, int chunk, double2 *cbuf, Epi &&epi) {
  using R = typename Store<S>::R;
  constexpr bool kL = std::is_same<R, double>::value;
  const int Vs = g.lx * g.ly * g.lz, xyz = x + g.lx * (y + g.ly * z);
  const int sy = g.lx, sz = g.lx * g.ly;
  const int xf = x == g.lx - 1 ? -(g.lx - 1) : 1, xb = x == 0 ? g.lx - 1 : -1;
  const int yf = y == g.ly - 1 ? -(g.ly - 1) * sy : sy, yb = y == 0 ? (g.ly - 1) * sy : -sy;
  const int zf = z == g.lz - 1 ? -(g.lz - 1) * sz : sz, zb = z == 0 ? (g.lz - 1) * sz : -sz;
  const S *inc = in + col;
  auto xyz_hops = [&](cx<R> (&acc)[12], int s) {
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = {0, 0};
    hop_dir<2, SF, S, KC, true>(acc, inc, U, g.V, s, s + zf, s + zb);
    hop_dir<0, SF, S, KC, true>(acc, inc, U, g.V, s, s + xf, s + xb);
    hop_dir<1, SF, S, KC, true>(acc, inc, U, g.V, s, s + yf, s + yb);
  };
  // the current slice's spinor: registers (FP32, BF16) or the LDS column (FP64)
  cx<R> creg[kL ? 1 : 12];
  auto cen = [&](int c) -> cx<R> {
    if constexpr (kL) {
      const double2 v = cbuf[c * kBlock + threadIdx.x];
      return {v.x, v.y};
    } else {
      return creg[c];
    }
  };
  auto set_cen = [&](const cx<R> (&p)[12]) {
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      if constexpr (kL)
        cbuf[c * kBlock + threadIdx.x] = make_double2(p[c].x, p[c].y);
      else
        creg[c] = p[c];
    }
  };
  const int t0 = chunk * m.tc, t1 = t0 + m.tc;
  cx<R> acc[12], carry[6];
  {
    const int s = xyz + Vs * t0, sp = xyz + Vs * (t0 == 0 ? g.lt - 1 : t0 - 1);
    cx<R> c0[12];
    load_spinor<S, KC>(c0, inc, g.V, s);
    set_cen(c0);
    cx<R> h[6];
    load_project<3, -SF, S, KC>(h, inc, g.V, sp);
    mult_t<true, S>(carry, h, U, g.V, sp);
    xyz_hops(acc, s);
  }
  for (int t = t0; t < t1; ++t) {
    int s = xyz + Vs * t, sn = xyz + Vs * (t == g.lt - 1 ? 0 : t + 1);
    // opaque site indices: the addresses are formed from them in each step
    // instead of being carried across steps in registers
    asm volatile("" : "+v"(s), "+v"(sn));
    cx<R> nxt[12];
    load_spinor<S, KC>(nxt, inc, g.V, sn);
    {
      cx<R> h[6], w[6];
      project_t<SF>(h, nxt);
      mult_t<false, S>(w, h, U, g.V, s);
      recon_t<SF>(acc, w);
      recon_t<-SF>(acc, carry);
#pragma unroll
      for (int a = 0; a < 3; ++a) {  // the t projector (1 - SF gamma_t) of the current slice
        h[a] = cen(a) + sgn<-SF>(cen(6 + a));
        h[3 + a] = cen(3 + a) + sgn<-SF>(cen(9 + a));
      }
      mult_t<true, S>(carry, h, U, g.V, s);
    }
    hop_fence();
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const size_t i = (size_t(c) * g.V + s) * KC + col;
      const cx<R> ci = cen(c);
      const cx<R> o = ci - k * acc[c];
      Store<S>::st(out, i, o);
      epi(c, i, o, ci);
    }
    set_cen(nxt);
    if (t + 1 < t1) xyz_hops(acc, sn);
  }
}

// Box coordinates of thread u (columns fastest) of a unit of box `box`.
struct MarchSite {
  int x, y, z, col;
};
template <int KC>
__device__ __forceinline__ MarchSite march_site(const Geom &g, const March &m, int box, int u) {
  const int col = u % KC, q = u / KC;
  const int nbx = g.lx / m.rx, nby = g.ly / m.ry;
  return {(box % nbx) * m.rx + q % m.rx, ((box / nbx) % nby) * m.ry + (q / m.rx) % m.ry,
          (box / (nbx * nby)) * m.rz + q / (m.rx * m.ry), col};
}

// EPI 0: out = in - kappa hop (the operator); 1: also the partials of
// (rhat, out) per column (the v pass of BiCGStab); 2: also (out, in) and
// (out, out) (the t pass).  Stopped columns skip the work (EPI > 0).
template <typename S, int KC, int SF, int EPI>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2, 2)))
    k_bmarch(S *__restrict__ out, const S *__restrict__ in, const S *__restrict__ U, Geom g, double kappa, March m,
             const S *__restrict__ rhat, int j, const KrylovState *K, double *__restrict__ part) {
  using R = typename Store<S>::R;
  constexpr int NV = EPI == 2 ? 3 : 2;
  const int bpu = m.rx * m.ry * m.rz * KC / kBlock;  // blocks per unit
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int unit = lb / bpu, u = (lb - unit * bpu) * kBlock + threadIdx.x;
  const int nch = g.lt / m.tc, box = unit / nch, chunk = unit - box * nch;
  const MarchSite ms = march_site<KC>(g, m, box, u);
  double d[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) d[i] = 0.0;
  bool act = true;
  if constexpr (EPI != 0) act = col_active(K, ms.col, j);
  __shared__ double2 cbuf[std::is_same<R, double>::value ? 12 * kBlock : 1];
  if (act)
    march_walk<S, KC, SF>(out, in, U, g, R(kappa), m, ms.x, ms.y, ms.z, ms.col, chunk, cbuf,
                          [&](int, size_t i, cx<R> o, cx<R> si) {
                            if constexpr (EPI == 1) {
                              const cx<R> hh = Store<S>::ld(rhat, i);
                              d[0] += double(hh.x) * o.x + double(hh.y) * o.y;
                              d[1] += double(hh.x) * o.y - double(hh.y) * o.x;
                            } else if constexpr (EPI == 2) {
                              d[0] += double(o.x) * si.x + double(o.y) * si.y;
                              d[1] += double(o.x) * si.y - double(o.y) * si.x;
                              d[NV - 1] += double(o.x) * o.x + double(o.y) * o.y;
                            }
                          });
  if constexpr (EPI != 0) block_partial_cols<NV, KC, kBlock>(d, part, blockIdx.x);
}

// The BiCG matvec in the t-marching form: Ap = D p with the partials of
// sigma = (phat, Ap), and Adp = D^+ phat.  Work item w is a unit (box and
// chunk) of D for even w and the same unit of D^+ for odd w, so the two walk
// the same slices on the same XCD at the same time and share the link loads
// in its L2.  G5 (the gamma5-Hermitian form): D units only, sigma =
// (gamma5 p, Ap) from the input at the site.  One record per block.
template <bool G5>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2, 2)))
    k_bicg_matvec_march(double2 *__restrict__ Ap, double2 *__restrict__ Adp, const double2 *__restrict__ p,
                        const double2 *__restrict__ ph, const double2 *__restrict__ U, Geom g, double kappa, March m,
                        int j, const KrylovState *S, double *__restrict__ part) {
  if (skip_iter(S, j)) return;
  const int bpu = m.rx * m.ry * m.rz / kBlock;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int item = lb / bpu, u = (lb - item * bpu) * kBlock + threadIdx.x;
  const int unit = G5 ? item : item >> 1;
  const bool adj = !G5 && (item & 1) != 0;
  const int nch = g.lt / m.tc, box = unit / nch, chunk = unit - box * nch;
  const MarchSite ms = march_site<1>(g, m, box, u);
  double d[2] = {0.0, 0.0};
  __shared__ double2 cbuf[12 * kBlock];
  if (!adj) {
    march_walk<double2, 1, -1>(Ap, p, U, g, kappa, m, ms.x, ms.y, ms.z, 0, chunk, cbuf,
                               [&](int c, size_t i, cx<double> o, cx<double> pv) {
                                 cx<double> dd;
                                 if constexpr (G5)
                                   dd = c < 6 ? cmulc(pv, o) : -cmulc(pv, o);
                                 else
                                   dd = cmulc(Store<double2>::ld(ph, i), o);
                                 d[0] += dd.x;
                                 d[1] += dd.y;
                               });
  } else {
    march_walk<double2, 1, +1>(Adp, ph, U, g, kappa, m, ms.x, ms.y, ms.z, 0, chunk, cbuf,
                               [](int, size_t, cx<double>, cx<double>) {});
  }
  block_partial<2, kBlock>(d, part, blockIdx.x);
}

// rhat = p = r; partials of ||r_col||^2
template <typename S, int KC>
__global__ void __launch_bounds__(kBlock)
    k_bstab_init(S *__restrict__ rhat, S *__restrict__ p, const S *__restrict__ r, size_t n,
                 double *__restrict__ part) {
  double v[1] = {0.0};
  for (size_t u = size_t(blockIdx.x) * kBlock + threadIdx.x; u < n; u += size_t(gridDim.x) * kBlock) {
    const auto rv = Store<S>::ld(r, u);
    Store<S>::st(rhat, u, rv);
    Store<S>::st(p, u, rv);
    v[0] += double(rv.x) * rv.x + double(rv.y) * rv.y;
  }
  block_partial_cols<1, KC, kBlock>(v, part, blockIdx.x);
}

template <int KC>
__global__ void __launch_bounds__(kBlock)
    k_bstab_init_finish(const double *__restrict__ part, int nblk, const double *__restrict__ tol_abs, int maxiter,
                        KrylovState *K, KrylovHistory h) {
  double v[KC];
  sum_partials<KC, kBlock>(part, nblk, v);
  if (threadIdx.x >= KC) return;
  const int col = threadIdx.x;
  const double rr = pick(v, col), rn = sqrt(rr);
  h.rho[col] = make_double2(rr, 0.0);
  h.rn[col] = rn;
  KrylovState &k = K[col];
  k.bnorm = 0.0;
  k.tol_abs = tol_abs[col];
  k.def_thr = 0.0;
  k.rnorm = rn;
  k.maxiter = maxiter;
  k.stopped = 0;
  k.stop_at = 0;
  k.reason = 0;
  if (rn <= tol_abs[col]) {
    k.stopped = 1;
    k.reason = 1;
  }
}

// v = D p; partials of (rhat, v) per column
template <typename S, int KC, bool STG, bool FENCE>
__global__ void __launch_bounds__(kBlock)
    k_bstab_v(S *__restrict__ vout, const S *__restrict__ p, const S *__restrict__ rhat, const S *__restrict__ U,
              Geom g, double kappa, int j, const KrylovState *K, double *__restrict__ part, Brick bk) {
  using R = typename Store<S>::R;
  const int col = threadIdx.x % KC;
  const bool act = col_active(K, col, j);
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const R k = R(kappa);
  double d[2] = {0.0, 0.0};
  auto epilogue = [&](int s, const cx<R> (&acc)[12], auto center) {
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const size_t i = (size_t(c) * g.V + s) * KC + col;
      const cx<R> o = center(c, i) - k * acc[c];
      Store<S>::st(vout, i, o);
      const cx<R> hh = Store<S>::ld(rhat, i);
      d[0] += double(hh.x) * o.x + double(hh.y) * o.y;
      d[1] += double(hh.x) * o.y - double(hh.y) * o.x;
    }
  };
  if constexpr (STG) {
    __shared__ S tile[12 * kBlock];
    constexpr int spt = kBlock / KC;
    const int ntiles = (g.V + spt - 1) / spt;
    for (int T = lb; T < ntiles; T += gridDim.x) {
      const int s0 = T * spt, s = s0 + threadIdx.x / KC;
      __syncthreads();
      stage_tile<S, KC>(tile, p, s0, g.V);
      __syncthreads();
      if (!act || s >= g.V) continue;
      cx<R> acc[12];
      hopping_t<-1, S>(acc, TileSrc<S, KC>{p + col, tile + col, s0, g.V}, U, g, s);
      epilogue(s, acc, [&](int c, size_t) { return Store<S>::ld(tile, size_t(c) * kBlock + threadIdx.x); });
    }
  } else if (act) {
    const size_t n = size_t(g.V) * KC;
    for (size_t u = size_t(lb) * kBlock + threadIdx.x; u < n; u += size_t(gridDim.x) * kBlock) {
      const int s = brick_site(int(u / KC), g, bk);
      cx<R> acc[12];
      hopping<-1, S, KC, FENCE>(acc, p + col, U, g, s);
      epilogue(s, acc, [&](int, size_t i) { return Store<S>::ld(p, i); });
    }
  }
  block_partial_cols<2, KC, kBlock>(d, part, blockIdx.x);
}

// alpha_j = rho_{j-1} / (rhat, v) per column (one block); a vanishing or
// non-finite (rhat, v) stops the column (breakdown).
template <int KC>
__global__ void __launch_bounds__(kBlock)
    k_bfin_alpha(const double *__restrict__ part, int nblk, int j, KrylovState *K, KrylovHistory h) {
  double d[2 * KC];
  sum_partials<2 * KC, kBlock>(part, nblk, d);
  if (threadIdx.x >= KC) return;
  const int col = threadIdx.x;
  if (!col_active(K, col, j)) return;
  const cx<double> den{pick(d, 2 * col), pick(d, 2 * col + 1)};
  const double dd = den.x * den.x + den.y * den.y;
  if (!(dd > 0.0) || !isfinite(dd)) {
    K[col].stopped = 1;
    K[col].stop_at = j - 1;
    K[col].reason = 2;
    return;
  }
  h.alpha[j * KC + col] = d2(cdiv(c2(h.rho[(j - 1) * KC + col]), den));
}

// s = r - alpha v
template <typename S, int KC>
__global__ void __launch_bounds__(kBlock)
    k_bstab_s(S *__restrict__ sv, const S *__restrict__ r, const S *__restrict__ v, size_t n, int j,
              const KrylovState *K, KrylovHistory h) {
  using R = typename Store<S>::R;
  const int col = threadIdx.x % KC;
  if (!col_active(K, col, j)) return;
  const cx<double> al = c2(h.alpha[j * KC + col]);
  const cx<R> a{R(al.x), R(al.y)};
  for (size_t u = size_t(blockIdx.x) * kBlock + threadIdx.x; u < n; u += size_t(gridDim.x) * kBlock)
    Store<S>::st(sv, u, Store<S>::ld(r, u) - a * Store<S>::ld(v, u));
}

// t = D s; partials of (t, s), (t, t) per column
template <typename S, int KC, bool STG, bool FENCE>
__global__ void __launch_bounds__(kBlock)
    k_bstab_t(S *__restrict__ tout, const S *__restrict__ sv, const S *__restrict__ U, Geom g, double kappa, int j,
              const KrylovState *K, double *__restrict__ part, Brick bk) {
  using R = typename Store<S>::R;
  const int col = threadIdx.x % KC;
  const bool act = col_active(K, col, j);
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const R k = R(kappa);
  double d[3] = {0.0, 0.0, 0.0};
  auto epilogue = [&](int s, const cx<R> (&acc)[12], auto center) {
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const size_t i = (size_t(c) * g.V + s) * KC + col;
      const cx<R> si = center(c, i);
      const cx<R> o = si - k * acc[c];
      Store<S>::st(tout, i, o);
      d[0] += double(o.x) * si.x + double(o.y) * si.y;
      d[1] += double(o.x) * si.y - double(o.y) * si.x;
      d[2] += double(o.x) * o.x + double(o.y) * o.y;
    }
  };
  if constexpr (STG) {
    __shared__ S tile[12 * kBlock];
    constexpr int spt = kBlock / KC;
    const int ntiles = (g.V + spt - 1) / spt;
    for (int T = lb; T < ntiles; T += gridDim.x) {
      const int s0 = T * spt, s = s0 + threadIdx.x / KC;
      __syncthreads();
      stage_tile<S, KC>(tile, sv, s0, g.V);
      __syncthreads();
      if (!act || s >= g.V) continue;
      cx<R> acc[12];
      hopping_t<-1, S>(acc, TileSrc<S, KC>{sv + col, tile + col, s0, g.V}, U, g, s);
      epilogue(s, acc, [&](int c, size_t) { return Store<S>::ld(tile, size_t(c) * kBlock + threadIdx.x); });
    }
  } else if (act) {
    const size_t n = size_t(g.V) * KC;
    for (size_t u = size_t(lb) * kBlock + threadIdx.x; u < n; u += size_t(gridDim.x) * kBlock) {
      const int s = brick_site(int(u / KC), g, bk);
      cx<R> acc[12];
      hopping<-1, S, KC, FENCE>(acc, sv + col, U, g, s);
      epilogue(s, acc, [&](int, size_t i) { return Store<S>::ld(sv, i); });
    }
  }
  block_partial_cols<3, KC, kBlock>(d, part, blockIdx.x);
}

// omega_j = (t, s) / (t, t) per column (one block); (t, t) = 0 stops the column.
template <int KC>
__global__ void __launch_bounds__(kBlock)
    k_bfin_omega(const double *__restrict__ part, int nblk, int j, KrylovState *K, KrylovHistory h) {
  double d[3 * KC];
  sum_partials<3 * KC, kBlock>(part, nblk, d);
  if (threadIdx.x >= KC) return;
  const int col = threadIdx.x;
  if (!col_active(K, col, j)) return;
  const double tt = pick(d, 3 * col + 2);
  if (!(tt > 0.0)) {
    K[col].stopped = 1;
    K[col].stop_at = j - 1;
    K[col].reason = 2;
    return;
  }
  h.omega[j * KC + col] = make_double2(pick(d, 3 * col) / tt, pick(d, 3 * col + 1) / tt);
}

// x += alpha p + omega s; r = s - omega t; partials of (rhat, r), ||r||^2
template <typename S, int KC>
__global__ void __launch_bounds__(kBlock)
    k_bstab_xr(S *__restrict__ x, S *__restrict__ r, const S *__restrict__ p, const S *__restrict__ sv,
               const S *__restrict__ t, const S *__restrict__ rhat, size_t n, int j, const KrylovState *K,
               KrylovHistory h, double *__restrict__ part) {
  using R = typename Store<S>::R;
  const int col = threadIdx.x % KC;
  double e[3] = {0.0, 0.0, 0.0};
  if (col_active(K, col, j)) {
    const cx<double> al = c2(h.alpha[j * KC + col]), om = c2(h.omega[j * KC + col]);
    const cx<R> a{R(al.x), R(al.y)}, w{R(om.x), R(om.y)};
    for (size_t u = size_t(blockIdx.x) * kBlock + threadIdx.x; u < n; u += size_t(gridDim.x) * kBlock) {
      const cx<R> si = Store<S>::ld(sv, u);
      Store<S>::st(x, u, Store<S>::ld(x, u) + a * Store<S>::ld(p, u) + w * si);
      const cx<R> ri = si - w * Store<S>::ld(t, u);
      Store<S>::st(r, u, ri);
      const cx<R> hh = Store<S>::ld(rhat, u);
      e[0] += double(hh.x) * ri.x + double(hh.y) * ri.y;
      e[1] += double(hh.x) * ri.y - double(hh.y) * ri.x;
      e[2] += double(ri.x) * ri.x + double(ri.y) * ri.y;
    }
  }
  block_partial_cols<3, KC, kBlock>(e, part, blockIdx.x);
}

// rho_j, ||r_j||, beta_j = (rho_j / rho_{j-1}) (alpha_j / omega_j) and the stop
// tests per column (one block)
template <int KC>
__global__ void __launch_bounds__(kBlock)
    k_bfin_beta(const double *__restrict__ part, int nblk, int j, KrylovState *K, KrylovHistory h) {
  double d[3 * KC];
  sum_partials<3 * KC, kBlock>(part, nblk, d);
  if (threadIdx.x >= KC) return;
  const int col = threadIdx.x;
  if (!col_active(K, col, j)) return;
  const cx<double> rho{pick(d, 3 * col), pick(d, 3 * col + 1)};
  const cx<double> be = cdiv(rho, c2(h.rho[(j - 1) * KC + col])) *
                        cdiv(c2(h.alpha[j * KC + col]), c2(h.omega[j * KC + col]));
  const double rnorm = sqrt(pick(d, 3 * col + 2));
  KrylovState &k = K[col];
  h.rho[j * KC + col] = d2(rho);
  h.beta[j * KC + col] = d2(be);
  h.rn[j * KC + col] = rnorm;
  k.rnorm = rnorm;
  if (rnorm <= k.tol_abs) {
    k.stopped = 1;
    k.stop_at = j;
    k.reason = 1;
  } else if (rho.x == 0.0 && rho.y == 0.0) {
    k.stopped = 1;
    k.stop_at = j;
    k.reason = 2;
  } else if (j >= k.maxiter) {
    k.stopped = 1;
    k.stop_at = j;
    k.reason = 4;
  }
}

// p = r + beta (p - omega v); a column that stopped at this j keeps its p
template <typename S, int KC>
__global__ void __launch_bounds__(kBlock)
    k_bstab_p(S *__restrict__ p, const S *__restrict__ r, const S *__restrict__ v, size_t n, int j,
              const KrylovState *K, KrylovHistory h) {
  using R = typename Store<S>::R;
  const int col = threadIdx.x % KC;
  if (K[col].stopped && j >= K[col].stop_at) return;
  const cx<double> be = c2(h.beta[j * KC + col]), om = c2(h.omega[j * KC + col]);
  const cx<R> b{R(be.x), R(be.y)}, w{R(om.x), R(om.y)};
  for (size_t u = size_t(blockIdx.x) * kBlock + threadIdx.x; u < n; u += size_t(gridDim.x) * kBlock)
    Store<S>::st(p, u, Store<S>::ld(r, u) + b * (Store<S>::ld(p, u) - w * Store<S>::ld(v, u)));
}

// ---- consumer-side scalars for small grids ------------------------------------
// When the producer's records are few (nblk NV KC doubles), every block of the
// consuming pass sums them itself, in the same fixed order as the one-block
// finish kernels, and block 0 stores the scalar and any stop in the history
// and state; the separate finish launch between the passes goes away.  Other
// blocks decide from their own (identical) totals, never from state that
// block 0 may be writing during the launch.
constexpr int kFuseMaxDoubles = 4096;
inline bool fuse_finish(int nblk, int nv, int kc) { return size_t(nblk) * nv * kc <= size_t(kFuseMaxDoubles); }

// alpha_j = rho_{j-1} / (rhat, v); s = r - alpha v
template <typename S, int KC>
__global__ void __launch_bounds__(kBlock)
    k_bstab_s_f(S *__restrict__ sv, const S *__restrict__ r, const S *__restrict__ v, size_t n, int j,
                KrylovState *K, KrylovHistory h, const double *__restrict__ part, int nblk) {
  using R = typename Store<S>::R;
  double d[2 * KC];
  sum_partials<2 * KC, kBlock>(part, nblk, d);
  const int col = threadIdx.x % KC;
  if (!col_active(K, col, j)) return;
  const cx<double> den{pick(d, 2 * col), pick(d, 2 * col + 1)};
  const double dd = den.x * den.x + den.y * den.y;
  const bool lead = blockIdx.x == 0 && threadIdx.x < KC;
  if (!(dd > 0.0) || !isfinite(dd)) {  // breakdown
    if (lead) {
      K[col].stopped = 1;
      K[col].stop_at = j - 1;
      K[col].reason = 2;
    }
    return;
  }
  const cx<double> al = cdiv(c2(h.rho[(j - 1) * KC + col]), den);
  if (lead) h.alpha[j * KC + col] = d2(al);
  const cx<R> a{R(al.x), R(al.y)};
  for (size_t u = size_t(blockIdx.x) * kBlock + threadIdx.x; u < n; u += size_t(gridDim.x) * kBlock)
    Store<S>::st(sv, u, Store<S>::ld(r, u) - a * Store<S>::ld(v, u));
}
// omega_j = (t, s) / (t, t); x += alpha p + omega s; r = s - omega t; records of (rhat, r), ||r||^2
template <typename S, int KC>
__global__ void __launch_bounds__(kBlock)
    k_bstab_xr_f(S *__restrict__ x, S *__restrict__ r, const S *__restrict__ p, const S *__restrict__ sv,
                 const S *__restrict__ t, const S *__restrict__ rhat, size_t n, int j, KrylovState *K,
                 KrylovHistory h, const double *__restrict__ part_t, int nblk, double *__restrict__ part) {
  using R = typename Store<S>::R;
  double d[3 * KC];
  sum_partials<3 * KC, kBlock>(part_t, nblk, d);
  const int col = threadIdx.x % KC;
  double e[3] = {0.0, 0.0, 0.0};
  if (col_active(K, col, j)) {
    const double tt = pick(d, 3 * col + 2);
    const bool lead = blockIdx.x == 0 && threadIdx.x < KC;
    if (!(tt > 0.0)) {  // breakdown
      if (lead) {
        K[col].stopped = 1;
        K[col].stop_at = j - 1;
        K[col].reason = 2;
      }
    } else {
      const cx<double> om{pick(d, 3 * col) / tt, pick(d, 3 * col + 1) / tt};
      if (lead) h.omega[j * KC + col] = d2(om);
      const cx<double> al = c2(h.alpha[j * KC + col]);
      const cx<R> a{R(al.x), R(al.y)}, w{R(om.x), R(om.y)};
      for (size_t u = size_t(blockIdx.x) * kBlock + threadIdx.x; u < n; u += size_t(gridDim.x) * kBlock) {
        const cx<R> si = Store<S>::ld(sv, u);
        Store<S>::st(x, u, Store<S>::ld(x, u) + a * Store<S>::ld(p, u) + w * si);
        const cx<R> ri = si - w * Store<S>::ld(t, u);
        Store<S>::st(r, u, ri);
        const cx<R> hh = Store<S>::ld(rhat, u);
        e[0] += double(hh.x) * ri.x + double(hh.y) * ri.y;
        e[1] += double(hh.x) * ri.y - double(hh.y) * ri.x;
        e[2] += double(ri.x) * ri.x + double(ri.y) * ri.y;
      }
    }
  }
  block_partial_cols<3, KC, kBlock>(e, part, blockIdx.x);
}
// rho_j, ||r_j||, beta_j and the stop tests; p = r + beta (p - omega v) for the
// columns that go on
template <typename S, int KC>
__global__ void __launch_bounds__(kBlock)
    k_bstab_p_f(S *__restrict__ p, const S *__restrict__ r, const S *__restrict__ v, size_t n, int j,
                KrylovState *K, KrylovHistory h, const double *__restrict__ part, int nblk) {
  using R = typename Store<S>::R;
  double d[3 * KC];
  sum_partials<3 * KC, kBlock>(part, nblk, d);
  const int col = threadIdx.x % KC;
  if (!col_active(K, col, j)) return;
  const cx<double> rho{pick(d, 3 * col), pick(d, 3 * col + 1)};
  const cx<double> be =
      cdiv(rho, c2(h.rho[(j - 1) * KC + col])) * cdiv(c2(h.alpha[j * KC + col]), c2(h.omega[j * KC + col]));
  const double rnorm = sqrt(pick(d, 3 * col + 2));
  int reason = 0;
  if (rnorm <= K[col].tol_abs)
    reason = 1;
  else if (rho.x == 0.0 && rho.y == 0.0)
    reason = 2;
  else if (j >= K[col].maxiter)
    reason = 4;
  if (blockIdx.x == 0 && threadIdx.x < KC) {
    h.rho[j * KC + col] = d2(rho);
    h.beta[j * KC + col] = d2(be);
    h.rn[j * KC + col] = rnorm;
    K[col].rnorm = rnorm;
    if (reason) {
      K[col].stopped = 1;
      K[col].stop_at = j;
      K[col].reason = reason;
    }
  }
  if (reason) return;  // the column stopped at this j: p keeps its value
  const cx<double> om = c2(h.omega[j * KC + col]);
  const cx<R> b{R(be.x), R(be.y)}, w{R(om.x), R(om.y)};
  for (size_t u = size_t(blockIdx.x) * kBlock + threadIdx.x; u < n; u += size_t(gridDim.x) * kBlock)
    Store<S>::st(p, u, Store<S>::ld(r, u) + b * (Store<S>::ld(p, u) - w * Store<S>::ld(v, u)));
}
// FP64 columns (column col at src + col N) <-> a batch in storage S
template <typename S, int KC>
__global__ void __launch_bounds__(kBlock)
    k_pack_batch(S *__restrict__ dst, const double2 *__restrict__ src, size_t N) {
  for (size_t u = size_t(blockIdx.x) * kBlock + threadIdx.x; u < N * KC; u += size_t(gridDim.x) * kBlock) {
    const double2 v = src[(u % KC) * N + u / KC];
    Store<S>::st(dst, u, cx<typename Store<S>::R>{typename Store<S>::R(v.x), typename Store<S>::R(v.y)});
  }
}
template <typename S, int KC>
__global__ void __launch_bounds__(kBlock)
    k_unpack_add_batch(double2 *__restrict__ x, const S *__restrict__ e, size_t N) {
  for (size_t u = size_t(blockIdx.x) * kBlock + threadIdx.x; u < N * KC; u += size_t(gridDim.x) * kBlock) {
    const auto v = Store<S>::ld(e, u);
    double2 &o = x[(u % KC) * N + u / KC];
    o = make_double2(o.x + double(v.x), o.y + double(v.y));
  }
}
// canonical spinors [KC][V][12] <-> batch
template <typename S, int KC>
__global__ void __launch_bounds__(kBlock) k_to_batch(S *__restrict__ dst, const S *__restrict__ src, int V) {
  const size_t n = size_t(V) * 12 * KC;
  for (size_t u = size_t(blockIdx.x) * kBlock + threadIdx.x; u < n; u += size_t(gridDim.x) * kBlock) {
    const int col = int(u % KC);
    const size_t cs = u / KC;  // c V + s
    const int c = int(cs / V), s = int(cs % V);
    dst[u] = src[(size_t(col) * V + s) * 12 + c];
  }
}
template <typename S, int KC>
__global__ void __launch_bounds__(kBlock) k_from_batch(S *__restrict__ dst, const S *__restrict__ src, int V) {
  const size_t n = size_t(V) * 12 * KC;
  for (size_t u = size_t(blockIdx.x) * kBlock + threadIdx.x; u < n; u += size_t(gridDim.x) * kBlock) {
    const int col = int(u % KC);
    const size_t cs = u / KC;
    const int c = int(cs / V), s = int(cs % V);
    dst[(size_t(col) * V + s) * 12 + c] = src[u];
  }
}

// ---- one column of a batch (serving sessions) ------------------------------
// A serving session keeps KC slots in one batch; a slot is (re)started or
// harvested while the other columns keep iterating, so these kernels touch
// column col only.
// r[:, col] = src (FP64 SoA column, N entries); e[:, col] = 0
template <typename S, int KC>
__global__ void __launch_bounds__(kBlock)
    k_slot_load(S *__restrict__ r, S *__restrict__ e, const double2 *__restrict__ src, size_t N, int col) {
  using R = typename Store<S>::R;
  for (size_t u = size_t(blockIdx.x) * kBlock + threadIdx.x; u < N; u += size_t(gridDim.x) * kBlock) {
    const double2 v = src[u];
    Store<S>::st(r, u * KC + col, cx<R>{R(v.x), R(v.y)});
    Store<S>::st(e, u * KC + col, cx<R>{R(0), R(0)});
  }
}
// rhat[:, col] = p[:, col] = r[:, col]; partials of ||r_col||^2
template <typename S, int KC>
__global__ void __launch_bounds__(kBlock)
    k_slot_init(S *__restrict__ rhat, S *__restrict__ p, const S *__restrict__ r, size_t N, int col,
                double *__restrict__ part) {
  double v[1] = {0.0};
  for (size_t u = size_t(blockIdx.x) * kBlock + threadIdx.x; u < N; u += size_t(gridDim.x) * kBlock) {
    const size_t i = u * KC + col;
    const auto rv = Store<S>::ld(r, i);
    Store<S>::st(rhat, i, rv);
    Store<S>::st(p, i, rv);
    v[0] += double(rv.x) * rv.x + double(rv.y) * rv.y;
  }
  block_partial_cols<1, 1, kBlock>(v, part, blockIdx.x);
}
// the column's state and rho_0 at history index col (iteration 0 of the
// session's next chunk); a column already at its target stops at once
template <int KC>
__global__ void __launch_bounds__(kBlock)
    k_slot_init_finish(const double *__restrict__ part, int nblk, int col, double tol_abs, int maxiter,
                       KrylovState *K, KrylovHistory h) {
  double v[1];
  sum_partials<1, kBlock>(part, nblk, v);
  if (threadIdx.x != 0) return;
  const double rn = sqrt(v[0]);
  h.rho[col] = make_double2(v[0], 0.0);
  h.rn[col] = rn;
  KrylovState &k = K[col];
  k.bnorm = 0.0;
  k.tol_abs = tol_abs;
  k.def_thr = 0.0;
  k.rnorm = rn;
  k.maxiter = maxiter;
  k.stopped = 0;
  k.stop_at = 0;
  k.reason = 0;
  if (rn <= tol_abs) {
    k.stopped = 1;
    k.reason = 1;
  }
}
// x (FP64 SoA column) += e[:, col]
template <typename S, int KC>
__global__ void __launch_bounds__(kBlock)
    k_slot_add(double2 *__restrict__ x, const S *__restrict__ e, size_t N, int col) {
  for (size_t u = size_t(blockIdx.x) * kBlock + threadIdx.x; u < N; u += size_t(gridDim.x) * kBlock) {
    const auto v = Store<S>::ld(e, u * KC + col);
    x[u] = make_double2(x[u].x + double(v.x), x[u].y + double(v.y));
  }
}
// End of a chunk of jl iterations: the next chunk counts from j = 1 again.  A
// running column carries rho_jl to index 0 and jl fewer iterations of budget;
// a stopped column stays inactive for every j >= 0.
template <int KC>
__global__ void k_batch_rebase(KrylovState *K, KrylovHistory h, int jl) {
  const int col = threadIdx.x;
  if (col >= KC) return;
  KrylovState &k = K[col];
  if (k.stopped) {
    k.stop_at = -1;
    return;
  }
  h.rho[col] = h.rho[size_t(jl) * KC + col];
  h.rn[col] = h.rn[size_t(jl) * KC + col];
  k.maxiter -= jl;
}

}  // namespace

bool batch_size_ok(int kc) { return kc == 1 || kc == 2 || kc == 4 || kc == 8 || kc == 16; }
int march_records(const Geom &g, int kc) { return march_blocks(g, kc, march_shape(g, kc)); }
int bicg_matvec_march_records(const Geom &g, bool g5) { return march_records(g, 1) * (g5 ? 1 : 2); }
void launch_bicg_matvec_march(double2 *Ap, double2 *Adp, const double2 *p, const double2 *ph, const double2 *U,
                              const Geom &g, double kappa, int j, KrylovState *S, const RedScratch &rs, bool g5,
                              hipStream_t st) {
  const March m = march_shape(g, 1);
  const dim3 grid(bicg_matvec_march_records(g, g5));
  if (g5)
    EB_LAUNCH(k_bicg_matvec_march<true>, grid, dim3(kBlock), 0, st, Ap, Adp, p, ph, U, g, kappa, m, j, S,
              region(rs, RG_SIGMA));
  else
    EB_LAUNCH(k_bicg_matvec_march<false>, grid, dim3(kBlock), 0, st, Ap, Adp, p, ph, U, g, kappa, m, j, S,
              region(rs, RG_SIGMA));
}
bool batch_tile_ok(const Geom &g, bool eo, int stage, int kc) {
  if (stage < -1 || stage >= kTileForms) return false;
  if (stage < 2) return true;
  if (stage == 5) return !eo;
  if (stage == kMarchForm) return !eo && march_shape(g, kc).rx > 0;
  const Brick b = brick_of(stage);  // bricked forms: full-lattice stencil, extents divisible by the brick
  return !eo && g.lx % b.bx == 0 && g.ly % b.by == 0 && g.lz % b.bz == 0 && g.lt % b.bt == 0;
}

template <typename S>
void launch_bdslash(S *out, const S *in, const S *U, const Geom &g, double kappa, bool dagger, int kc, hipStream_t st,
                    int stage) {
  dispatch_kc(kc, [&](auto kt) {
    constexpr int KC = decltype(kt)::value;
    if (stage == kMarchForm) {
      const March m = march_shape(g, KC);
      const dim3 grid(march_blocks(g, KC, m));
      if (dagger)
        EB_LAUNCH((k_bmarch<S, KC, +1, 0>), grid, dim3(kBlock), 0, st, out, in, U, g, kappa, m, nullptr, 0, nullptr,
                  nullptr);
      else
        EB_LAUNCH((k_bmarch<S, KC, -1, 0>), grid, dim3(kBlock), 0, st, out, in, U, g, kappa, m, nullptr, 0, nullptr,
                  nullptr);
      return;
    }
    dispatch_stage<S, KC>(stage, [&](auto sg, auto fg) {
      constexpr bool STG = decltype(sg)::value, FENCE = decltype(fg)::value;
      const dim3 grid(nblocks_for(size_t(g.V) * KC));
      if (dagger)
        EB_LAUNCH((k_bdslash<S, KC, +1, STG, FENCE>), grid, dim3(kBlock), 0, st, out, in, U, g, kappa,
                  brick_of(stage));
      else
        EB_LAUNCH((k_bdslash<S, KC, -1, STG, FENCE>), grid, dim3(kBlock), 0, st, out, in, U, g, kappa,
                  brick_of(stage));
    });
  });
}

template <typename S>
void launch_bstab_init(S *rhat, S *p, const S *r, size_t N, int kc, const double *tol_abs, int maxiter,
                       KrylovState *K, KrylovHistory h, const RedScratch &rs, hipStream_t st) {
  dispatch_kc(kc, [&](auto kt) {
    constexpr int KC = decltype(kt)::value;
    const int nb = batch_red_grid(N * KC, KC, 1);
    EB_LAUNCH((k_bstab_init<S, KC>), dim3(nb), dim3(kBlock), 0, st, rhat, p, r, N * KC, region(rs, RG_INIT));
    EB_LAUNCH(k_bstab_init_finish<KC>, dim3(1), dim3(kBlock), 0, st, region(rs, RG_INIT), nb, tol_abs, maxiter, K, h);
  });
}

template <typename S>
void launch_bstab_v(S *v, const S *p, const S *rhat, const S *U, const Geom &g, double kappa, int j, int kc,
                    KrylovState *K, const RedScratch &rs, hipStream_t st, int stage) {
  dispatch_kc(kc, [&](auto kt) {
    constexpr int KC = decltype(kt)::value;
    if (stage == kMarchForm) {
      const March m = march_shape(g, KC);
      EB_LAUNCH((k_bmarch<S, KC, -1, 1>), dim3(march_blocks(g, KC, m)), dim3(kBlock), 0, st, v, p, U, g, kappa, m,
                rhat, j, K, region(rs, RG_V));
      return;
    }
    dispatch_stage<S, KC>(stage, [&](auto sg, auto fg) {
      EB_LAUNCH((k_bstab_v<S, KC, decltype(sg)::value, decltype(fg)::value>), dim3(batch_stencil_grid(g.V, KC, 2)), dim3(kBlock), 0, st,
                v, p, rhat, U, g, kappa, j, K, region(rs, RG_V), brick_of(stage));
    });
  });
}

template <typename S>
void launch_bstab_s(S *sv, const S *r, const S *v, const Geom &g, int j, int kc, KrylovState *K, KrylovHistory h,
                    const RedScratch &rs, hipStream_t st, int stage) {
  dispatch_kc(kc, [&](auto kt) {
    constexpr int KC = decltype(kt)::value;
    const size_t n = size_t(12) * g.V * KC;
    const int nblk = stencil_records(g, KC, 2, stage);
    if (fuse_finish(nblk, 2, KC)) {
      EB_LAUNCH((k_bstab_s_f<S, KC>), dim3(stream_grid(n)), dim3(kBlock), 0, st, sv, r, v, n, j, K, h,
                region(rs, RG_V), nblk);
      return;
    }
    EB_LAUNCH(k_bfin_alpha<KC>, dim3(1), dim3(kBlock), 0, st, region(rs, RG_V), nblk, j, K, h);
    EB_LAUNCH((k_bstab_s<S, KC>), dim3(stream_grid(n)), dim3(kBlock), 0, st, sv, r, v, n, j, K, h);
  });
}

template <typename S>
void launch_bstab_t(S *t, const S *sv, const S *U, const Geom &g, double kappa, int j, int kc, KrylovState *K,
                    const RedScratch &rs, hipStream_t st, int stage) {
  dispatch_kc(kc, [&](auto kt) {
    constexpr int KC = decltype(kt)::value;
    if (stage == kMarchForm) {
      const March m = march_shape(g, KC);
      EB_LAUNCH((k_bmarch<S, KC, -1, 2>), dim3(march_blocks(g, KC, m)), dim3(kBlock), 0, st, t, sv, U, g, kappa, m,
                nullptr, j, K, region(rs, RG_T));
      return;
    }
    dispatch_stage<S, KC>(stage, [&](auto sg, auto fg) {
      EB_LAUNCH((k_bstab_t<S, KC, decltype(sg)::value, decltype(fg)::value>), dim3(batch_stencil_grid(g.V, KC, 3)), dim3(kBlock), 0, st,
                t, sv, U, g, kappa, j, K, region(rs, RG_T), brick_of(stage));
    });
  });
}

template <typename S>
void launch_bstab_xr(S *x, S *r, const S *p, const S *sv, const S *t, const S *rhat, const Geom &g, int j, int kc,
                     KrylovState *K, KrylovHistory h, const RedScratch &rs, hipStream_t st, int stage) {
  dispatch_kc(kc, [&](auto kt) {
    constexpr int KC = decltype(kt)::value;
    const size_t n = size_t(12) * g.V * KC;
    const int nblk = stencil_records(g, KC, 3, stage);
    if (fuse_finish(nblk, 3, KC)) {
      EB_LAUNCH((k_bstab_xr_f<S, KC>), dim3(batch_red_grid(n, KC, 3)), dim3(kBlock), 0, st, x, r, p, sv, t, rhat, n,
                j, K, h, region(rs, RG_T), nblk, region(rs, RG_XR));
      return;
    }
    EB_LAUNCH(k_bfin_omega<KC>, dim3(1), dim3(kBlock), 0, st, region(rs, RG_T), nblk, j, K, h);
    EB_LAUNCH((k_bstab_xr<S, KC>), dim3(batch_red_grid(n, KC, 3)), dim3(kBlock), 0, st, x, r, p, sv, t, rhat, n, j, K,
              h, region(rs, RG_XR));
  });
}

template <typename S>
void launch_bstab_p(S *p, const S *r, const S *v, const Geom &g, int j, int kc, KrylovState *K, KrylovHistory h,
                    const RedScratch &rs, hipStream_t st) {
  dispatch_kc(kc, [&](auto kt) {
    constexpr int KC = decltype(kt)::value;
    const size_t n = size_t(12) * g.V * KC;
    const int nblk = batch_red_grid(n, KC, 3);
    if (fuse_finish(nblk, 3, KC)) {
      EB_LAUNCH((k_bstab_p_f<S, KC>), dim3(stream_grid(n)), dim3(kBlock), 0, st, p, r, v, n, j, K, h,
                region(rs, RG_XR), nblk);
      return;
    }
    EB_LAUNCH(k_bfin_beta<KC>, dim3(1), dim3(kBlock), 0, st, region(rs, RG_XR), nblk, j, K, h);
    EB_LAUNCH((k_bstab_p<S, KC>), dim3(stream_grid(n)), dim3(kBlock), 0, st, p, r, v, n, j, K, h);
  });
}

template <typename S>
void launch_pack_batch(S *dst, const double2 *src, size_t N, int kc, hipStream_t st) {
  dispatch_kc(kc, [&](auto kt) {
    constexpr int KC = decltype(kt)::value;
    EB_LAUNCH((k_pack_batch<S, KC>), dim3(stream_grid(N * KC)), dim3(kBlock), 0, st, dst, src, N);
  });
}
template <typename S>
void launch_unpack_add_batch(double2 *x, const S *e, size_t N, int kc, hipStream_t st) {
  dispatch_kc(kc, [&](auto kt) {
    constexpr int KC = decltype(kt)::value;
    EB_LAUNCH((k_unpack_add_batch<S, KC>), dim3(stream_grid(N * KC)), dim3(kBlock), 0, st, x, e, N);
  });
}
template <typename S>
void launch_to_batch(S *dst, const S *src, const Geom &g, int kc, hipStream_t st) {
  dispatch_kc(kc, [&](auto kt) {
    constexpr int KC = decltype(kt)::value;
    EB_LAUNCH((k_to_batch<S, KC>), dim3(stream_grid(size_t(12) * g.V * KC)), dim3(kBlock), 0, st, dst, src, g.V);
  });
}
template <typename S>
void launch_from_batch(S *dst, const S *src, const Geom &g, int kc, hipStream_t st) {
  dispatch_kc(kc, [&](auto kt) {
    constexpr int KC = decltype(kt)::value;
    EB_LAUNCH((k_from_batch<S, KC>), dim3(stream_grid(size_t(12) * g.V * KC)), dim3(kBlock), 0, st, dst, src, g.V);
  });
}

template <typename S>
void launch_slot_load(S *r, S *e, const double2 *src, size_t N, int kc, int col, hipStream_t st) {
  dispatch_kc(kc, [&](auto kt) {
    constexpr int KC = decltype(kt)::value;
    EB_LAUNCH((k_slot_load<S, KC>), dim3(stream_grid(N)), dim3(kBlock), 0, st, r, e, src, N, col);
  });
}
template <typename S>
void launch_slot_init(S *rhat, S *p, const S *r, size_t N, int kc, int col, double tol_abs, int maxiter,
                      KrylovState *K, KrylovHistory h, const RedScratch &rs, hipStream_t st) {
  dispatch_kc(kc, [&](auto kt) {
    constexpr int KC = decltype(kt)::value;
    const int nb = batch_red_grid(N, 1, 1);
    EB_LAUNCH((k_slot_init<S, KC>), dim3(nb), dim3(kBlock), 0, st, rhat, p, r, N, col, region(rs, RG_INIT));
    EB_LAUNCH(k_slot_init_finish<KC>, dim3(1), dim3(kBlock), 0, st, region(rs, RG_INIT), nb, col, tol_abs, maxiter, K,
              h);
  });
}
template <typename S>
void launch_slot_add(double2 *x, const S *e, size_t N, int kc, int col, hipStream_t st) {
  dispatch_kc(kc, [&](auto kt) {
    constexpr int KC = decltype(kt)::value;
    EB_LAUNCH((k_slot_add<S, KC>), dim3(stream_grid(N)), dim3(kBlock), 0, st, x, e, N, col);
  });
}
void launch_batch_rebase(KrylovState *K, KrylovHistory h, int kc, int jl, hipStream_t st) {
  dispatch_kc(kc, [&](auto kt) {
    constexpr int KC = decltype(kt)::value;
    EB_LAUNCH(k_batch_rebase<KC>, dim3(1), dim3(64), 0, st, K, h, jl);
  });
}

#define EB_BATCH_INST(S)                                                                                           \
  template void launch_bdslash<S>(S *, const S *, const S *, const Geom &, double, bool, int, hipStream_t, int);   \
  template void launch_bstab_init<S>(S *, S *, const S *, size_t, int, const double *, int, KrylovState *,         \
                                     KrylovHistory, const RedScratch &, hipStream_t);                              \
  template void launch_bstab_v<S>(S *, const S *, const S *, const S *, const Geom &, double, int, int,            \
                                  KrylovState *, const RedScratch &, hipStream_t, int);                            \
  template void launch_bstab_s<S>(S *, const S *, const S *, const Geom &, int, int, KrylovState *, KrylovHistory, \
                                  const RedScratch &, hipStream_t, int);                                           \
  template void launch_bstab_t<S>(S *, const S *, const S *, const Geom &, double, int, int, KrylovState *,        \
                                  const RedScratch &, hipStream_t, int);                                           \
  template void launch_bstab_xr<S>(S *, S *, const S *, const S *, const S *, const S *, const Geom &, int, int,   \
                                   KrylovState *, KrylovHistory, const RedScratch &, hipStream_t, int);            \
  template void launch_bstab_p<S>(S *, const S *, const S *, const Geom &, int, int, KrylovState *, KrylovHistory, \
                                  const RedScratch &, hipStream_t);                                                \
  template void launch_pack_batch<S>(S *, const double2 *, size_t, int, hipStream_t);                              \
  template void launch_unpack_add_batch<S>(double2 *, const S *, size_t, int, hipStream_t);                        \
  template void launch_to_batch<S>(S *, const S *, const Geom &, int, hipStream_t);                                \
  template void launch_from_batch<S>(S *, const S *, const Geom &, int, hipStream_t);                                \
  template void launch_slot_load<S>(S *, S *, const double2 *, size_t, int, int, hipStream_t);                     \
  template void launch_slot_init<S>(S *, S *, const S *, size_t, int, int, double, int, KrylovState *,            \
                                    KrylovHistory, const RedScratch &, hipStream_t);                              \
  template void launch_slot_add<S>(double2 *, const S *, size_t, int, int, hipStream_t);
EB_BATCH_INST(double2)
EB_BATCH_INST(float2)
EB_BATCH_INST(bf16c)

}  // namespace ebicg
