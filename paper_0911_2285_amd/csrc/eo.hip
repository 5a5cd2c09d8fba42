// Even-odd (Schur) form of the Wilson operator, FP64.
//
// The paper's test matrices are even-odd preconditioned Wilson operators
// (Sec. 3, "Results").  With the sites split by parity (x+y+z+t even or odd),
// D = 1 - kappa H has the block form [[1, -kappa H_eo], [-kappa H_oe, 1]] and
// the Krylov solvers run on the Schur complement of the even sites,
//     Dhat = 1 - kappa^2 H_eo H_oe,   Dhat^+ = 1 - kappa^2 H^+_eo H^+_oe,
// with b_hat = b_e + kappa H_eo b_o and x_o = b_o + kappa H_oe x_e.
//
// Half-lattice layout: the sites of one parity in increasing site order;
// with every extent even, site s of parity P has index h = s / 2.  Spinors
// are SoA [12][V/2]; links [parity][4 mu][9][V/2] with the antiperiodic sign
// folded into U_t at t = Lt - 1, so a hop from parity P reads its forward link
// at its own index h and its backward link at the neighbour's index.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_common.h"
#include "kernel_util.h"
#include "kernels.h"
#include "stencil.h"

namespace ebicg {
namespace {

// canonical [V][4][3] <-> SoA [12][V/2] per parity (odd part zero if o is null)
__global__ void __launch_bounds__(kBlock)
    k_to_eo(double2 *__restrict__ e, double2 *__restrict__ o, const double2 *__restrict__ src, Geom g) {
  const size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x;  // canonical s * 12 + c
  if (i >= size_t(g.V) * 12) return;
  const int s = int(i / 12), c = int(i % 12);
  const int x = s % g.lx, y = (s / g.lx) % g.ly, z = (s / (g.lx * g.ly)) % g.lz, t = s / (g.lx * g.ly * g.lz);
  double2 *dst = ((x + y + z + t) & 1) ? o : e;
  dst[size_t(c) * (g.V / 2) + (s >> 1)] = src[i];
}

__global__ void __launch_bounds__(kBlock)
    k_from_eo(double2 *__restrict__ dst, const double2 *__restrict__ e, const double2 *__restrict__ o, Geom g) {
  const size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= size_t(g.V) * 12) return;
  const int s = int(i / 12), c = int(i % 12);
  const int x = s % g.lx, y = (s / g.lx) % g.ly, z = (s / (g.lx * g.ly)) % g.lz, t = s / (g.lx * g.ly * g.lz);
  const double2 *srcp = ((x + y + z + t) & 1) ? o : e;
  dst[i] = srcp ? srcp[size_t(c) * (g.V / 2) + (s >> 1)] : make_double2(0.0, 0.0);
}

// canonical gauge [4][V][3][3] -> [parity][mu][9][V/2], boundary sign folded
__global__ void __launch_bounds__(kBlock)
    k_pack_gauge_eo(double2 *__restrict__ dst, const double2 *__restrict__ src, Geom g, int bc_t) {
  const size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x;  // (mu V + s) 9 + e
  if (i >= size_t(g.V) * 36) return;
  const int e = int(i % 9);
  const size_t ms = i / 9;
  const int mu = int(ms / g.V), s = int(ms % g.V);
  const int x = s % g.lx, y = (s / g.lx) % g.ly, z = (s / (g.lx * g.ly)) % g.lz, t = s / (g.lx * g.ly * g.lz);
  double2 u = src[i];
  if (mu == 3 && bc_t != 1 && t == g.lt - 1) {
    u.x *= double(bc_t);
    u.y *= double(bc_t);
  }
  const int par = (x + y + z + t) & 1;
  const size_t Vh = size_t(g.V / 2);
  dst[(size_t(par) * 36 + mu * 9 + e) * Vh + (s >> 1)] = u;
}

// One direction of the hop onto a parity-P site (half index h): the forward
// neighbour's half spinor with U_mu(x) (own parity, index h), the backward
// neighbour's with U_mu(x - mu)^+ (other parity, index hb).  The input comes
// through an LDS tile of the same index range as the block's outputs: x and
// most y neighbours fall inside it.
template <int MU, int SF, typename S, typename Src>
__device__ __forceinline__ void hop_dir_eo(cx<typename Store<S>::R> (&acc)[12], const Src &src,
                                           const S *__restrict__ Uf, const S *__restrict__ Ub, int Vh, int h, int hf,
                                           int hb) {
  cx<typename Store<S>::R> hh[6];
  load_project_t<MU, SF, S>(hh, src, hf);
  mult_accum<MU, SF, false, S>(acc, hh, Uf, Vh, h);
  if constexpr (Src::kFence) hop_fence();
  load_project_t<MU, -SF, S>(hh, src, hb);
  mult_accum<MU, -SF, true, S>(acc, hh, Ub, Vh, hb);
  if constexpr (Src::kFence) hop_fence();
}

// The hop sum onto the parity-P site of half index h (all four directions).
template <int SF, typename S, typename Src>
__device__ __forceinline__ void eo_hops(cx<typename Store<S>::R> (&acc)[12], const Src &src,
                                        const S *__restrict__ Uf, const S *__restrict__ Ub, const Geom &g, int P,
                                        int h) {
  const int Vh = g.V / 2, lxh = g.lx / 2;
  const int sy = g.lx, sz = g.lx * g.ly, stt = sz * g.lz;
  const int xh = h % lxh, r1 = h / lxh;
  const int y = r1 % g.ly, r2 = r1 / g.ly;
  const int z = r2 % g.lz, t = r2 / g.lz;
  const int x = 2 * xh + ((P + y + z + t) & 1);
  const int s = x + g.lx * r1;
#pragma unroll
  for (int c = 0; c < 12; ++c) acc[c] = {0, 0};
  // z and t first, as in the full-lattice stencil
  hop_dir_eo<2, SF, S>(acc, src, Uf, Ub, Vh, h, (z == g.lz - 1 ? s - (g.lz - 1) * sz : s + sz) >> 1,
                           (z == 0 ? s + (g.lz - 1) * sz : s - sz) >> 1);
  hop_dir_eo<3, SF, S>(acc, src, Uf, Ub, Vh, h, (t == g.lt - 1 ? s - (g.lt - 1) * stt : s + stt) >> 1,
                           (t == 0 ? s + (g.lt - 1) * stt : s - stt) >> 1);
  hop_dir_eo<0, SF, S>(acc, src, Uf, Ub, Vh, h, (x == g.lx - 1 ? s - (g.lx - 1) : s + 1) >> 1,
                           (x == 0 ? s + (g.lx - 1) : s - 1) >> 1);
  hop_dir_eo<1, SF, S>(acc, src, Uf, Ub, Vh, h, (y == g.ly - 1 ? s - (g.ly - 1) * sy : s + sy) >> 1,
                           (y == 0 ? s + (g.ly - 1) * sy : s - sy) >> 1);
}

enum EoEpi : int {
  EO_TMP = 0,  // out = H in
  EO_SCHUR,    // out = id - a H in
  EO_SIGMA,    // EO_SCHUR, partials of (dv, out)
  EO_SIGMA5,   // EO_SCHUR, partials of (gamma5 id, out)
  EO_STABT,    // EO_SCHUR, partials of (out, id) and ||out||^2
  EO_RESID,    // out = dv - (id - a H in), partials of ||out||^2 and ||dv||^2
  EO_PREP,     // out = id + a H in
};
template <int E>
struct EoNV {
  static constexpr int v = (E == EO_SIGMA || E == EO_SIGMA5 || E == EO_RESID) ? 2 : (E == EO_STABT ? 3 : 0);
};

// out (parity P, half index) from in (parity 1 - P); SF = -1: H, +1: H^+.
// Storage S (FP64, FP32 or BF16 with FP32 arithmetic); the partial sums are
// FP64.  Blocks loop over tiles of kBlock sites; producers of partial sums
// write one record per block of the launch (blocks beyond the tiles write
// zeros).
template <typename S, int SF, int E>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1, 2)))
    k_hop_eo(S *__restrict__ out, const S *__restrict__ in, const S *__restrict__ Uf, const S *__restrict__ Ub,
             Geom g, int P, double a_, const S *__restrict__ id, const S *__restrict__ dv, int j,
             const KrylovState *K, double *__restrict__ part) {
  using R = typename Store<S>::R;
  if (K && skip_iter(K, j)) return;
  constexpr int NV = EoNV<E>::v;
  const R a = R(a_);
  __shared__ S tile[12 * kBlock];
  const int Vh = g.V / 2;
  double v[NV > 0 ? NV : 1];
#pragma unroll
  for (int k = 0; k < (NV > 0 ? NV : 1); ++k) v[k] = 0.0;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int ntiles = (Vh + kBlock - 1) / kBlock;
  for (int T = lb; T < ntiles; T += gridDim.x) {
    const int h0 = T * kBlock, h = h0 + int(threadIdx.x);
    __syncthreads();  // the previous tile's readers are done
    stage_tile(tile, in, h0, Vh);
    __syncthreads();
    if (h >= Vh) continue;
    cx<R> acc[12];
    eo_hops<SF, S>(acc, TileSrc<S>{in, tile, h0, Vh}, Uf, Ub, g, P, h);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const size_t i = size_t(c) * Vh + h;
      if constexpr (E == EO_TMP) {
        Store<S>::st(out, i, acc[c]);
      } else if constexpr (E == EO_PREP) {
        Store<S>::st(out, i, Store<S>::ld(id, i) + a * acc[c]);
      } else if constexpr (E == EO_RESID) {
        const cx<R> bv = Store<S>::ld(dv, i);
        const cx<R> rv = bv - (Store<S>::ld(id, i) - a * acc[c]);
        Store<S>::st(out, i, rv);
        v[0] += double(rv.x) * rv.x + double(rv.y) * rv.y;
        v[1] += double(bv.x) * bv.x + double(bv.y) * bv.y;
      } else {
        const cx<R> iv = Store<S>::ld(id, i);
        const cx<R> o = iv - a * acc[c];
        Store<S>::st(out, i, o);
        if constexpr (E == EO_SIGMA) {  // conj(dv) o
          const cx<R> hv = Store<S>::ld(dv, i);
          v[0] += double(hv.x) * o.x + double(hv.y) * o.y;
          v[1] += double(hv.x) * o.y - double(hv.y) * o.x;
        } else if constexpr (E == EO_SIGMA5) {  // conj(gamma5 id) o
          const double dr = double(iv.x) * o.x + double(iv.y) * o.y, di = double(iv.x) * o.y - double(iv.y) * o.x;
          v[0] += c < 6 ? dr : -dr;
          v[1] += c < 6 ? di : -di;
        } else if constexpr (E == EO_STABT) {  // conj(o) id, |o|^2
          v[0] += double(o.x) * iv.x + double(o.y) * iv.y;
          v[1] += double(o.x) * iv.y - double(o.y) * iv.x;
          v[2] += double(o.x) * o.x + double(o.y) * o.y;
        }
      }
    }
  }
  if constexpr (NV > 0) block_partial<NV, kBlock>(v, part, blockIdx.x);
}

template <int NV>
__global__ void __launch_bounds__(kBlock) k_eo_finish(const double *__restrict__ part, int nblk, double *out) {
  double v[NV];
  sum_partials<NV, kBlock>(part, nblk, v);
  if (threadIdx.x == 0)
    for (int i = 0; i < NV; ++i) out[i] = v[i];
}

// Multi-RHS: KC half-lattice spinors in the batch layout (element
// (c, h, col) at (c Vh + h) KC + col; the KC lanes of a site share its link
// loads), tiles of kBlock / KC sites.  Each column is its own BiCGStab
// recurrence: a column that has stopped (K non-null) skips the work and adds
// nothing to its partial sums, which are per column.  The input goes through
// LDS where the full-lattice batches found staging to pay (one column, or
// BF16 entries); FP64 / FP32 batches read their neighbours from global memory.
template <typename S, int KC>
constexpr bool kStageEo = KC == 1 || std::is_same<S, bf16c>::value;

template <typename S, int KC, int SF, int E, bool STG>
__global__ void __launch_bounds__(kBlock)
    k_bhop_eo(S *__restrict__ out, const S *__restrict__ in, const S *__restrict__ Uf, const S *__restrict__ Ub,
              Geom g, int P, double a_, const S *__restrict__ id, const S *__restrict__ dv, int j,
              const KrylovState *K, double *__restrict__ part) {
  using R = typename Store<S>::R;
  static_assert(E == EO_TMP || E == EO_SCHUR || E == EO_SIGMA || E == EO_STABT, "batched epilogues");
  constexpr int NV = EoNV<E>::v, spt = kBlock / KC;
  const int col = int(threadIdx.x) % KC;
  const bool act = !K || !skip_iter(K + col, j);
  const R a = R(a_);
  __shared__ S tile[12 * kBlock];
  const int Vh = g.V / 2;
  double v[NV > 0 ? NV : 1];
#pragma unroll
  for (int k = 0; k < (NV > 0 ? NV : 1); ++k) v[k] = 0.0;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int ntiles = (Vh + spt - 1) / spt;
  for (int T = lb; T < ntiles; T += gridDim.x) {
    const int h0 = T * spt, h = h0 + int(threadIdx.x) / KC;
    if constexpr (STG) {
      __syncthreads();  // the previous tile's readers are done
      stage_tile<S, KC>(tile, in, h0, Vh);
      __syncthreads();
    }
    if (!act || h >= Vh) continue;
    cx<R> acc[12];
    if constexpr (STG)
      eo_hops<SF, S>(acc, TileSrc<S, KC>{in + col, tile + col, h0, Vh}, Uf, Ub, g, P, h);
    else
      eo_hops<SF, S>(acc, GlobSrc<S, KC>{in + col, Vh}, Uf, Ub, g, P, h);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const size_t i = (size_t(c) * Vh + h) * KC + col;
      if constexpr (E == EO_TMP) {
        Store<S>::st(out, i, acc[c]);
      } else {
        const cx<R> iv = Store<S>::ld(id, i);
        const cx<R> o = iv - a * acc[c];
        Store<S>::st(out, i, o);
        if constexpr (E == EO_SIGMA) {  // conj(dv) o
          const cx<R> hv = Store<S>::ld(dv, i);
          v[0] += double(hv.x) * o.x + double(hv.y) * o.y;
          v[1] += double(hv.x) * o.y - double(hv.y) * o.x;
        } else if constexpr (E == EO_STABT) {  // conj(o) id, |o|^2
          v[0] += double(o.x) * iv.x + double(o.y) * iv.y;
          v[1] += double(o.x) * iv.y - double(o.y) * iv.x;
          v[2] += double(o.x) * o.x + double(o.y) * o.y;
        }
      }
    }
  }
  if constexpr (NV > 0) block_partial_cols<NV, KC, kBlock>(v, part, blockIdx.x);
}

inline int eo_grid(const Geom &g) { return stencil_grid(g.V / 2); }
template <typename S>
inline const S *links_of(const S *Ueo, const Geom &g, int par) {
  return Ueo + size_t(par) * 36 * size_t(g.V / 2);
}

// out (parity P) = epilogue(H_{P, 1-P} in) on `grid` blocks
template <int SF, int E, typename S>
void hop(S *out, const S *in, const S *Ueo, const Geom &g, int P, double a, const S *id, const S *dv, int j,
         const KrylovState *K, double *part, int grid, hipStream_t st) {
  EB_LAUNCH((k_hop_eo<S, SF, E>), dim3(grid), dim3(kBlock), 0, st, out, in, links_of(Ueo, g, P),
            links_of(Ueo, g, 1 - P), g, P, a, id, dv, j, K, part);
}

// batched: out (parity P) = epilogue(H_{P, 1-P} in) for kc columns; a
// producer of partial sums uses batch_stencil_grid(V/2, kc, NV) blocks, the
// count the batched BiCGStab's consumers read for spinors of V/2 sites
template <int SF, int E, typename S>
void bhop(S *out, const S *in, const S *Ueo, const Geom &g, int P, double a, const S *id, const S *dv, int j,
          const KrylovState *K, double *part, int kc, hipStream_t st, int stage) {
  dispatch_kc(kc, [&](auto kt) {
    constexpr int KC = decltype(kt)::value;
    constexpr int NV = EoNV<E>::v;
    const int grid = batch_stencil_grid(g.V / 2, KC, NV > 0 ? NV : 1);
    if (stage < 0 ? kStageEo<S, KC> : stage == 1)
      EB_LAUNCH((k_bhop_eo<S, KC, SF, E, true>), dim3(grid), dim3(kBlock), 0, st, out, in, links_of(Ueo, g, P),
                links_of(Ueo, g, 1 - P), g, P, a, id, dv, j, K, part);
    else
      EB_LAUNCH((k_bhop_eo<S, KC, SF, E, false>), dim3(grid), dim3(kBlock), 0, st, out, in, links_of(Ueo, g, P),
                links_of(Ueo, g, 1 - P), g, P, a, id, dv, j, K, part);
  });
}

}  // namespace

bool eo_geometry_ok(const Geom &g) {
  return g.lx % 2 == 0 && g.ly % 2 == 0 && g.lz % 2 == 0 && g.lt % 2 == 0 && g.lx >= 2;
}

void launch_to_eo(double2 *e, double2 *o, const double2 *canon, const Geom &g, hipStream_t st) {
  EB_LAUNCH(k_to_eo, dim3(nblocks_for(size_t(g.V) * 12)), dim3(kBlock), 0, st, e, o, canon, g);
}
void launch_from_eo(double2 *canon, const double2 *e, const double2 *o, const Geom &g, hipStream_t st) {
  EB_LAUNCH(k_from_eo, dim3(nblocks_for(size_t(g.V) * 12)), dim3(kBlock), 0, st, canon, e, o, g);
}
void launch_pack_gauge_eo(double2 *Ueo, const double2 *canon, const Geom &g, int bc_t, hipStream_t st) {
  EB_LAUNCH(k_pack_gauge_eo, dim3(nblocks_for(size_t(g.V) * 36)), dim3(kBlock), 0, st, Ueo, canon, g, bc_t);
}

void launch_schur_eo(double2 *out, const double2 *in, double2 *tmp, const double2 *Ueo, const Geom &g, double kappa,
                     bool dagger, hipStream_t st) {
  launch_schur_eo_s<double2>(out, in, tmp, Ueo, g, kappa, dagger, st);
}

void launch_prep_eo(double2 *out, const double2 *id, const double2 *in, const Geom &g, const double2 *Ueo,
                    double kappa, int out_parity, hipStream_t st) {
  hop<-1, EO_PREP, double2>(out, in, Ueo, g, out_parity, kappa, id, nullptr, 0, nullptr, nullptr, eo_grid(g), st);
}

void launch_residual_eo(double2 *r, const double2 *b, const double2 *x, double2 *tmp, const double2 *Ueo,
                        const Geom &g, double kappa, double *res, const RedScratch &rs, hipStream_t st) {
  const int G = eo_grid(g);
  hop<-1, EO_TMP, double2>(tmp, x, Ueo, g, 1, 0.0, nullptr, nullptr, 0, nullptr, nullptr, G, st);
  hop<-1, EO_RESID, double2>(r, tmp, Ueo, g, 0, kappa * kappa, x, b, 0, nullptr, region(rs, RG_RES), G, st);
  EB_LAUNCH(k_eo_finish<2>, dim3(1), dim3(kBlock), 0, st, region(rs, RG_RES), G, res);
}

void launch_bicg_matvec_eo(double2 *Ap, double2 *Adp, const double2 *p, const double2 *ph, double2 *tmp,
                           const double2 *Ueo, const Geom &g, double kappa, int j, KrylovState *S,
                           const RedScratch &rs, bool g5, hipStream_t st) {
  // the sigma records: as many as the update kernel of the form expects for
  // spinors of length 12 V/2 (one per block of its matvec grid)
  const int G = eo_grid(g), Gs = g5 ? stencil_grid(g.V / 2) : matvec_grid(g.V / 2);
  const double k2 = kappa * kappa;
  hop<-1, EO_TMP, double2>(tmp, p, Ueo, g, 1, 0.0, nullptr, nullptr, j, S, nullptr, G, st);
  if (g5) {
    hop<-1, EO_SIGMA5, double2>(Ap, tmp, Ueo, g, 0, k2, p, nullptr, j, S, region(rs, RG_SIGMA), Gs, st);
  } else {
    hop<-1, EO_SIGMA, double2>(Ap, tmp, Ueo, g, 0, k2, p, ph, j, S, region(rs, RG_SIGMA), Gs, st);
    hop<+1, EO_TMP, double2>(tmp, ph, Ueo, g, 1, 0.0, nullptr, nullptr, j, S, nullptr, G, st);
    hop<+1, EO_SCHUR, double2>(Adp, tmp, Ueo, g, 0, k2, ph, nullptr, j, S, nullptr, G, st);
  }
}

template <typename S>
void launch_stab_v_eo(S *v, const S *p, const S *rhat, S *tmp, const S *Ueo, const Geom &g, double kappa, int j,
                      KrylovState *K, const RedScratch &rs, hipStream_t st) {
  const int G = eo_grid(g);
  hop<-1, EO_TMP, S>(tmp, p, Ueo, g, 1, 0.0, nullptr, nullptr, j, K, nullptr, G, st);
  hop<-1, EO_SIGMA, S>(v, tmp, Ueo, g, 0, kappa * kappa, p, rhat, j, K, region(rs, RG_V), G, st);
}

template <typename S>
void launch_stab_t_eo(S *t, const S *sv, S *tmp, const S *Ueo, const Geom &g, double kappa, int j, KrylovState *K,
                      const RedScratch &rs, hipStream_t st) {
  const int G = eo_grid(g);
  hop<-1, EO_TMP, S>(tmp, sv, Ueo, g, 1, 0.0, nullptr, nullptr, j, K, nullptr, G, st);
  hop<-1, EO_STABT, S>(t, tmp, Ueo, g, 0, kappa * kappa, sv, nullptr, j, K, region(rs, RG_T), G, st);
}

template <typename S>
void launch_schur_eo_s(S *out, const S *in, S *tmp, const S *Ueo, const Geom &g, double kappa, bool dagger,
                       hipStream_t st) {
  const int G = eo_grid(g);
  if (dagger) {
    hop<+1, EO_TMP, S>(tmp, in, Ueo, g, 1, 0.0, nullptr, nullptr, 0, nullptr, nullptr, G, st);
    hop<+1, EO_SCHUR, S>(out, tmp, Ueo, g, 0, kappa * kappa, in, nullptr, 0, nullptr, nullptr, G, st);
  } else {
    hop<-1, EO_TMP, S>(tmp, in, Ueo, g, 1, 0.0, nullptr, nullptr, 0, nullptr, nullptr, G, st);
    hop<-1, EO_SCHUR, S>(out, tmp, Ueo, g, 0, kappa * kappa, in, nullptr, 0, nullptr, nullptr, G, st);
  }
}

template <typename S>
void launch_bschur_eo(S *out, const S *in, S *tmp, const S *Ueo, const Geom &g, double kappa, bool dagger, int kc,
                      hipStream_t st, int stage) {
  if (dagger) {
    bhop<+1, EO_TMP, S>(tmp, in, Ueo, g, 1, 0.0, nullptr, nullptr, 0, nullptr, nullptr, kc, st, stage);
    bhop<+1, EO_SCHUR, S>(out, tmp, Ueo, g, 0, kappa * kappa, in, nullptr, 0, nullptr, nullptr, kc, st, stage);
  } else {
    bhop<-1, EO_TMP, S>(tmp, in, Ueo, g, 1, 0.0, nullptr, nullptr, 0, nullptr, nullptr, kc, st, stage);
    bhop<-1, EO_SCHUR, S>(out, tmp, Ueo, g, 0, kappa * kappa, in, nullptr, 0, nullptr, nullptr, kc, st, stage);
  }
}

template <typename S>
void launch_bstab_v_eo(S *v, const S *p, const S *rhat, S *tmp, const S *Ueo, const Geom &g, double kappa, int j,
                       int kc, KrylovState *K, const RedScratch &rs, hipStream_t st, int stage) {
  bhop<-1, EO_TMP, S>(tmp, p, Ueo, g, 1, 0.0, nullptr, nullptr, j, K, nullptr, kc, st, stage);
  bhop<-1, EO_SIGMA, S>(v, tmp, Ueo, g, 0, kappa * kappa, p, rhat, j, K, region(rs, RG_V), kc, st, stage);
}

template <typename S>
void launch_bstab_t_eo(S *t, const S *sv, S *tmp, const S *Ueo, const Geom &g, double kappa, int j, int kc,
                       KrylovState *K, const RedScratch &rs, hipStream_t st, int stage) {
  bhop<-1, EO_TMP, S>(tmp, sv, Ueo, g, 1, 0.0, nullptr, nullptr, j, K, nullptr, kc, st, stage);
  bhop<-1, EO_STABT, S>(t, tmp, Ueo, g, 0, kappa * kappa, sv, nullptr, j, K, region(rs, RG_T), kc, st, stage);
}

#define EB_EO_INST(S)                                                                                              \
  template void launch_stab_v_eo<S>(S *, const S *, const S *, S *, const S *, const Geom &, double, int,          \
                                    KrylovState *, const RedScratch &, hipStream_t);                                \
  template void launch_stab_t_eo<S>(S *, const S *, S *, const S *, const Geom &, double, int, KrylovState *,       \
                                    const RedScratch &, hipStream_t);                                               \
  template void launch_schur_eo_s<S>(S *, const S *, S *, const S *, const Geom &, double, bool, hipStream_t);    \
  template void launch_bschur_eo<S>(S *, const S *, S *, const S *, const Geom &, double, bool, int, hipStream_t,  \
                                    int);                                                                          \
  template void launch_bstab_v_eo<S>(S *, const S *, const S *, S *, const S *, const Geom &, double, int, int,    \
                                     KrylovState *, const RedScratch &, hipStream_t, int);                        \
  template void launch_bstab_t_eo<S>(S *, const S *, S *, const S *, const Geom &, double, int, int,              \
                                     KrylovState *, const RedScratch &, hipStream_t, int);
EB_EO_INST(double2)
EB_EO_INST(float2)
EB_EO_INST(bf16c)

}  // namespace ebicg
