// HIP kernels for gfx950: layouts, the Wilson-Dirac stencil, the fused BiCG
// and BiCGStab passes with device-resident scalars, the window rotation of
// Alg. BiCG-eigen and the tall-skinny deflation projections.
//
// Internal layout (HBM): a spinor is SoA [12][V] complex (component c =
// spin*3 + colour), so every load instruction of a wavefront reads 64
// consecutive complex numbers; links are SoA [4][9][V] complex with the
// t-boundary factor folded into U_t at t = Lt-1.
//
// Reductions: a reducing kernel writes one partial record per block; the next
// kernel on the stream sums the records in a fixed order in its prologue (the
// same totals in every block, deterministic run to run) and its block 0
// records the resulting scalars.  There are no grid-wide fences or atomics,
// and no extra launches on the iteration path.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_common.h"
#include "kernels.h"
#include "kernel_util.h"
#include "stencil.h"

namespace ebicg {

namespace {

// ----------------------------------------------------------------------------
// Layout kernels
// ----------------------------------------------------------------------------
template <typename S>
__global__ void __launch_bounds__(kBlock) k_to_soa(S *__restrict__ dst, const S *__restrict__ src, int V) {
  const size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x;  // canonical index s*12 + c
  if (i >= size_t(V) * 12) return;
  const int s = int(i / 12), c = int(i % 12);
  dst[size_t(c) * V + s] = src[i];
}

template <typename S>
__global__ void __launch_bounds__(kBlock) k_from_soa(S *__restrict__ dst, const S *__restrict__ src, int V) {
  const size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x;  // canonical index s*12 + c
  if (i >= size_t(V) * 12) return;
  const int s = int(i / 12), c = int(i % 12);
  dst[i] = src[size_t(c) * V + s];
}

__global__ void __launch_bounds__(kBlock)
    k_pack_gauge(double2 *__restrict__ dst, const double2 *__restrict__ src, Geom g, int bc_t) {
  const size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x;  // canonical (mu*V + s)*9 + e
  if (i >= size_t(g.V) * 36) return;
  const int e = int(i % 9);
  const size_t ms = i / 9;
  const int mu = int(ms / g.V), s = int(ms % g.V);
  double2 u = src[i];
  if (mu == 3 && bc_t != 1 && s / (g.lx * g.ly * g.lz) == g.lt - 1) {
    u.x *= double(bc_t);
    u.y *= double(bc_t);
  }
  dst[size_t(mu * 9 + e) * g.V + s] = u;
}

template <typename D, typename Sx>
__global__ void __launch_bounds__(kBlock) k_convert(D *__restrict__ dst, const Sx *__restrict__ src, size_t n) {
  const size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= n) return;
  auto v = Store<Sx>::ld(src, i);
  cx<typename Store<D>::R> w{typename Store<D>::R(v.x), typename Store<D>::R(v.y)};
  Store<D>::st(dst, i, w);
}

// ----------------------------------------------------------------------------
// Operator kernels
// ----------------------------------------------------------------------------
template <typename S, int SF>
__global__ void __launch_bounds__(kBlock)
    k_dslash(S *__restrict__ out, const S *__restrict__ in, const S *__restrict__ U, Geom g, double kappa) {
  using R = typename Store<S>::R;
  __shared__ S tile[12 * kBlock];
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const R k = R(kappa);
  const int ntiles = (g.V + kBlock - 1) / kBlock;
  for (int T = lb; T < ntiles; T += gridDim.x) {
    const int s0 = T * kBlock, s = s0 + threadIdx.x;
    __syncthreads();  // the previous tile's readers are done
    stage_tile(tile, in, s0, g.V);
    __syncthreads();
    if (s < g.V) {
      cx<R> acc[12];
      hopping_t<SF, S>(acc, TileSrc<S>{in, tile, s0, g.V}, U, g, s);
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        const cx<R> v = Store<S>::ld(tile, size_t(c) * kBlock + threadIdx.x);
        Store<S>::st(out, size_t(c) * g.V + s, v - k * acc[c]);
      }
    }
  }
}

// r = b - D x with partials of ||r||^2 and ||b||^2 (FP64)
__global__ void __launch_bounds__(kBlock)
    k_residual(double2 *__restrict__ r, const double2 *__restrict__ b, const double2 *__restrict__ xin,
               const double2 *__restrict__ U, Geom g, double kappa, double *__restrict__ part) {
  __shared__ double2 tile[12 * kBlock];
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  double v[2] = {0.0, 0.0};
  const int ntiles = (g.V + kBlock - 1) / kBlock;
  for (int T = lb; T < ntiles; T += gridDim.x) {
    const int s0 = T * kBlock, s = s0 + threadIdx.x;
    __syncthreads();
    stage_tile(tile, xin, s0, g.V);
    __syncthreads();
    if (s >= g.V) continue;
    cx<double> acc[12];
    hopping_t<-1, double2>(acc, TileSrc<double2>{xin, tile, s0, g.V}, U, g, s);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const size_t i = size_t(c) * g.V + s;
      const cx<double> xv = Store<double2>::ld(tile, size_t(c) * kBlock + threadIdx.x), bv = Store<double2>::ld(b, i);
      const cx<double> rv = bv - (xv - kappa * acc[c]);
      Store<double2>::st(r, i, rv);
      v[0] += rv.x * rv.x + rv.y * rv.y;
      v[1] += bv.x * bv.x + bv.y * bv.y;
    }
  }
  block_partial<2, kBlock>(v, part, blockIdx.x);
}

// sum of partial records -> out (one block)
template <int NV>
__global__ void __launch_bounds__(kBlock) k_finish(const double *__restrict__ part, int nblk, double *out) {
  double v[NV];
  sum_partials<NV, kBlock>(part, nblk, v);
  if (threadIdx.x == 0)
    for (int i = 0; i < NV; ++i) out[i] = v[i];
}

// ----------------------------------------------------------------------------
// BiCG (Alg. eigBiCG loop), FP64.  Iteration j: matvec -> update_r -> update_p.
// ----------------------------------------------------------------------------
// rhat_mode 0: rhat_0 = r_0; 1: rhat_0 = gamma5 r_0; 2: gamma5 r_0 as well, but
// the shadow vectors are never formed (rhat and ph are not written).
__global__ void __launch_bounds__(kBlock)
    k_bicg_init(double2 *__restrict__ rhat, double2 *__restrict__ p, double2 *__restrict__ ph,
                const double2 *__restrict__ r, size_t N, int rhat_mode, double *__restrict__ part) {
  double v[2] = {0.0, 0.0};
  for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < N; i += size_t(gridDim.x) * kBlock) {
    cx<double> rv = Store<double2>::ld(r, i);
    // gamma5 = diag(1, 1, -1, -1): components 6..11 of the SoA layout, the
    // second half of the spinor (N = 12 V, or 12 V / 2 on the even sites), flip sign
    cx<double> hv = (rhat_mode != 0 && i >= N / 2) ? -rv : rv;
    Store<double2>::st(p, i, rv);
    if (rhat_mode != 2) {
      Store<double2>::st(rhat, i, hv);
      Store<double2>::st(ph, i, hv);
    }
    cx<double> d = cmulc(hv, rv);
    v[0] += d.x;
    v[1] += d.y;
  }
  block_partial<2, kBlock>(v, part, blockIdx.x);
}

__global__ void __launch_bounds__(kBlock)
    k_bicg_init_finish(const double *__restrict__ part_rho, int nb_rho, const double *__restrict__ res, double tol,
                       int maxiter, KrylovState *S, KrylovHistory h) {
  double v[2];
  sum_partials<2, kBlock>(part_rho, nb_rho, v);
  if (threadIdx.x != 0) return;
  const double rn = sqrt(res[0]), bn = sqrt(res[1]);
  h.rho[0] = make_double2(v[0], v[1]);
  h.rn[0] = rn;
  S->bnorm = bn;
  S->tol_abs = tol * bn;
  S->def_thr = 0;
  S->rnorm = rn;
  S->maxiter = maxiter;
  S->stopped = 0;
  S->stop_at = 0;
  S->reason = 0;
  if (rn <= S->tol_abs) {
    S->stopped = 1;
    S->reason = 1;
  } else if (v[0] == 0.0 && v[1] == 0.0) {
    S->stopped = 1;
    S->reason = 2;
  }
}

// Ap = D p with the partials of sigma = (phat, Ap), and Adp = D^+ phat.
// G5 (the gamma5-Hermitian form, Sec. 4): phat = gamma5 p is never formed and
// D^+ phat = gamma5 D p is not computed; sigma = (gamma5 p, Ap) takes p from
// the staged tile, and the work items are the tiles alone.
// Work item w is one LDS-staged pass over tile w / 2: D p for even w, D^+ phat
// for odd w, so both passes of a tile run on the same XCD (the links stay in
// its L2) and a 16^3 x 32 lattice gives 1024 blocks instead of 512.  The
// register budget of two waves per SIMD lets the compiler overlap the loads
// of several hops; at this lattice size the grid holds no more waves anyway.
template <bool G5>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1, 2)))
    k_bicg_matvec(double2 *__restrict__ Ap, double2 *__restrict__ Adp, const double2 *__restrict__ p,
                  const double2 *__restrict__ ph, const double2 *__restrict__ U, Geom g, double kappa, int j,
                  const KrylovState *S, double *__restrict__ part) {
  if (skip_iter(S, j)) return;
  __shared__ double2 tile[12 * kBlock];
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  double v[2] = {0.0, 0.0};
  const int ntiles = (g.V + kBlock - 1) / kBlock;
  constexpr int kItems = G5 ? 1 : 2;  // work items per tile
  for (int w = lb; w < kItems * ntiles; w += gridDim.x) {
    const int T = G5 ? w : w >> 1, s0 = T * kBlock, s = s0 + threadIdx.x;
    const bool adj = !G5 && (w & 1) != 0;
    __syncthreads();
    stage_tile(tile, adj ? ph : p, s0, g.V);
    __syncthreads();
    if (s >= g.V) continue;
    cx<double> acc[12];
    if (!adj) {
      hopping_t<-1, double2>(acc, TileSrc<double2>{p, tile, s0, g.V}, U, g, s);
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        const size_t i = size_t(c) * g.V + s;
        const cx<double> pv = Store<double2>::ld(tile, size_t(c) * kBlock + threadIdx.x);
        const cx<double> o = pv - kappa * acc[c];
        Store<double2>::st(Ap, i, o);
        const cx<double> d = G5 ? (c < 6 ? cmulc(pv, o) : -cmulc(pv, o)) : cmulc(Store<double2>::ld(ph, i), o);
        v[0] += d.x;
        v[1] += d.y;
      }
    } else {
      hopping_t<+1, double2>(acc, TileSrc<double2>{ph, tile, s0, g.V}, U, g, s);
#pragma unroll
      for (int c = 0; c < 12; ++c)
        Store<double2>::st(Adp, size_t(c) * g.V + s,
                           Store<double2>::ld(tile, size_t(c) * kBlock + threadIdx.x) - kappa * acc[c]);
    }
  }
  block_partial<2, kBlock>(v, part, blockIdx.x);
}

// G5: rhat = gamma5 r is not formed; rho = (gamma5 r, r).
template <bool G5>
__global__ void __launch_bounds__(kBlock)
    k_bicg_update_r(double2 *__restrict__ r_out, double2 *__restrict__ rh_out, const double2 *__restrict__ r_in,
                    const double2 *__restrict__ rh_in, const double2 *__restrict__ Ap,
                    const double2 *__restrict__ Adp, size_t N, int j, KrylovState *S, KrylovHistory h,
                    const double *__restrict__ part_sigma, int nb_sigma, double *__restrict__ part,
                    float2 *__restrict__ w32r, float2 *__restrict__ w32rh) {
  if (skip_iter(S, j)) return;
  double sg[2];
  sum_partials<2, kBlock>(part_sigma, nb_sigma, sg);
  const cx<double> sigma{sg[0], sg[1]};
  const double den = sigma.x * sigma.x + sigma.y * sigma.y;
  if (!(den > 0.0) || !isfinite(den)) {  // (phat, A p) = 0: breakdown
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      S->stopped = 1;
      S->stop_at = j - 1;
      S->reason = 2;
    }
    return;
  }
  const cx<double> a = cdiv(c2(h.rho[j - 1]), sigma);
  if (blockIdx.x == 0 && threadIdx.x == 0) h.alpha[j - 1] = d2(a);
  const cx<double> ac = cconj(a);
  double v[3] = {0.0, 0.0, 0.0};
  const size_t half = N / 2;  // gamma5 flips components 6..11 (N = 12 V)
  for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < N; i += size_t(gridDim.x) * kBlock) {
    cx<double> r = Store<double2>::ld(r_in, i) - a * Store<double2>::ld(Ap, i);
    Store<double2>::st(r_out, i, r);
    if (w32r) Store<float2>::st(w32r, i, r);
    const double rr = r.x * r.x + r.y * r.y;
    if constexpr (G5) {
      v[0] += i < half ? rr : -rr;
    } else {
      cx<double> rh = Store<double2>::ld(rh_in, i) - ac * Store<double2>::ld(Adp, i);
      Store<double2>::st(rh_out, i, rh);
      if (w32rh) Store<float2>::st(w32rh, i, rh);
      cx<double> d = cmulc(rh, r);
      v[0] += d.x;
      v[1] += d.y;
    }
    v[2] += rr;
  }
  block_partial<3, kBlock>(v, part, blockIdx.x);
}

// G5: phat = gamma5 p is not formed.
template <bool G5>
__global__ void __launch_bounds__(kBlock)
    k_bicg_update_p(double2 *__restrict__ x, double2 *__restrict__ p, double2 *__restrict__ ph,
                    const double2 *__restrict__ r, const double2 *__restrict__ rh, size_t N, int j, KrylovState *S,
                    KrylovHistory h, const double *__restrict__ part_rr, int nb_rr) {
  if (skip_iter(S, j)) return;
  double rr[3];
  sum_partials<3, kBlock>(part_rr, nb_rr, rr);
  const cx<double> rho_new{rr[0], rr[1]};
  const cx<double> a = c2(h.alpha[j - 1]);
  const cx<double> b = cdiv(rho_new, c2(h.rho[j - 1]));
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const double rnorm = sqrt(rr[2]);
    h.beta[j - 1] = d2(b);
    h.rho[j] = d2(rho_new);
    h.rn[j] = rnorm;
    S->rnorm = rnorm;
    if (rnorm <= S->tol_abs) {
      S->stopped = 1;
      S->stop_at = j;
      S->reason = 1;
    } else if (rho_new.x == 0.0 && rho_new.y == 0.0) {
      S->stopped = 1;
      S->stop_at = j;
      S->reason = 2;
    } else if (j >= S->maxiter) {
      S->stopped = 1;
      S->stop_at = j;
      S->reason = 4;
    }
  }
  const cx<double> bc = cconj(b);
  for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < N; i += size_t(gridDim.x) * kBlock) {
    cx<double> pv = Store<double2>::ld(p, i);
    Store<double2>::st(x, i, Store<double2>::ld(x, i) + a * pv);
    Store<double2>::st(p, i, Store<double2>::ld(r, i) + b * pv);
    if constexpr (!G5) Store<double2>::st(ph, i, Store<double2>::ld(rh, i) + bc * Store<double2>::ld(ph, i));
  }
}

// G5: D^+ phat = gamma5 D p, so GA = gamma5 (Ap - conj(beta) q) from the A p
// buffers (Adp and s are not read).
template <bool G5>
__global__ void __launch_bounds__(kBlock)
    k_arrow_vectors(double2 *__restrict__ GA, double2 *__restrict__ GB, const double2 *__restrict__ Adp,
                    const double2 *__restrict__ s, const double2 *__restrict__ Ap, const double2 *__restrict__ q,
                    size_t N, int j, const KrylovState *S, KrylovHistory h) {
  if (skip_iter(S, j)) return;
  const cx<double> b = c2(h.beta[j - 2]), bc = cconj(b);
  const size_t half = N / 2;
  for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < N; i += size_t(gridDim.x) * kBlock) {
    const cx<double> apv = Store<double2>::ld(Ap, i), qv = Store<double2>::ld(q, i);
    if constexpr (G5) {
      const cx<double> ga = apv - bc * qv;
      Store<double2>::st(GA, i, i < half ? ga : -ga);
    } else {
      Store<double2>::st(GA, i, Store<double2>::ld(Adp, i) - bc * Store<double2>::ld(s, i));
    }
    Store<double2>::st(GB, i, apv - b * qv);
  }
}

// partials of out[a + b*nx] = sum_i conj(X_a[i]) Y_b[i] over a tile XT x YT.
template <int XT, int YT>
__global__ void __launch_bounds__(kBlock)
    k_ts_dot(const double2 *__restrict__ X, size_t ldx, int nx, const double2 *__restrict__ Y, size_t ldy, int ny,
             size_t N, double *__restrict__ part) {
  const int a0 = blockIdx.y * XT, b0 = blockIdx.z * YT;
  double v[2 * XT * YT];
#pragma unroll
  for (int e = 0; e < 2 * XT * YT; ++e) v[e] = 0.0;
  for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < N; i += size_t(gridDim.x) * kBlock) {
    cx<double> yv[YT];
#pragma unroll
    for (int b = 0; b < YT; ++b)
      yv[b] = (b0 + b < ny) ? Store<double2>::ld(Y + size_t(b0 + b) * ldy, i) : cx<double>{0, 0};
#pragma unroll
    for (int a = 0; a < XT; ++a) {
      if (a0 + a < nx) {
        const cx<double> xv = Store<double2>::ld(X + size_t(a0 + a) * ldx, i);
#pragma unroll
        for (int b = 0; b < YT; ++b) {
          cx<double> d = cmulc(xv, yv[b]);
          v[2 * (a * YT + b)] += d.x;
          v[2 * (a * YT + b) + 1] += d.y;
        }
      }
    }
  }
  const int tile = blockIdx.y + gridDim.y * blockIdx.z;
  block_partial<2 * XT * YT, kBlock>(v, part + size_t(tile) * gridDim.x * 2 * XT * YT, blockIdx.x);
}

template <int XT, int YT>
__global__ void __launch_bounds__(kBlock)
    k_ts_dot_finish(double2 *out, const double *__restrict__ part, int nblk, int nx, int ny, int tiles_x) {
  double v[2 * XT * YT];
  const int tile = blockIdx.x;
  sum_partials<2 * XT * YT, kBlock>(part + size_t(tile) * nblk * 2 * XT * YT, nblk, v);
  const int a0 = (tile % tiles_x) * XT, b0 = (tile / tiles_x) * YT;
  if (threadIdx.x == 0)
    for (int a = 0; a < XT; ++a)
      for (int b = 0; b < YT; ++b)
        if (a0 + a < nx && b0 + b < ny)
          out[(a0 + a) + size_t(b0 + b) * nx] = make_double2(v[2 * (a * YT + b)], v[2 * (a * YT + b) + 1]);
}

// y += sgn * sum_a X_a c[a] (one column; wider blocks use the matrix cores)
__global__ void __launch_bounds__(kBlock)
    k_ts_update1(double2 *__restrict__ y, int nx, const double2 *__restrict__ X, size_t ldx,
                 const double2 *__restrict__ c, double sgn, size_t N) {
  __shared__ double2 sC[kMaxCols];
  for (int a = threadIdx.x; a < nx; a += kBlock) sC[a] = make_double2(sgn * c[a].x, sgn * c[a].y);
  __syncthreads();
  for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < N; i += size_t(gridDim.x) * kBlock) {
    cx<double> acc{0, 0};
    for (int a = 0; a < nx; ++a) {
      const double2 cc = sC[a];
      cfma(acc, Store<double2>::ld(X + size_t(a) * ldx, i), cx<double>{cc.x, cc.y});
    }
    Store<double2>::st(y, i, Store<double2>::ld(y, i) + acc);
  }
}

__global__ void __launch_bounds__(kBlock) k_copy(double2 *__restrict__ d, const double2 *__restrict__ s, size_t n) {
  for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += size_t(gridDim.x) * kBlock) d[i] = s[i];
}
__global__ void __launch_bounds__(kBlock) k_scale(double2 *__restrict__ x, double2 a, size_t n) {
  const cx<double> av{a.x, a.y};
  for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += size_t(gridDim.x) * kBlock)
    Store<double2>::st(x, i, av * Store<double2>::ld(x, i));
}
__global__ void __launch_bounds__(kBlock) k_add(double2 *__restrict__ y, const double2 *__restrict__ x, size_t n) {
  for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += size_t(gridDim.x) * kBlock)
    Store<double2>::st(y, i, Store<double2>::ld(y, i) + Store<double2>::ld(x, i));
}

// ----------------------------------------------------------------------------
// BiCGStab (van der Vorst), storage S, FP64 reductions and scalars.
// Iteration j: v -> s -> t -> xr -> p.
// ----------------------------------------------------------------------------
template <typename S>
__global__ void __launch_bounds__(kBlock)
    k_stab_init(S *__restrict__ rhat, S *__restrict__ p, const S *__restrict__ r, size_t N,
                double *__restrict__ part) {
  double v[1] = {0.0};
  for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < N; i += size_t(gridDim.x) * kBlock) {
    auto rv = Store<S>::ld(r, i);
    Store<S>::st(rhat, i, rv);
    Store<S>::st(p, i, rv);
    v[0] += double(rv.x) * rv.x + double(rv.y) * rv.y;
  }
  block_partial<1, kBlock>(v, part, blockIdx.x);
}

__global__ void __launch_bounds__(kBlock)
    k_stab_init_finish(const double *__restrict__ part, int nblk, double tol_abs, double def_thr, int maxiter,
                       KrylovState *K, KrylovHistory h) {
  double v[1];
  sum_partials<1, kBlock>(part, nblk, v);
  if (threadIdx.x != 0) return;
  h.rho[0] = make_double2(v[0], 0.0);
  h.rn[0] = sqrt(v[0]);
  K->rnorm = sqrt(v[0]);
  K->tol_abs = tol_abs;
  K->def_thr = def_thr;
  K->maxiter = maxiter;
  K->stopped = 0;
  K->stop_at = 0;
  K->reason = 0;
  if (K->rnorm <= tol_abs) {
    K->stopped = 1;
    K->reason = 1;
  }
}

// v = D p ; partials of (rhat, v)
template <typename S>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1, 2)))
    k_stab_v(S *__restrict__ vout, const S *__restrict__ p, const S *__restrict__ rhat, const S *__restrict__ U,
             Geom g, double kappa, int j, const KrylovState *K, double *__restrict__ part) {
  using R = typename Store<S>::R;
  if (skip_iter(K, j)) return;
  __shared__ S tile[12 * kBlock];
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const R k = R(kappa);
  double v[2] = {0.0, 0.0};
  const int ntiles = (g.V + kBlock - 1) / kBlock;
  for (int T = lb; T < ntiles; T += gridDim.x) {
    const int s0 = T * kBlock, s = s0 + threadIdx.x;
    __syncthreads();
    stage_tile(tile, p, s0, g.V);
    __syncthreads();
    if (s >= g.V) continue;
    cx<R> acc[12];
    hopping_t<-1, S>(acc, TileSrc<S>{p, tile, s0, g.V}, U, g, s);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const size_t i = size_t(c) * g.V + s;
      const cx<R> o = Store<S>::ld(tile, size_t(c) * kBlock + threadIdx.x) - k * acc[c];
      Store<S>::st(vout, i, o);
      const cx<R> hh = Store<S>::ld(rhat, i);
      v[0] += double(hh.x) * o.x + double(hh.y) * o.y;
      v[1] += double(hh.x) * o.y - double(hh.y) * o.x;
    }
  }
  block_partial<2, kBlock>(v, part, blockIdx.x);
}

// alpha_j = rho_{j-1} / (rhat, v) ; s = r - alpha v
template <typename S>
__global__ void __launch_bounds__(kBlock)
    k_stab_s(S *__restrict__ sv, const S *__restrict__ r, const S *__restrict__ v, size_t N, int j, KrylovState *K,
             KrylovHistory h, const double *__restrict__ part_v, int nb_v) {
  using R = typename Store<S>::R;
  if (skip_iter(K, j)) return;
  double d[2];
  sum_partials<2, kBlock>(part_v, nb_v, d);
  const cx<double> den{d[0], d[1]};
  const double dd = den.x * den.x + den.y * den.y;
  if (!(dd > 0.0) || !isfinite(dd)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      K->stopped = 1;
      K->stop_at = j - 1;
      K->reason = 2;
    }
    return;
  }
  const cx<double> al = cdiv(c2(h.rho[j - 1]), den);
  if (blockIdx.x == 0 && threadIdx.x == 0) h.alpha[j] = d2(al);
  const cx<R> a{R(al.x), R(al.y)};
  for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < N; i += size_t(gridDim.x) * kBlock)
    Store<S>::st(sv, i, Store<S>::ld(r, i) - a * Store<S>::ld(v, i));
}

// t = D s ; partials of (t, s), (t, t)
template <typename S>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1, 2)))
    k_stab_t(S *__restrict__ tout, const S *__restrict__ sv, const S *__restrict__ U, Geom g, double kappa, int j,
             const KrylovState *K, double *__restrict__ part) {
  using R = typename Store<S>::R;
  if (skip_iter(K, j)) return;
  __shared__ S tile[12 * kBlock];
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const R k = R(kappa);
  double v[3] = {0.0, 0.0, 0.0};
  const int ntiles = (g.V + kBlock - 1) / kBlock;
  for (int T = lb; T < ntiles; T += gridDim.x) {
    const int s0 = T * kBlock, s = s0 + threadIdx.x;
    __syncthreads();
    stage_tile(tile, sv, s0, g.V);
    __syncthreads();
    if (s >= g.V) continue;
    cx<R> acc[12];
    hopping_t<-1, S>(acc, TileSrc<S>{sv, tile, s0, g.V}, U, g, s);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const size_t i = size_t(c) * g.V + s;
      const cx<R> si = Store<S>::ld(tile, size_t(c) * kBlock + threadIdx.x);
      const cx<R> o = si - k * acc[c];
      Store<S>::st(tout, i, o);
      v[0] += double(o.x) * si.x + double(o.y) * si.y;
      v[1] += double(o.x) * si.y - double(o.y) * si.x;
      v[2] += double(o.x) * o.x + double(o.y) * o.y;
    }
  }
  block_partial<3, kBlock>(v, part, blockIdx.x);
}

// omega_j = (t, s) / (t, t) ; x += alpha p + omega s ; r = s - omega t ; partials of (rhat, r), ||r||^2
template <typename S>
__global__ void __launch_bounds__(kBlock)
    k_stab_xr(S *__restrict__ x, S *__restrict__ r, const S *__restrict__ p, const S *__restrict__ sv,
              const S *__restrict__ t, const S *__restrict__ rhat, size_t N, int j, KrylovState *K,
              KrylovHistory h, const double *__restrict__ part_t, int nb_t, double *__restrict__ part) {
  using R = typename Store<S>::R;
  if (skip_iter(K, j)) return;
  double d[3];
  sum_partials<3, kBlock>(part_t, nb_t, d);
  if (!(d[2] > 0.0)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      K->stopped = 1;
      K->stop_at = j - 1;
      K->reason = 2;
    }
    return;
  }
  const cx<double> om{d[0] / d[2], d[1] / d[2]};
  if (blockIdx.x == 0 && threadIdx.x == 0) h.omega[j] = d2(om);
  const cx<double> al = c2(h.alpha[j]);
  const cx<R> a{R(al.x), R(al.y)}, w{R(om.x), R(om.y)};
  double v[3] = {0.0, 0.0, 0.0};
  for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < N; i += size_t(gridDim.x) * kBlock) {
    const cx<R> si = Store<S>::ld(sv, i);
    Store<S>::st(x, i, Store<S>::ld(x, i) + a * Store<S>::ld(p, i) + w * si);
    const cx<R> ri = si - w * Store<S>::ld(t, i);
    Store<S>::st(r, i, ri);
    const cx<R> hh = Store<S>::ld(rhat, i);
    v[0] += double(hh.x) * ri.x + double(hh.y) * ri.y;
    v[1] += double(hh.x) * ri.y - double(hh.y) * ri.x;
    v[2] += double(ri.x) * ri.x + double(ri.y) * ri.y;
  }
  block_partial<3, kBlock>(v, part, blockIdx.x);
}

// rho_j, beta_j = (rho_j / rho_{j-1}) (alpha_j / omega_j), stop tests ; p = r + beta (p - omega v)
template <typename S>
__global__ void __launch_bounds__(kBlock)
    k_stab_p(S *__restrict__ p, const S *__restrict__ r, const S *__restrict__ v, size_t N, int j, KrylovState *K,
             KrylovHistory h, const double *__restrict__ part_xr, int nb_xr) {
  using R = typename Store<S>::R;
  if (skip_iter(K, j)) return;
  double d[3];
  sum_partials<3, kBlock>(part_xr, nb_xr, d);
  const cx<double> rho{d[0], d[1]};
  const cx<double> om = c2(h.omega[j]);
  const cx<double> be = cdiv(rho, c2(h.rho[j - 1])) * cdiv(c2(h.alpha[j]), om);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const double rnorm = sqrt(d[2]);
    h.rho[j] = d2(rho);
    h.beta[j] = d2(be);
    h.rn[j] = rnorm;
    K->rnorm = rnorm;
    if (rnorm <= K->tol_abs) {
      K->stopped = 1;
      K->stop_at = j;
      K->reason = 1;
    } else if (K->def_thr > 0.0 && rnorm < K->def_thr) {
      K->stopped = 1;
      K->stop_at = j;
      K->reason = 3;
    } else if (rho.x == 0.0 && rho.y == 0.0) {
      K->stopped = 1;
      K->stop_at = j;
      K->reason = 2;
    } else if (j >= K->maxiter) {
      K->stopped = 1;
      K->stop_at = j;
      K->reason = 4;
    }
  }
  const cx<R> b{R(be.x), R(be.y)}, w{R(om.x), R(om.y)};
  for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < N; i += size_t(gridDim.x) * kBlock)
    Store<S>::st(p, i, Store<S>::ld(r, i) + b * (Store<S>::ld(p, i) - w * Store<S>::ld(v, i)));
}

}  // namespace

// ============================================================================
// launch wrappers
// ============================================================================
LaunchStamp &launch_stamp() {
  static thread_local LaunchStamp ls;
  return ls;
}
int &stencil_block_cap() {
  static thread_local int cap = kDefaultStencilCap;
  return cap;
}

void launch_to_soa_f64(double2 *d, const double2 *s, const Geom &g, hipStream_t st) {
  EB_LAUNCH(k_to_soa<double2>, dim3(nblocks_for(size_t(g.V) * 12)), dim3(kBlock), 0, st, d, s, g.V);
}
void launch_from_soa_f64(double2 *d, const double2 *s, const Geom &g, hipStream_t st) {
  EB_LAUNCH(k_from_soa<double2>, dim3(nblocks_for(size_t(g.V) * 12)), dim3(kBlock), 0, st, d, s, g.V);
}
void launch_to_soa_f32(float2 *d, const float2 *s, const Geom &g, hipStream_t st) {
  EB_LAUNCH(k_to_soa<float2>, dim3(nblocks_for(size_t(g.V) * 12)), dim3(kBlock), 0, st, d, s, g.V);
}
void launch_from_soa_f32(float2 *d, const float2 *s, const Geom &g, hipStream_t st) {
  EB_LAUNCH(k_from_soa<float2>, dim3(nblocks_for(size_t(g.V) * 12)), dim3(kBlock), 0, st, d, s, g.V);
}
void launch_pack_gauge_f64(double2 *d, const double2 *s, const Geom &g, int bc_t, hipStream_t st) {
  EB_LAUNCH(k_pack_gauge, dim3(nblocks_for(size_t(g.V) * 36)), dim3(kBlock), 0, st, d, s, g, bc_t);
}
void launch_convert_f64_f32(float2 *d, const double2 *s, size_t n, hipStream_t st) {
  EB_LAUNCH((k_convert<float2, double2>), dim3(nblocks_for(n)), dim3(kBlock), 0, st, d, s, n);
}
void launch_convert_f32_f64(double2 *d, const float2 *s, size_t n, hipStream_t st) {
  EB_LAUNCH((k_convert<double2, float2>), dim3(nblocks_for(n)), dim3(kBlock), 0, st, d, s, n);
}

template <typename S>
static void dslash_any(S *out, const S *in, const S *U, const Geom &g, double kappa, bool dagger, hipStream_t st) {
  dim3 grid(nblocks_for(g.V));
  if (dagger)
    EB_LAUNCH((k_dslash<S, +1>), grid, dim3(kBlock), 0, st, out, in, U, g, kappa);
  else
    EB_LAUNCH((k_dslash<S, -1>), grid, dim3(kBlock), 0, st, out, in, U, g, kappa);
}
void launch_dslash_f64(double2 *o, const double2 *i, const double2 *U, const Geom &g, double k, bool d, hipStream_t st) {
  dslash_any(o, i, U, g, k, d, st);
}
void launch_dslash_f32(float2 *o, const float2 *i, const float2 *U, const Geom &g, double k, bool d, hipStream_t st) {
  dslash_any(o, i, U, g, k, d, st);
}
void launch_dslash_bf16(bf16c *o, const bf16c *i, const bf16c *U, const Geom &g, double k, bool d, hipStream_t st) {
  dslash_any(o, i, U, g, k, d, st);
}
void launch_to_soa_bf16(bf16c *d, const bf16c *s, const Geom &g, hipStream_t st) {
  EB_LAUNCH(k_to_soa<bf16c>, dim3(nblocks_for(size_t(g.V) * 12)), dim3(kBlock), 0, st, d, s, g.V);
}
void launch_from_soa_bf16(bf16c *d, const bf16c *s, const Geom &g, hipStream_t st) {
  EB_LAUNCH(k_from_soa<bf16c>, dim3(nblocks_for(size_t(g.V) * 12)), dim3(kBlock), 0, st, d, s, g.V);
}
void launch_convert_f64_bf16(bf16c *d, const double2 *s, size_t n, hipStream_t st) {
  EB_LAUNCH((k_convert<bf16c, double2>), dim3(nblocks_for(n)), dim3(kBlock), 0, st, d, s, n);
}
void launch_convert_bf16_f64(double2 *d, const bf16c *s, size_t n, hipStream_t st) {
  EB_LAUNCH((k_convert<double2, bf16c>), dim3(nblocks_for(n)), dim3(kBlock), 0, st, d, s, n);
}

void launch_residual_f64(double2 *r, const double2 *b, const double2 *x, const double2 *U, const Geom &g, double kappa,
                         double *res, const RedScratch &rs, hipStream_t st) {
  const int nb = stencil_grid(g.V);
  EB_LAUNCH(k_residual, dim3(nb), dim3(kBlock), 0, st, r, b, x, U, g, kappa, region(rs, RG_RES));
  EB_LAUNCH(k_finish<2>, dim3(1), dim3(kBlock), 0, st, region(rs, RG_RES), nb, res);
}

void launch_bicg_init(double2 *rhat, double2 *p, double2 *ph, const double2 *r, const double *res, size_t N,
                      int rhat_mode, const Geom &g, double tol, int maxiter, KrylovState *S, KrylovHistory h,
                      const RedScratch &rs, hipStream_t st) {
  const int nb = red_grid(N);
  EB_LAUNCH(k_bicg_init, dim3(nb), dim3(kBlock), 0, st, rhat, p, ph, r, N, rhat_mode, region(rs, RG_INIT));
  EB_LAUNCH(k_bicg_init_finish, dim3(1), dim3(kBlock), 0, st, region(rs, RG_INIT), nb, res, tol, maxiter, S, h);
}
void launch_bicg_matvec(double2 *Ap, double2 *Adp, const double2 *p, const double2 *ph, const double2 *U,
                        const Geom &g, double kappa, int j, KrylovState *S, KrylovHistory, const RedScratch &rs,
                        bool g5, hipStream_t st) {
  if (g5)
    EB_LAUNCH(k_bicg_matvec<true>, dim3(stencil_grid(g.V)), dim3(kBlock), 0, st, Ap, Adp, p, ph, U, g, kappa, j, S,
              region(rs, RG_SIGMA));
  else
    EB_LAUNCH(k_bicg_matvec<false>, dim3(matvec_grid(g.V)), dim3(kBlock), 0, st, Ap, Adp, p, ph, U, g, kappa, j, S,
              region(rs, RG_SIGMA));
}
void launch_bicg_update_r(double2 *r_out, double2 *rh_out, const double2 *r_in, const double2 *rh_in,
                          const double2 *Ap, const double2 *Adp, size_t N, int j, KrylovState *S, KrylovHistory h,
                          const RedScratch &rs, bool g5, hipStream_t st, float2 *w32r, float2 *w32rh, int nrec) {
  // the matvec wrote one sigma record per block of its grid; N = 12 V
  const int V = int(N / 12);
  if (g5)
    EB_LAUNCH(k_bicg_update_r<true>, dim3(red_grid(N)), dim3(kBlock), 0, st, r_out, rh_out, r_in, rh_in, Ap, Adp, N,
              j, S, h, region(rs, RG_SIGMA), nrec > 0 ? nrec : stencil_grid(V), region(rs, RG_RR), w32r, w32rh);
  else
    EB_LAUNCH(k_bicg_update_r<false>, dim3(red_grid(N)), dim3(kBlock), 0, st, r_out, rh_out, r_in, rh_in, Ap, Adp, N,
              j, S, h, region(rs, RG_SIGMA), nrec > 0 ? nrec : matvec_grid(V), region(rs, RG_RR), w32r, w32rh);
}
void launch_bicg_update_p(double2 *x, double2 *p, double2 *ph, const double2 *r, const double2 *rh, size_t N, int j,
                          KrylovState *S, KrylovHistory h, const RedScratch &rs, bool g5, hipStream_t st) {
  if (g5)
    EB_LAUNCH(k_bicg_update_p<true>, dim3(stream_grid(N)), dim3(kBlock), 0, st, x, p, ph, r, rh, N, j, S, h,
              region(rs, RG_RR), red_grid(N));
  else
    EB_LAUNCH(k_bicg_update_p<false>, dim3(stream_grid(N)), dim3(kBlock), 0, st, x, p, ph, r, rh, N, j, S, h,
              region(rs, RG_RR), red_grid(N));
}
void launch_arrow_vectors(double2 *GA, double2 *GB, const double2 *Adp, const double2 *s, const double2 *Ap,
                          const double2 *q, size_t N, int j, const KrylovState *S, KrylovHistory h, bool g5,
                          hipStream_t st) {
  if (g5)
    EB_LAUNCH(k_arrow_vectors<true>, dim3(stream_grid(N)), dim3(kBlock), 0, st, GA, GB, Adp, s, Ap, q, N, j, S, h);
  else
    EB_LAUNCH(k_arrow_vectors<false>, dim3(stream_grid(N)), dim3(kBlock), 0, st, GA, GB, Adp, s, Ap, q, N, j, S, h);
}

void launch_rotate(double2 *out_base, const SlotList &out_slots, const double2 *in_base, const SlotList &in_slots,
                   const double2 *C, size_t N, const double2 *g, int conj_out, double2 *dots, int jtag,
                   const KrylovState *S, const RedScratch &rs, hipStream_t st) {
  launch_combine(out_base, out_slots, N, in_base, in_slots, N, C, 1.0, false, N, g, conj_out, dots, jtag, S,
                      region(rs, RG_GEN), kMaxPartials - size_t(RG_GEN) * kRegion, st);
}
void launch_rotate(float2 *out_base, const SlotList &out_slots, const float2 *in_base, const SlotList &in_slots,
                   const double2 *C, size_t N, const double2 *g, int conj_out, double2 *dots, int jtag,
                   const KrylovState *S, const RedScratch &rs, hipStream_t st) {
  launch_combine(out_base, out_slots, N, in_base, in_slots, N, C, N, g, conj_out, dots, jtag, S, region(rs, RG_GEN),
                 kMaxPartials - size_t(RG_GEN) * kRegion, st);
}
void launch_rotate(double2 *out_base, const SlotList &out_slots, const float2 *in_base, const SlotList &in_slots,
                   const double2 *C, size_t N, const double2 *g, int conj_out, double2 *dots, int jtag,
                   const KrylovState *S, const RedScratch &rs, hipStream_t st) {
  launch_combine(out_base, out_slots, N, in_base, in_slots, N, C, N, g, conj_out, dots, jtag, S, region(rs, RG_GEN),
                 kMaxPartials - size_t(RG_GEN) * kRegion, st);
}

template <int XT, int YT>
static void ts_dot_tiled(double2 *out, const double2 *X, size_t ldx, int nx, const double2 *Y, size_t ldy, int ny,
                         size_t N, const RedScratch &rs, hipStream_t st) {
  const int tx = (nx + XT - 1) / XT, ty = (ny + YT - 1) / YT;
  const int tiles = tx * ty;
  // every tile keeps nb partial records of 2 XT YT doubles
  double *part = region(rs, RG_GEN);
  const size_t avail = kMaxPartials - size_t(RG_GEN) * kRegion;
  int nb = stream_grid(N);
  const int cap = int(avail / (size_t(tiles) * 2 * XT * YT));
  nb = nb < 1024 ? nb : 1024;
  nb = nb < cap ? nb : cap;
  nb = nb < 1 ? 1 : nb;
  EB_LAUNCH((k_ts_dot<XT, YT>), dim3(nb, tx, ty), dim3(kBlock), 0, st, X, ldx, nx, Y, ldy, ny, N, part);
  EB_LAUNCH((k_ts_dot_finish<XT, YT>), dim3(tiles), dim3(kBlock), 0, st, out, part, nb, nx, ny, tx);
}
// One or two Y columns: VALU tiles of 8 X columns (the products are HBM-bound
// and a matrix-core tile would be mostly padding); wider blocks: matrix cores.
void launch_ts_dot(double2 *out, const double2 *X, size_t ldx, int nx, const double2 *Y, size_t ldy, int ny, size_t N,
                   const RedScratch &rs, hipStream_t st) {
  if (ny == 1)
    ts_dot_tiled<8, 1>(out, X, ldx, nx, Y, ldy, ny, N, rs, st);
  else if (ny == 2 || nx > kMaxCols)
    ts_dot_tiled<8, 2>(out, X, ldx, nx, Y, ldy, ny, N, rs, st);
  else
    launch_gram_mfma(out, X, ldx, nx, Y, ldy, ny, N, region(rs, RG_GEN), kMaxPartials - size_t(RG_GEN) * kRegion,
                     st);
}
void launch_ts_update(double2 *Y, size_t ldy, int ny, const double2 *X, size_t ldx, int nx, const double2 *C,
                      double sgn, size_t N, hipStream_t st) {
  if (nx < 1 || ny < 1) return;
  if (ny == 1) {
    EB_LAUNCH(k_ts_update1, dim3(stream_grid(N)), dim3(kBlock), 0, st, Y, nx, X, ldx, C, sgn, N);
    return;
  }
  SlotList in{}, out{};
  in.n = nx;
  for (int a = 0; a < nx; ++a) in.idx[a] = a;
  out.n = ny;
  for (int b = 0; b < ny; ++b) out.idx[b] = b;
  launch_combine(Y, out, ldy, X, in, ldx, C, sgn, true, N, nullptr, 0, nullptr, 0, nullptr, nullptr, 0, st);
}

void launch_copy_f64(double2 *d, const double2 *s, size_t n, hipStream_t st) {
  EB_LAUNCH(k_copy, dim3(stream_grid(n)), dim3(kBlock), 0, st, d, s, n);
}
void launch_scale_f64(double2 *x, double2 a, size_t n, hipStream_t st) {
  EB_LAUNCH(k_scale, dim3(stream_grid(n)), dim3(kBlock), 0, st, x, a, n);
}
void launch_add_f64(double2 *y, const double2 *x, size_t n, hipStream_t st) {
  EB_LAUNCH(k_add, dim3(stream_grid(n)), dim3(kBlock), 0, st, y, x, n);
}

template <typename S>
void launch_stab_init(S *rhat, S *p, const S *r, size_t N, double tol_abs, double def_thr, int maxiter,
                      KrylovState *K, KrylovHistory h, const RedScratch &rs, hipStream_t st) {
  const int nb = red_grid(N);
  EB_LAUNCH(k_stab_init<S>, dim3(nb), dim3(kBlock), 0, st, rhat, p, r, N, region(rs, RG_INIT));
  EB_LAUNCH(k_stab_init_finish, dim3(1), dim3(kBlock), 0, st, region(rs, RG_INIT), nb, tol_abs, def_thr, maxiter, K,
            h);
}
template <typename S>
void launch_stab_v(S *v, const S *p, const S *rhat, const S *U, const Geom &g, double kappa, int j, KrylovState *K,
                   KrylovHistory, const RedScratch &rs, hipStream_t st) {
  EB_LAUNCH(k_stab_v<S>, dim3(stencil_grid(g.V)), dim3(kBlock), 0, st, v, p, rhat, U, g, kappa, j, K,
            region(rs, RG_V));
}
template <typename S>
void launch_stab_s(S *s, const S *r, const S *v, size_t N, int j, KrylovState *K, KrylovHistory h,
                   const RedScratch &rs, hipStream_t st, int nrec) {
  EB_LAUNCH(k_stab_s<S>, dim3(stream_grid(N)), dim3(kBlock), 0, st, s, r, v, N, j, K, h, region(rs, RG_V),
            nrec > 0 ? nrec : stencil_grid(int(N / 12)));
}
template <typename S>
void launch_stab_t(S *t, const S *s, const S *U, const Geom &g, double kappa, int j, KrylovState *K, KrylovHistory,
                   const RedScratch &rs, hipStream_t st) {
  EB_LAUNCH(k_stab_t<S>, dim3(stencil_grid(g.V)), dim3(kBlock), 0, st, t, s, U, g, kappa, j, K, region(rs, RG_T));
}
template <typename S>
void launch_stab_xr(S *x, S *r, const S *p, const S *s, const S *t, const S *rhat, size_t N, int j, KrylovState *K,
                    KrylovHistory h, const RedScratch &rs, hipStream_t st, int nrec) {
  EB_LAUNCH(k_stab_xr<S>, dim3(red_grid(N)), dim3(kBlock), 0, st, x, r, p, s, t, rhat, N, j, K, h, region(rs, RG_T),
            nrec > 0 ? nrec : stencil_grid(int(N / 12)), region(rs, RG_XR));
}
template <typename S>
void launch_stab_p(S *p, const S *r, const S *v, size_t N, int j, KrylovState *K, KrylovHistory h,
                   const RedScratch &rs, hipStream_t st) {
  EB_LAUNCH(k_stab_p<S>, dim3(stream_grid(N)), dim3(kBlock), 0, st, p, r, v, N, j, K, h, region(rs, RG_XR),
            red_grid(N));
}

#define EB_STAB_INST(S)                                                                                              \
  template void launch_stab_init<S>(S *, S *, const S *, size_t, double, double, int, KrylovState *, KrylovHistory, \
                                    const RedScratch &, hipStream_t);                                                \
  template void launch_stab_v<S>(S *, const S *, const S *, const S *, const Geom &, double, int, KrylovState *,    \
                                 KrylovHistory, const RedScratch &, hipStream_t);                                    \
  template void launch_stab_s<S>(S *, const S *, const S *, size_t, int, KrylovState *, KrylovHistory,              \
                                 const RedScratch &, hipStream_t, int);                                              \
  template void launch_stab_t<S>(S *, const S *, const S *, const Geom &, double, int, KrylovState *, KrylovHistory, \
                                 const RedScratch &, hipStream_t);                                                   \
  template void launch_stab_xr<S>(S *, S *, const S *, const S *, const S *, const S *, size_t, int, KrylovState *, \
                                  KrylovHistory, const RedScratch &, hipStream_t, int);                              \
  template void launch_stab_p<S>(S *, const S *, const S *, size_t, int, KrylovState *, KrylovHistory,              \
                                 const RedScratch &, hipStream_t);
EB_STAB_INST(double2)
EB_STAB_INST(float2)
EB_STAB_INST(bf16c)

}  // namespace ebicg
