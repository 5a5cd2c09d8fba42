// HIP kernels for gfx950: layouts, the Wilson-Dirac stencil, the fused BiCG
// and BiCGStab passes with device-resident scalars, the window rotation of
// Alg. BiCG-eigen and the tall-skinny deflation projections.
//
// Internal layout (HBM): a spinor is SoA [12][V] complex (component c =
// spin*3 + colour), so every load instruction of a wavefront reads 64
// consecutive complex numbers; links are SoA [4][9][V] complex with the
// t-boundary factor folded into U_t at t = Lt-1.  Reductions accumulate in
// FP64 whatever the storage precision, and finish deterministically in the
// last block (no host round trip per iteration).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_common.h"
#include "kernels.h"

namespace ebicg {

namespace {

inline int nblocks_for(size_t n, int per_thread = 1) {
  size_t t = (n + per_thread - 1) / per_thread;
  return int((t + kBlock - 1) / kBlock);
}

__device__ __forceinline__ bool skip_iter(const KrylovState *S, int j) {
  return S->stopped && j > S->stop_at;
}

// ----------------------------------------------------------------------------
// Wilson hopping term.  Gamma basis (chiral): gamma_k = [[0,-i s_k],[i s_k,0]],
// gamma_t = [[0,1],[1,0]].  For the projector (1 + sg gamma_mu) the spinor
// collapses to two spin components h0, h1 (the upper half of the result);
// the lower half is a fixed multiple of (h0, h1):
//   mu=x: h0 = p0 - sg i p3, h1 = p1 - sg i p2;  lower = (sg i h1,  sg i h0)
//   mu=y: h0 = p0 - sg p3,   h1 = p1 + sg p2;    lower = (sg h1,   -sg h0)
//   mu=z: h0 = p0 - sg i p2, h1 = p1 + sg i p3;  lower = (sg i h0, -sg i h1)
//   mu=t: h0 = p0 + sg p2,   h1 = p1 + sg p3;    lower = (sg h0,    sg h1)
// ----------------------------------------------------------------------------
template <int SG, typename R>
__device__ __forceinline__ cx<R> sgn(cx<R> a) {
  return SG > 0 ? a : -a;
}

template <int MU, int SG, typename R>
__device__ __forceinline__ void project(const cx<R> (&p)[12], cx<R> (&h)[6]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const cx<R> p0 = p[a], p1 = p[3 + a], p2 = p[6 + a], p3 = p[9 + a];
    if constexpr (MU == 0) {
      h[a] = p0 - sgn<SG>(ci(p3));
      h[3 + a] = p1 - sgn<SG>(ci(p2));
    } else if constexpr (MU == 1) {
      h[a] = p0 - sgn<SG>(p3);
      h[3 + a] = p1 + sgn<SG>(p2);
    } else if constexpr (MU == 2) {
      h[a] = p0 - sgn<SG>(ci(p2));
      h[3 + a] = p1 + sgn<SG>(ci(p3));
    } else {
      h[a] = p0 + sgn<SG>(p2);
      h[3 + a] = p1 + sgn<SG>(p3);
    }
  }
}

template <int MU, int SG, typename R>
__device__ __forceinline__ void accum(cx<R> (&acc)[12], const cx<R> (&u)[6]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const cx<R> u0 = u[a], u1 = u[3 + a];
    acc[a] = acc[a] + u0;
    acc[3 + a] = acc[3 + a] + u1;
    if constexpr (MU == 0) {
      acc[6 + a] = acc[6 + a] + sgn<SG>(ci(u1));
      acc[9 + a] = acc[9 + a] + sgn<SG>(ci(u0));
    } else if constexpr (MU == 1) {
      acc[6 + a] = acc[6 + a] + sgn<SG>(u1);
      acc[9 + a] = acc[9 + a] - sgn<SG>(u0);
    } else if constexpr (MU == 2) {
      acc[6 + a] = acc[6 + a] + sgn<SG>(ci(u0));
      acc[9 + a] = acc[9 + a] - sgn<SG>(ci(u1));
    } else {
      acc[6 + a] = acc[6 + a] + sgn<SG>(u0);
      acc[9 + a] = acc[9 + a] + sgn<SG>(u1);
    }
  }
}

template <typename S>
__device__ __forceinline__ void load_spinor(cx<typename Store<S>::R> (&p)[12], const S *__restrict__ in, int V, int s) {
#pragma unroll
  for (int c = 0; c < 12; ++c) p[c] = Store<S>::ld(in, size_t(c) * V + s);
}

// One direction mu: forward hop with projector (1 + SF gamma_mu) and U_mu(x),
// backward hop with (1 - SF gamma_mu) and U_mu(x - mu)^+.
template <int MU, int SF, typename S>
__device__ __forceinline__ void hop_dir(cx<typename Store<S>::R> (&acc)[12], const S *__restrict__ in,
                                        const S *__restrict__ U, int V, int s, int sf, int sb) {
  using R = typename Store<S>::R;
  cx<R> p[12], h[6], uh[6], u[9];
  // forward
  load_spinor<S>(p, in, V, sf);
#pragma unroll
  for (int e = 0; e < 9; ++e) u[e] = Store<S>::ld(U, size_t(MU * 9 + e) * V + s);
  project<MU, SF>(p, h);
#pragma unroll
  for (int k = 0; k < 2; ++k)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cx<R> t = u[a * 3] * h[k * 3];
      cfma(t, u[a * 3 + 1], h[k * 3 + 1]);
      cfma(t, u[a * 3 + 2], h[k * 3 + 2]);
      uh[k * 3 + a] = t;
    }
  accum<MU, SF>(acc, uh);
  // backward
  load_spinor<S>(p, in, V, sb);
#pragma unroll
  for (int e = 0; e < 9; ++e) u[e] = Store<S>::ld(U, size_t(MU * 9 + e) * V + sb);
  project<MU, -SF>(p, h);
#pragma unroll
  for (int k = 0; k < 2; ++k)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cx<R> t = cmulc(u[a], h[k * 3]);
      cfmac(t, u[3 + a], h[k * 3 + 1]);
      cfmac(t, u[6 + a], h[k * 3 + 2]);
      uh[k * 3 + a] = t;
    }
  accum<MU, -SF>(acc, uh);
}

// Hopping sum at site s: sum_mu [ (1 + SF g) U psi(x+mu) + (1 - SF g) U^+ psi(x-mu) ].
// D uses SF = -1, D^+ uses SF = +1.
template <int SF, typename S>
__device__ __forceinline__ void hopping(cx<typename Store<S>::R> (&acc)[12], const S *__restrict__ in,
                                        const S *__restrict__ U, const Geom &g, int s) {
#pragma unroll
  for (int c = 0; c < 12; ++c) acc[c] = {0, 0};
  const int x = s % g.lx;
  const int y = (s / g.lx) % g.ly;
  const int z = (s / (g.lx * g.ly)) % g.lz;
  const int t = s / (g.lx * g.ly * g.lz);
  const int sy = g.lx, sz = g.lx * g.ly, stt = g.lx * g.ly * g.lz;
  hop_dir<0, SF, S>(acc, in, U, g.V, s, x == g.lx - 1 ? s - (g.lx - 1) : s + 1, x == 0 ? s + (g.lx - 1) : s - 1);
  hop_dir<1, SF, S>(acc, in, U, g.V, s, y == g.ly - 1 ? s - (g.ly - 1) * sy : s + sy,
                    y == 0 ? s + (g.ly - 1) * sy : s - sy);
  hop_dir<2, SF, S>(acc, in, U, g.V, s, z == g.lz - 1 ? s - (g.lz - 1) * sz : s + sz,
                    z == 0 ? s + (g.lz - 1) * sz : s - sz);
  hop_dir<3, SF, S>(acc, in, U, g.V, s, t == g.lt - 1 ? s - (g.lt - 1) * stt : s + stt,
                    t == 0 ? s + (g.lt - 1) * stt : s - stt);
}

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
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int s = lb * kBlock + threadIdx.x;
  if (s >= g.V) return;
  cx<R> acc[12];
  hopping<SF, S>(acc, in, U, g, s);
  const R k = R(kappa);
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    cx<R> v = Store<S>::ld(in, size_t(c) * g.V + s);
    Store<S>::st(out, size_t(c) * g.V + s, v - k * acc[c]);
  }
}

// r = b - D x with ||r||^2 and ||b||^2 (FP64)
__global__ void __launch_bounds__(kBlock)
    k_residual(double2 *__restrict__ r, const double2 *__restrict__ b, const double2 *__restrict__ xin,
               const double2 *__restrict__ U, Geom g, double kappa, double *res, RedScratch rs) {
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int s = lb * kBlock + threadIdx.x;
  double v[2] = {0.0, 0.0};
  if (s < g.V) {
    cx<double> acc[12];
    hopping<-1, double2>(acc, xin, U, g, s);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const size_t i = size_t(c) * g.V + s;
      cx<double> xv = Store<double2>::ld(xin, i), bv = Store<double2>::ld(b, i);
      cx<double> rv = bv - (xv - kappa * acc[c]);
      Store<double2>::st(r, i, rv);
      v[0] += rv.x * rv.x + rv.y * rv.y;
      v[1] += bv.x * bv.x + bv.y * bv.y;
    }
  }
  if (grid_sum<2, kBlock>(v, rs.partials, rs.tickets, blockIdx.x, gridDim.x)) {
    res[0] = v[0];
    res[1] = v[1];
  }
}

// ----------------------------------------------------------------------------
// BiCG (Alg. eigBiCG loop), FP64
// ----------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock)
    k_bicg_init(double2 *__restrict__ rhat, double2 *__restrict__ p, double2 *__restrict__ ph,
                const double2 *__restrict__ r, const double *res, size_t N, int V, int rhat_mode, double tol,
                int maxiter, KrylovState *S, KrylovHistory h, RedScratch rs) {
  const size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x;
  double v[2] = {0.0, 0.0};
  if (i < N) {
    cx<double> rv = Store<double2>::ld(r, i);
    // gamma5 = diag(1, 1, -1, -1): components 6..11 of the SoA layout flip sign
    cx<double> hv = (rhat_mode == 1 && i >= size_t(6) * V) ? -rv : rv;
    Store<double2>::st(rhat, i, hv);
    Store<double2>::st(p, i, rv);
    Store<double2>::st(ph, i, hv);
    cx<double> d = cmulc(hv, rv);
    v[0] = d.x;
    v[1] = d.y;
  }
  if (grid_sum<2, kBlock>(v, rs.partials, rs.tickets, blockIdx.x, gridDim.x)) {
    const double rn = sqrt(res[0]), bn = sqrt(res[1]);
    S->rho = make_double2(v[0], v[1]);
    S->alpha = S->beta = S->omega = make_double2(0, 0);
    S->rnorm = rn;
    S->bnorm = bn;
    S->tol_abs = tol * bn;
    S->def_thr = 0;
    S->maxiter = maxiter;
    h.rho[0] = S->rho;
    h.rn[0] = rn;
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
}

// Blocks [0, nb) compute Ap = D p (and the sigma partial), blocks [nb, 2nb)
// compute Adp = D^+ phat.  Linear block b -> (site block b/2, half b%2) after
// the XCD remap, so both halves of one site block run on the same XCD and the
// links they share are read from HBM once.
__global__ void __launch_bounds__(kBlock)
    k_bicg_matvec(double2 *__restrict__ Ap, double2 *__restrict__ Adp, const double2 *__restrict__ p,
                  const double2 *__restrict__ ph, const double2 *__restrict__ U, Geom g, double kappa, int j,
                  KrylovState *S, KrylovHistory h, RedScratch rs) {
  if (skip_iter(S, j)) return;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int half = lb & 1;
  const int s = (lb >> 1) * kBlock + threadIdx.x;
  double v[2] = {0.0, 0.0};
  if (s < g.V) {
    cx<double> acc[12];
    if (half == 0) {
      hopping<-1, double2>(acc, p, U, g, s);
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        const size_t i = size_t(c) * g.V + s;
        cx<double> o = Store<double2>::ld(p, i) - kappa * acc[c];
        Store<double2>::st(Ap, i, o);
        cx<double> d = cmulc(Store<double2>::ld(ph, i), o);
        v[0] += d.x;
        v[1] += d.y;
      }
    } else {
      hopping<+1, double2>(acc, ph, U, g, s);
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        const size_t i = size_t(c) * g.V + s;
        Store<double2>::st(Adp, i, Store<double2>::ld(ph, i) - kappa * acc[c]);
      }
    }
  }
  if (grid_sum<2, kBlock>(v, rs.partials, rs.tickets, blockIdx.x, gridDim.x)) {
    const cx<double> sig{v[0], v[1]};
    const double2 rho = S->rho;
    const double den = sig.x * sig.x + sig.y * sig.y;
    if (!(den > 0.0) || !isfinite(den)) {
      S->stopped = 1;
      S->stop_at = j - 1;
      S->reason = 2;
    } else {
      // alpha = rho / sigma
      cx<double> a{(rho.x * sig.x + rho.y * sig.y) / den, (rho.y * sig.x - rho.x * sig.y) / den};
      S->alpha = make_double2(a.x, a.y);
      h.alpha[j - 1] = S->alpha;
    }
  }
}

__global__ void __launch_bounds__(kBlock)
    k_bicg_update_r(double2 *__restrict__ r_out, double2 *__restrict__ rh_out, const double2 *__restrict__ r_in,
                    const double2 *__restrict__ rh_in, const double2 *__restrict__ Ap,
                    const double2 *__restrict__ Adp, size_t N, int j, KrylovState *S, KrylovHistory h,
                    RedScratch rs) {
  if (skip_iter(S, j)) return;
  const double2 a2 = S->alpha;
  const cx<double> a{a2.x, a2.y}, ac{a2.x, -a2.y};
  double v[3] = {0.0, 0.0, 0.0};
  for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < N; i += size_t(gridDim.x) * kBlock) {
    cx<double> r = Store<double2>::ld(r_in, i) - a * Store<double2>::ld(Ap, i);
    cx<double> rh = Store<double2>::ld(rh_in, i) - ac * Store<double2>::ld(Adp, i);
    Store<double2>::st(r_out, i, r);
    Store<double2>::st(rh_out, i, rh);
    cx<double> d = cmulc(rh, r);
    v[0] += d.x;
    v[1] += d.y;
    v[2] += r.x * r.x + r.y * r.y;
  }
  if (grid_sum<3, kBlock>(v, rs.partials, rs.tickets, blockIdx.x, gridDim.x)) {
    const double2 rho0 = S->rho;
    const cx<double> rn{v[0], v[1]};
    const double den = rho0.x * rho0.x + rho0.y * rho0.y;
    cx<double> beta{(rn.x * rho0.x + rn.y * rho0.y) / den, (rn.y * rho0.x - rn.x * rho0.y) / den};
    const double rnorm = sqrt(v[2]);
    S->beta = make_double2(beta.x, beta.y);
    S->rho = make_double2(rn.x, rn.y);
    S->rnorm = rnorm;
    h.beta[j - 1] = S->beta;
    h.rho[j] = S->rho;
    h.rn[j] = rnorm;
    if (rnorm <= S->tol_abs) {
      S->stopped = 1;
      S->stop_at = j;
      S->reason = 1;
    } else if (rn.x == 0.0 && rn.y == 0.0) {
      S->stopped = 1;
      S->stop_at = j;
      S->reason = 2;
    } else if (j >= S->maxiter) {
      S->stopped = 1;
      S->stop_at = j;
      S->reason = 4;
    }
  }
}

__global__ void __launch_bounds__(kBlock)
    k_bicg_update_p(double2 *__restrict__ x, double2 *__restrict__ p, double2 *__restrict__ ph,
                    const double2 *__restrict__ r, const double2 *__restrict__ rh, size_t N, int j,
                    const KrylovState *S) {
  if (skip_iter(S, j)) return;
  const double2 a2 = S->alpha, b2 = S->beta;
  const cx<double> a{a2.x, a2.y}, b{b2.x, b2.y}, bc{b2.x, -b2.y};
  for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < N; i += size_t(gridDim.x) * kBlock) {
    cx<double> pv = Store<double2>::ld(p, i);
    Store<double2>::st(x, i, Store<double2>::ld(x, i) + a * pv);
    Store<double2>::st(p, i, Store<double2>::ld(r, i) + b * pv);
    Store<double2>::st(ph, i, Store<double2>::ld(rh, i) + bc * Store<double2>::ld(ph, i));
  }
}

__global__ void __launch_bounds__(kBlock)
    k_arrow_vectors(double2 *__restrict__ GA, double2 *__restrict__ GB, const double2 *__restrict__ Adp,
                    const double2 *__restrict__ s, const double2 *__restrict__ Ap, const double2 *__restrict__ q,
                    size_t N, int j, const KrylovState *S, KrylovHistory h) {
  if (skip_iter(S, j)) return;
  const double2 b2 = h.beta[j - 2];
  const cx<double> b{b2.x, b2.y}, bc{b2.x, -b2.y};
  for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < N; i += size_t(gridDim.x) * kBlock) {
    Store<double2>::st(GA, i, Store<double2>::ld(Adp, i) - bc * Store<double2>::ld(s, i));
    Store<double2>::st(GB, i, Store<double2>::ld(Ap, i) - b * Store<double2>::ld(q, i));
  }
}

// out[k] = sum_c in[c] C[c + k*nin], k in this block's output tile of NT.
template <int NT>
__global__ void __launch_bounds__(kBlock)
    k_rotate(double2 *__restrict__ out_base, SlotList out_slots, const double2 *__restrict__ in_base,
             SlotList in_slots, const double2 *__restrict__ C, size_t N, const double2 *__restrict__ g,
             int conj_out, double2 *dots, int jtag, const KrylovState *S, RedScratch rs) {
  if (S && skip_iter(S, jtag)) return;
  extern __shared__ double2 sC[];  // nin x NT tile of C
  const int nin = in_slots.n;
  const int k0 = blockIdx.y * NT;
  const int nk = min(NT, out_slots.n - k0);
  for (int e = threadIdx.x; e < nin * NT; e += kBlock) {
    const int c = e % nin, k = e / nin;
    sC[e] = (k < nk) ? C[c + size_t(k0 + k) * nin] : make_double2(0, 0);
  }
  __syncthreads();
  double dv[2 * NT];
#pragma unroll
  for (int k = 0; k < 2 * NT; ++k) dv[k] = 0.0;
  for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < N; i += size_t(gridDim.x) * kBlock) {
    cx<double> acc[NT];
#pragma unroll
    for (int k = 0; k < NT; ++k) acc[k] = {0, 0};
    for (int c = 0; c < nin; ++c) {
      const cx<double> v = Store<double2>::ld(in_base + size_t(in_slots.idx[c]) * N, i);
#pragma unroll
      for (int k = 0; k < NT; ++k) {
        const double2 cc = sC[c + k * nin];
        cfma(acc[k], v, cx<double>{cc.x, cc.y});
      }
    }
    cx<double> gv{0, 0};
    if (g) gv = Store<double2>::ld(g, i);
#pragma unroll
    for (int k = 0; k < NT; ++k) {
      if (k < nk) {
        Store<double2>::st(out_base + size_t(out_slots.idx[k0 + k]) * N, i, acc[k]);
        cx<double> d = conj_out ? cmulc(acc[k], gv) : cmulc(gv, acc[k]);
        dv[2 * k] += d.x;
        dv[2 * k + 1] += d.y;
      }
    }
  }
  if (!g) return;
  const int nblk = gridDim.x;
  if (grid_sum<2 * NT, kBlock>(dv, rs.partials + size_t(blockIdx.y) * nblk * 2 * NT, rs.tickets + blockIdx.y,
                               blockIdx.x, nblk)) {
    for (int k = 0; k < nk; ++k) dots[k0 + k] = make_double2(dv[2 * k], dv[2 * k + 1]);
  }
}

// out[a + b*nx] = sum_i conj(X_a[i]) Y_b[i] over a tile XT x YT.
template <int XT, int YT>
__global__ void __launch_bounds__(kBlock)
    k_ts_dot(double2 *out, const double2 *__restrict__ X, size_t ldx, int nx, const double2 *__restrict__ Y,
             size_t ldy, int ny, size_t N, RedScratch rs) {
  const int a0 = blockIdx.y * XT, b0 = blockIdx.z * YT;
  double v[2 * XT * YT];
#pragma unroll
  for (int e = 0; e < 2 * XT * YT; ++e) v[e] = 0.0;
  for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < N; i += size_t(gridDim.x) * kBlock) {
    cx<double> yv[YT];
#pragma unroll
    for (int b = 0; b < YT; ++b) yv[b] = (b0 + b < ny) ? Store<double2>::ld(Y + size_t(b0 + b) * ldy, i) : cx<double>{0, 0};
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
  const int nblk = gridDim.x;
  if (grid_sum<2 * XT * YT, kBlock>(v, rs.partials + size_t(tile) * nblk * 2 * XT * YT, rs.tickets + tile,
                                    blockIdx.x, nblk)) {
    for (int a = 0; a < XT; ++a)
      for (int b = 0; b < YT; ++b)
        if (a0 + a < nx && b0 + b < ny)
          out[(a0 + a) + size_t(b0 + b) * nx] = make_double2(v[2 * (a * YT + b)], v[2 * (a * YT + b) + 1]);
  }
}

// Y_b += sgn * sum_a X_a C[a + b*nx] for b in this block's tile of YT.
template <int YT>
__global__ void __launch_bounds__(kBlock)
    k_ts_update(double2 *__restrict__ Y, size_t ldy, int ny, const double2 *__restrict__ X, size_t ldx, int nx,
                const double2 *__restrict__ C, double sgn, size_t N) {
  extern __shared__ double2 sC[];  // nx x YT
  const int b0 = blockIdx.y * YT;
  for (int e = threadIdx.x; e < nx * YT; e += kBlock) {
    const int a = e % nx, b = e / nx;
    const double2 c = (b0 + b < ny) ? C[a + size_t(b0 + b) * nx] : make_double2(0, 0);
    sC[e] = make_double2(sgn * c.x, sgn * c.y);
  }
  __syncthreads();
  for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < N; i += size_t(gridDim.x) * kBlock) {
    cx<double> acc[YT];
#pragma unroll
    for (int b = 0; b < YT; ++b) acc[b] = {0, 0};
    for (int a = 0; a < nx; ++a) {
      const cx<double> xv = Store<double2>::ld(X + size_t(a) * ldx, i);
#pragma unroll
      for (int b = 0; b < YT; ++b) {
        const double2 c = sC[a + b * nx];
        cfma(acc[b], xv, cx<double>{c.x, c.y});
      }
    }
#pragma unroll
    for (int b = 0; b < YT; ++b)
      if (b0 + b < ny) {
        double2 *yb = Y + size_t(b0 + b) * ldy;
        Store<double2>::st(yb, i, Store<double2>::ld(yb, i) + acc[b]);
      }
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
// BiCGStab (van der Vorst), storage S, FP64 reductions and scalars
// ----------------------------------------------------------------------------
template <typename S>
__global__ void __launch_bounds__(kBlock)
    k_stab_init(S *__restrict__ rhat, S *__restrict__ p, const S *__restrict__ r, size_t N, double tol_abs,
                double def_thr, int maxiter, KrylovState *K, RedScratch rs) {
  double v[1] = {0.0};
  for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < N; i += size_t(gridDim.x) * kBlock) {
    auto rv = Store<S>::ld(r, i);
    Store<S>::st(rhat, i, rv);
    Store<S>::st(p, i, rv);
    v[0] += double(rv.x) * rv.x + double(rv.y) * rv.y;
  }
  if (grid_sum<1, kBlock>(v, rs.partials, rs.tickets, blockIdx.x, gridDim.x)) {
    K->rho = make_double2(v[0], 0.0);
    K->alpha = make_double2(1, 0);
    K->omega = make_double2(1, 0);
    K->beta = make_double2(0, 0);
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
}

// v = D p ; alpha = rho / (rhat, v)
template <typename S>
__global__ void __launch_bounds__(kBlock)
    k_stab_v(S *__restrict__ vout, const S *__restrict__ p, const S *__restrict__ rhat, const S *__restrict__ U,
             Geom g, double kappa, int j, KrylovState *K, RedScratch rs) {
  using R = typename Store<S>::R;
  if (skip_iter(K, j)) return;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int s = lb * kBlock + threadIdx.x;
  double v[2] = {0.0, 0.0};
  if (s < g.V) {
    cx<R> acc[12];
    hopping<-1, S>(acc, p, U, g, s);
    const R k = R(kappa);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const size_t i = size_t(c) * g.V + s;
      cx<R> o = Store<S>::ld(p, i) - k * acc[c];
      Store<S>::st(vout, i, o);
      o = Store<S>::ld(vout, i);  // the stored (rounded) v enters the dot, as in later passes
      cx<R> h = Store<S>::ld(rhat, i);
      v[0] += double(h.x) * o.x + double(h.y) * o.y;
      v[1] += double(h.x) * o.y - double(h.y) * o.x;
    }
  }
  if (grid_sum<2, kBlock>(v, rs.partials, rs.tickets, blockIdx.x, gridDim.x)) {
    const double den = v[0] * v[0] + v[1] * v[1];
    if (!(den > 0.0) || !isfinite(den)) {
      K->stopped = 1;
      K->stop_at = j - 1;
      K->reason = 2;
    } else {
      const double2 rho = K->rho;
      K->alpha = make_double2((rho.x * v[0] + rho.y * v[1]) / den, (rho.y * v[0] - rho.x * v[1]) / den);
    }
  }
}

template <typename S>
__global__ void __launch_bounds__(kBlock)
    k_stab_s(S *__restrict__ sv, const S *__restrict__ r, const S *__restrict__ v, size_t N, int j,
             const KrylovState *K) {
  using R = typename Store<S>::R;
  if (skip_iter(K, j)) return;
  const double2 a2 = K->alpha;
  const cx<R> a{R(a2.x), R(a2.y)};
  for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < N; i += size_t(gridDim.x) * kBlock)
    Store<S>::st(sv, i, Store<S>::ld(r, i) - a * Store<S>::ld(v, i));
}

// t = D s ; omega = (t, s) / (t, t)
template <typename S>
__global__ void __launch_bounds__(kBlock)
    k_stab_t(S *__restrict__ tout, const S *__restrict__ sv, const S *__restrict__ U, Geom g, double kappa, int j,
             KrylovState *K, RedScratch rs) {
  using R = typename Store<S>::R;
  if (skip_iter(K, j)) return;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int s = lb * kBlock + threadIdx.x;
  double v[3] = {0.0, 0.0, 0.0};
  if (s < g.V) {
    cx<R> acc[12];
    hopping<-1, S>(acc, sv, U, g, s);
    const R k = R(kappa);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const size_t i = size_t(c) * g.V + s;
      cx<R> si = Store<S>::ld(sv, i);
      cx<R> o = si - k * acc[c];
      Store<S>::st(tout, i, o);
      o = Store<S>::ld(tout, i);
      v[0] += double(o.x) * si.x + double(o.y) * si.y;
      v[1] += double(o.x) * si.y - double(o.y) * si.x;
      v[2] += double(o.x) * o.x + double(o.y) * o.y;
    }
  }
  if (grid_sum<3, kBlock>(v, rs.partials, rs.tickets, blockIdx.x, gridDim.x)) {
    if (!(v[2] > 0.0)) {
      K->omega = make_double2(0, 0);
      K->stopped = 1;
      K->stop_at = j - 1;
      K->reason = 2;
    } else {
      K->omega = make_double2(v[0] / v[2], v[1] / v[2]);
    }
  }
}

// x += alpha p + omega s ; r = s - omega t ; rho' = (rhat, r), ||r||
template <typename S>
__global__ void __launch_bounds__(kBlock)
    k_stab_xr(S *__restrict__ x, S *__restrict__ r, const S *__restrict__ p, const S *__restrict__ sv,
              const S *__restrict__ t, const S *__restrict__ rhat, size_t N, int j, KrylovState *K, RedScratch rs) {
  using R = typename Store<S>::R;
  if (skip_iter(K, j)) return;
  const double2 a2 = K->alpha, w2 = K->omega;
  const cx<R> a{R(a2.x), R(a2.y)}, w{R(w2.x), R(w2.y)};
  double v[3] = {0.0, 0.0, 0.0};
  for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < N; i += size_t(gridDim.x) * kBlock) {
    const cx<R> si = Store<S>::ld(sv, i);
    Store<S>::st(x, i, Store<S>::ld(x, i) + a * Store<S>::ld(p, i) + w * si);
    Store<S>::st(r, i, si - w * Store<S>::ld(t, i));
    const cx<R> ri = Store<S>::ld(r, i), h = Store<S>::ld(rhat, i);
    v[0] += double(h.x) * ri.x + double(h.y) * ri.y;
    v[1] += double(h.x) * ri.y - double(h.y) * ri.x;
    v[2] += double(ri.x) * ri.x + double(ri.y) * ri.y;
  }
  if (grid_sum<3, kBlock>(v, rs.partials, rs.tickets, blockIdx.x, gridDim.x)) {
    const double2 rho0 = K->rho, al = K->alpha, om = K->omega;
    const cx<double> rn{v[0], v[1]};
    // beta = (rho'/rho) (alpha/omega)
    const double d0 = rho0.x * rho0.x + rho0.y * rho0.y;
    const cx<double> q{(rn.x * rho0.x + rn.y * rho0.y) / d0, (rn.y * rho0.x - rn.x * rho0.y) / d0};
    const double d1 = om.x * om.x + om.y * om.y;
    const cx<double> ao{(al.x * om.x + al.y * om.y) / d1, (al.y * om.x - al.x * om.y) / d1};
    const cx<double> beta = q * ao;
    K->beta = make_double2(beta.x, beta.y);
    K->rho = make_double2(rn.x, rn.y);
    const double rnorm = sqrt(v[2]);
    K->rnorm = rnorm;
    if (rnorm <= K->tol_abs) {
      K->stopped = 1;
      K->stop_at = j;
      K->reason = 1;
    } else if (K->def_thr > 0.0 && rnorm < K->def_thr) {
      K->stopped = 1;
      K->stop_at = j;
      K->reason = 3;
    } else if (rn.x == 0.0 && rn.y == 0.0) {
      K->stopped = 1;
      K->stop_at = j;
      K->reason = 2;
    } else if (j >= K->maxiter) {
      K->stopped = 1;
      K->stop_at = j;
      K->reason = 4;
    }
  }
}

// p = r + beta (p - omega v)
template <typename S>
__global__ void __launch_bounds__(kBlock)
    k_stab_p(S *__restrict__ p, const S *__restrict__ r, const S *__restrict__ v, size_t N, int j,
             const KrylovState *K) {
  using R = typename Store<S>::R;
  if (skip_iter(K, j)) return;
  const double2 b2 = K->beta, w2 = K->omega;
  const cx<R> b{R(b2.x), R(b2.y)}, w{R(w2.x), R(w2.y)};
  for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < N; i += size_t(gridDim.x) * kBlock)
    Store<S>::st(p, i, Store<S>::ld(r, i) + b * (Store<S>::ld(p, i) - w * Store<S>::ld(v, i)));
}

// grid size of the streaming (grid-stride) kernels: a function of n only, so
// reductions are reproducible run to run
inline int stream_grid(size_t n) {
  int nb = nblocks_for(n, 4);
  return nb < 1 ? 1 : (nb > 8192 ? 8192 : nb);
}

}  // namespace

// ============================================================================
// launch wrappers
// ============================================================================
#define EB_LAUNCH(kernel, grid, block, shmem, st, ...) hipLaunchKernelGGL(kernel, grid, block, shmem, st, __VA_ARGS__)

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
void launch_to_soa_bf16(bf16c *d, const bf16c *s, const Geom &g, hipStream_t st) {
  EB_LAUNCH(k_to_soa<bf16c>, dim3(nblocks_for(size_t(g.V) * 12)), dim3(kBlock), 0, st, d, s, g.V);
}
void launch_from_soa_bf16(bf16c *d, const bf16c *s, const Geom &g, hipStream_t st) {
  EB_LAUNCH(k_from_soa<bf16c>, dim3(nblocks_for(size_t(g.V) * 12)), dim3(kBlock), 0, st, d, s, g.V);
}
void launch_pack_gauge_f64(double2 *d, const double2 *s, const Geom &g, int bc_t, hipStream_t st) {
  EB_LAUNCH(k_pack_gauge, dim3(nblocks_for(size_t(g.V) * 36)), dim3(kBlock), 0, st, d, s, g, bc_t);
}
void launch_convert_f64_f32(float2 *d, const double2 *s, size_t n, hipStream_t st) {
  EB_LAUNCH((k_convert<float2, double2>), dim3(nblocks_for(n)), dim3(kBlock), 0, st, d, s, n);
}
void launch_convert_f64_bf16(bf16c *d, const double2 *s, size_t n, hipStream_t st) {
  EB_LAUNCH((k_convert<bf16c, double2>), dim3(nblocks_for(n)), dim3(kBlock), 0, st, d, s, n);
}
void launch_convert_f32_f64(double2 *d, const float2 *s, size_t n, hipStream_t st) {
  EB_LAUNCH((k_convert<double2, float2>), dim3(nblocks_for(n)), dim3(kBlock), 0, st, d, s, n);
}
void launch_convert_bf16_f64(double2 *d, const bf16c *s, size_t n, hipStream_t st) {
  EB_LAUNCH((k_convert<double2, bf16c>), dim3(nblocks_for(n)), dim3(kBlock), 0, st, d, s, n);
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

void launch_residual_f64(double2 *r, const double2 *b, const double2 *x, const double2 *U, const Geom &g, double kappa,
                         double *res, const RedScratch &rs, hipStream_t st) {
  EB_LAUNCH(k_residual, dim3(nblocks_for(g.V)), dim3(kBlock), 0, st, r, b, x, U, g, kappa, res, rs);
}

void launch_bicg_init(double2 *rhat, double2 *p, double2 *ph, const double2 *r, const double *res, size_t N,
                      int rhat_mode, const Geom &g, double tol, int maxiter, KrylovState *S, KrylovHistory h,
                      const RedScratch &rs, hipStream_t st) {
  EB_LAUNCH(k_bicg_init, dim3(nblocks_for(N)), dim3(kBlock), 0, st, rhat, p, ph, r, res, N, g.V, rhat_mode, tol,
            maxiter, S, h, rs);
}
void launch_bicg_matvec(double2 *Ap, double2 *Adp, const double2 *p, const double2 *ph, const double2 *U,
                        const Geom &g, double kappa, int j, KrylovState *S, KrylovHistory h, const RedScratch &rs,
                        hipStream_t st) {
  EB_LAUNCH(k_bicg_matvec, dim3(2 * nblocks_for(g.V)), dim3(kBlock), 0, st, Ap, Adp, p, ph, U, g, kappa, j, S, h, rs);
}
void launch_bicg_update_r(double2 *r_out, double2 *rh_out, const double2 *r_in, const double2 *rh_in,
                          const double2 *Ap, const double2 *Adp, size_t N, int j, KrylovState *S, KrylovHistory h,
                          const RedScratch &rs, hipStream_t st) {
  EB_LAUNCH(k_bicg_update_r, dim3(stream_grid(N)), dim3(kBlock), 0, st, r_out, rh_out, r_in, rh_in, Ap, Adp, N, j, S,
            h, rs);
}
void launch_bicg_update_p(double2 *x, double2 *p, double2 *ph, const double2 *r, const double2 *rh, size_t N, int j,
                          const KrylovState *S, hipStream_t st) {
  EB_LAUNCH(k_bicg_update_p, dim3(stream_grid(N)), dim3(kBlock), 0, st, x, p, ph, r, rh, N, j, S);
}
void launch_arrow_vectors(double2 *GA, double2 *GB, const double2 *Adp, const double2 *s, const double2 *Ap,
                          const double2 *q, size_t N, int j, const KrylovState *S, KrylovHistory h, hipStream_t st) {
  EB_LAUNCH(k_arrow_vectors, dim3(stream_grid(N)), dim3(kBlock), 0, st, GA, GB, Adp, s, Ap, q, N, j, S, h);
}

void launch_rotate(double2 *out_base, const SlotList &out_slots, const double2 *in_base, const SlotList &in_slots,
                   const double2 *C, size_t N, const double2 *g, int conj_out, double2 *dots, int jtag,
                   const KrylovState *S, const RedScratch &rs, hipStream_t st) {
  const int nout = out_slots.n;
  const int nb = stream_grid(N);
  auto go = [&](auto nt_tag) {
    constexpr int NT = decltype(nt_tag)::value;
    dim3 grid(nb, (nout + NT - 1) / NT);
    size_t sh = size_t(in_slots.n) * NT * sizeof(double2);
    EB_LAUNCH(k_rotate<NT>, grid, dim3(kBlock), sh, st, out_base, out_slots, in_base, in_slots, C, N, g, conj_out,
              dots, jtag, S, rs);
  };
  if (nout <= 4)
    go(std::integral_constant<int, 4>{});
  else if (nout <= 8)
    go(std::integral_constant<int, 8>{});
  else if (nout <= 16)
    go(std::integral_constant<int, 16>{});
  else
    go(std::integral_constant<int, 24>{});
}

void launch_ts_dot(double2 *out, const double2 *X, size_t ldx, int nx, const double2 *Y, size_t ldy, int ny, size_t N,
                   const RedScratch &rs, hipStream_t st) {
  constexpr int XT = 8, YT = 2;
  const int tx = (nx + XT - 1) / XT, ty = (ny + YT - 1) / YT;
  const int tiles = tx * ty;
  if (tiles > kMaxTickets) return;  // callers stay within kMaxCols x kMaxCols
  // every tile keeps nb partials of 2 XT YT doubles in the shared scratch
  int nb = stream_grid(N);
  const int cap = int(kMaxPartials / (size_t(tiles) * 2 * XT * YT));
  nb = nb < 1024 ? nb : 1024;
  nb = nb < cap ? nb : cap;
  dim3 grid(nb, tx, ty);
  EB_LAUNCH((k_ts_dot<XT, YT>), grid, dim3(kBlock), 0, st, out, X, ldx, nx, Y, ldy, ny, N, rs);
}
void launch_ts_update(double2 *Y, size_t ldy, int ny, const double2 *X, size_t ldx, int nx, const double2 *C,
                      double sgn, size_t N, hipStream_t st) {
  constexpr int YT = 4;
  dim3 grid(stream_grid(N), (ny + YT - 1) / YT);
  EB_LAUNCH(k_ts_update<YT>, grid, dim3(kBlock), size_t(nx) * YT * sizeof(double2), st, Y, ldy, ny, X, ldx, nx, C,
            sgn, N);
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
                      KrylovState *K, const RedScratch &rs, hipStream_t st) {
  EB_LAUNCH(k_stab_init<S>, dim3(stream_grid(N)), dim3(kBlock), 0, st, rhat, p, r, N, tol_abs, def_thr, maxiter, K,
            rs);
}
template <typename S>
void launch_stab_v(S *v, const S *p, const S *rhat, const S *U, const Geom &g, double kappa, int j, KrylovState *K,
                   const RedScratch &rs, hipStream_t st) {
  EB_LAUNCH(k_stab_v<S>, dim3(nblocks_for(g.V)), dim3(kBlock), 0, st, v, p, rhat, U, g, kappa, j, K, rs);
}
template <typename S>
void launch_stab_s(S *s, const S *r, const S *v, size_t N, int j, const KrylovState *K, hipStream_t st) {
  EB_LAUNCH(k_stab_s<S>, dim3(stream_grid(N)), dim3(kBlock), 0, st, s, r, v, N, j, K);
}
template <typename S>
void launch_stab_t(S *t, const S *s, const S *U, const Geom &g, double kappa, int j, KrylovState *K,
                   const RedScratch &rs, hipStream_t st) {
  EB_LAUNCH(k_stab_t<S>, dim3(nblocks_for(g.V)), dim3(kBlock), 0, st, t, s, U, g, kappa, j, K, rs);
}
template <typename S>
void launch_stab_xr(S *x, S *r, const S *p, const S *s, const S *t, const S *rhat, size_t N, int j, KrylovState *K,
                    const RedScratch &rs, hipStream_t st) {
  EB_LAUNCH(k_stab_xr<S>, dim3(stream_grid(N)), dim3(kBlock), 0, st, x, r, p, s, t, rhat, N, j, K, rs);
}
template <typename S>
void launch_stab_p(S *p, const S *r, const S *v, size_t N, int j, const KrylovState *K, hipStream_t st) {
  EB_LAUNCH(k_stab_p<S>, dim3(stream_grid(N)), dim3(kBlock), 0, st, p, r, v, N, j, K);
}

#define EB_STAB_INST(S)                                                                                              \
  template void launch_stab_init<S>(S *, S *, const S *, size_t, double, double, int, KrylovState *,               \
                                    const RedScratch &, hipStream_t);                                                \
  template void launch_stab_v<S>(S *, const S *, const S *, const S *, const Geom &, double, int, KrylovState *,    \
                                 const RedScratch &, hipStream_t);                                                   \
  template void launch_stab_s<S>(S *, const S *, const S *, size_t, int, const KrylovState *, hipStream_t);         \
  template void launch_stab_t<S>(S *, const S *, const S *, const Geom &, double, int, KrylovState *,               \
                                 const RedScratch &, hipStream_t);                                                   \
  template void launch_stab_xr<S>(S *, S *, const S *, const S *, const S *, const S *, size_t, int, KrylovState *, \
                                  const RedScratch &, hipStream_t);                                                  \
  template void launch_stab_p<S>(S *, const S *, const S *, size_t, int, const KrylovState *, hipStream_t);
EB_STAB_INST(double2)
EB_STAB_INST(float2)

}  // namespace ebicg
