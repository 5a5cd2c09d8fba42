// Wilson hopping term at one lattice site (device code shared by the
// single- and multi-RHS kernels).
#pragma once

#include "device_common.h"
#include "kernels.h"

namespace ebicg {

// ----------------------------------------------------------------------------
// Wilson hopping term.  Gamma basis (chiral): gamma_k = [[0,-i s_k],[i s_k,0]],
// gamma_t = [[0,1],[1,0]].  For the projector (1 + sg gamma_mu) the spinor
// collapses to two spin components h0, h1 (the upper half of the result);
// the lower half is a fixed multiple of (h0, h1):
//   mu=x: h0 = p0 - sg i p3, h1 = p1 - sg i p2;  lower = (sg i h1,  sg i h0)
//   mu=y: h0 = p0 - sg p3,   h1 = p1 + sg p2;    lower = (sg h1,   -sg h0)
//   mu=z: h0 = p0 - sg i p2, h1 = p1 + sg i p3;  lower = (sg i h0, -sg i h1)
//   mu=t: h0 = p0 + sg p2,   h1 = p1 + sg p3;    lower = (sg h0,    sg h1)
// The colour matrix acts on the two-component half spinor only (half the
// flops), and one output colour row is finished at a time so that only one
// row of the link is live.
// ----------------------------------------------------------------------------
template <int SG, typename R>
__device__ __forceinline__ cx<R> sgn(cx<R> a) {
  return SG > 0 ? a : -a;
}

// Spinor element (component c, site s) sits at (c V + s) KC: KC right-hand
// sides are interleaved (in points at the first entry of this thread's one).
template <int MU, int SG, typename S, int KC = 1>
__device__ __forceinline__ void load_project(cx<typename Store<S>::R> (&h)[6], const S *__restrict__ in, int V,
                                             int sn) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const auto p0 = Store<S>::ld(in, (size_t(a) * V + sn) * KC);
    const auto p1 = Store<S>::ld(in, (size_t(3 + a) * V + sn) * KC);
    const auto p2 = Store<S>::ld(in, (size_t(6 + a) * V + sn) * KC);
    const auto p3 = Store<S>::ld(in, (size_t(9 + a) * V + sn) * KC);
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

// acc += (spin reconstruction of) U h  (ADJ: U^+ h), U = U_mu at site sl.
template <int MU, int SG, bool ADJ, typename S>
__device__ __forceinline__ void mult_accum(cx<typename Store<S>::R> (&acc)[12], const cx<typename Store<S>::R> (&h)[6],
                                           const S *__restrict__ U, int V, int sl) {
  using R = typename Store<S>::R;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cx<R> t0, t1;
    if constexpr (!ADJ) {  // row a of U
      const cx<R> u0 = Store<S>::ld(U, size_t(MU * 9 + a * 3 + 0) * V + sl);
      const cx<R> u1 = Store<S>::ld(U, size_t(MU * 9 + a * 3 + 1) * V + sl);
      const cx<R> u2 = Store<S>::ld(U, size_t(MU * 9 + a * 3 + 2) * V + sl);
      t0 = u0 * h[0];
      cfma(t0, u1, h[1]);
      cfma(t0, u2, h[2]);
      t1 = u0 * h[3];
      cfma(t1, u1, h[4]);
      cfma(t1, u2, h[5]);
    } else {  // column a of U, conjugated
      const cx<R> u0 = Store<S>::ld(U, size_t(MU * 9 + 0 + a) * V + sl);
      const cx<R> u1 = Store<S>::ld(U, size_t(MU * 9 + 3 + a) * V + sl);
      const cx<R> u2 = Store<S>::ld(U, size_t(MU * 9 + 6 + a) * V + sl);
      t0 = cmulc(u0, h[0]);
      cfmac(t0, u1, h[1]);
      cfmac(t0, u2, h[2]);
      t1 = cmulc(u0, h[3]);
      cfmac(t1, u1, h[4]);
      cfmac(t1, u2, h[5]);
    }
    acc[a] = acc[a] + t0;
    acc[3 + a] = acc[3 + a] + t1;
    if constexpr (MU == 0) {
      acc[6 + a] = acc[6 + a] + sgn<SG>(ci(t1));
      acc[9 + a] = acc[9 + a] + sgn<SG>(ci(t0));
    } else if constexpr (MU == 1) {
      acc[6 + a] = acc[6 + a] + sgn<SG>(t1);
      acc[9 + a] = acc[9 + a] - sgn<SG>(t0);
    } else if constexpr (MU == 2) {
      acc[6 + a] = acc[6 + a] + sgn<SG>(ci(t0));
      acc[9 + a] = acc[9 + a] - sgn<SG>(ci(t1));
    } else {
      acc[6 + a] = acc[6 + a] + sgn<SG>(t0);
      acc[9 + a] = acc[9 + a] + sgn<SG>(t1);
    }
  }
}

// Keeps the compiler from hoisting the next hop's loads above this point, so
// the live state stays at one hop (half spinor + link row + accumulator) and
// the kernel runs several waves per SIMD instead of spilling.
__device__ __forceinline__ void hop_fence() { asm volatile("" ::: "memory"); }

// One direction mu: forward hop with projector (1 + SF gamma_mu) and U_mu(x),
// backward hop with (1 - SF gamma_mu) and U_mu(x - mu)^+.  FENCE = false
// lets the compiler overlap the loads of several hops (more registers).
template <int MU, int SF, typename S, int KC = 1, bool FENCE = true>
__device__ __forceinline__ void hop_dir(cx<typename Store<S>::R> (&acc)[12], const S *__restrict__ in,
                                        const S *__restrict__ U, int V, int s, int sf, int sb) {
  using R = typename Store<S>::R;
  cx<R> h[6];
  load_project<MU, SF, S, KC>(h, in, V, sf);
  mult_accum<MU, SF, false, S>(acc, h, U, V, s);
  if constexpr (FENCE) hop_fence();
  load_project<MU, -SF, S, KC>(h, in, V, sb);
  mult_accum<MU, -SF, true, S>(acc, h, U, V, sb);
  if constexpr (FENCE) hop_fence();
}

// Hopping sum at site s: sum_mu [ (1 + SF g) U psi(x+mu) + (1 - SF g) U^+ psi(x-mu) ].
// D uses SF = -1, D^+ uses SF = +1.
template <int SF, typename S, int KC = 1, bool FENCE = true>
__device__ __forceinline__ void hopping(cx<typename Store<S>::R> (&acc)[12], const S *__restrict__ in,
                                        const S *__restrict__ U, const Geom &g, int s) {
#pragma unroll
  for (int c = 0; c < 12; ++c) acc[c] = {0, 0};
  const int sy = g.lx, sz = g.lx * g.ly, stt = sz * g.lz;
  const int x = s % g.lx;
  const int y = (s / sy) % g.ly;
  const int z = (s / sz) % g.lz;
  const int t = s / stt;
  hop_dir<0, SF, S, KC, FENCE>(acc, in, U, g.V, s, x == g.lx - 1 ? s - (g.lx - 1) : s + 1, x == 0 ? s + (g.lx - 1) : s - 1);
  hop_dir<1, SF, S, KC, FENCE>(acc, in, U, g.V, s, y == g.ly - 1 ? s - (g.ly - 1) * sy : s + sy,
                    y == 0 ? s + (g.ly - 1) * sy : s - sy);
  hop_dir<2, SF, S, KC, FENCE>(acc, in, U, g.V, s, z == g.lz - 1 ? s - (g.lz - 1) * sz : s + sz,
                    z == 0 ? s + (g.lz - 1) * sz : s - sz);
  hop_dir<3, SF, S, KC, FENCE>(acc, in, U, g.V, s, t == g.lt - 1 ? s - (g.lt - 1) * stt : s + stt,
                    t == 0 ? s + (g.lt - 1) * stt : s - stt);
}

// ---------------------------------------------------------------------------
// LDS-staged form.  A block stages its tile of 256 consecutive sites of the
// input field into LDS (component-major [12][256]) in one coalesced sweep and
// takes every neighbour inside the tile from LDS; neighbours outside the tile
// come from global memory, where the neighbouring blocks' own staging sweeps
// have just brought them into L2.  Without staging, every hop of every
// resident wave sweeps the whole per-XCD share of the field, which does not
// fit in L2, and each neighbour read misses.
// ---------------------------------------------------------------------------
// With KC interleaved right-hand sides (batch layout), a tile is kBlock / KC
// sites times KC columns; glob and lds point at this thread's column.
template <typename S, int KC = 1>
struct TileSrc {
  static constexpr bool kFence = false;
  const S *__restrict__ glob;
  const S *lds;
  int s0, V;
  __device__ __forceinline__ cx<typename Store<S>::R> ld(int c, int sn) const {
    const unsigned d = unsigned(sn - s0);
    return d < unsigned(kBlock / KC) ? Store<S>::ld(lds, size_t(c) * kBlock + d * KC)
                                     : Store<S>::ld(glob, (size_t(c) * V + sn) * KC);
  }
};

// The same interface without a tile: every neighbour from global memory.  Its
// users fence between hops (kFence), as the unstaged stencil does.
template <typename S, int KC = 1>
struct GlobSrc {
  static constexpr bool kFence = true;
  const S *__restrict__ glob;
  int V;
  __device__ __forceinline__ cx<typename Store<S>::R> ld(int c, int sn) const {
    return Store<S>::ld(glob, (size_t(c) * V + sn) * KC);
  }
};

// Stage sites [s0, s0 + kBlock / KC) of `in` (all KC columns; sites < V); the
// caller synchronises.  Entry (c, site, col) goes to lds[c kBlock + (site - s0) KC + col].
template <typename S, int KC = 1>
__device__ __forceinline__ void stage_tile(S *lds, const S *__restrict__ in, int s0, int V) {
  const int s = s0 + int(threadIdx.x) / KC;
  if (s < V) {
#pragma unroll
    for (int c = 0; c < 12; ++c)
      lds[c * kBlock + threadIdx.x] = in[(size_t(c) * V + s0) * KC + threadIdx.x];
  }
}

template <int MU, int SG, typename S, typename Src>
__device__ __forceinline__ void load_project_t(cx<typename Store<S>::R> (&h)[6], const Src &src, int sn) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const auto p0 = src.ld(a, sn);
    const auto p1 = src.ld(3 + a, sn);
    const auto p2 = src.ld(6 + a, sn);
    const auto p3 = src.ld(9 + a, sn);
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

// No fence between the hops here: with neighbours in LDS the live state is
// smaller, and the kernels that use this form choose their register budget
// (and so how far the scheduler may overlap the hops' loads) themselves.
template <int MU, int SF, typename S, int KC>
__device__ __forceinline__ void hop_dir_t(cx<typename Store<S>::R> (&acc)[12], const TileSrc<S, KC> &src,
                                          const S *__restrict__ U, int V, int s, int sf, int sb) {
  using R = typename Store<S>::R;
  cx<R> h[6];
  load_project_t<MU, SF, S>(h, src, sf);
  mult_accum<MU, SF, false, S>(acc, h, U, V, s);
  load_project_t<MU, -SF, S>(h, src, sb);
  mult_accum<MU, -SF, true, S>(acc, h, U, V, sb);
}

template <int SF, typename S, int KC>
__device__ __forceinline__ void hopping_t(cx<typename Store<S>::R> (&acc)[12], const TileSrc<S, KC> &src,
                                          const S *__restrict__ U, const Geom &g, int s) {
#pragma unroll
  for (int c = 0; c < 12; ++c) acc[c] = {0, 0};
  const int sy = g.lx, sz = g.lx * g.ly, stt = sz * g.lz;
  const int x = s % g.lx;
  const int y = (s / sy) % g.ly;
  const int z = (s / sz) % g.lz;
  const int t = s / stt;
  // z and t first: their neighbours lie outside the tile, and right after the
  // staging sweeps the neighbouring tiles are most likely still in L2
  hop_dir_t<2, SF, S, KC>(acc, src, U, g.V, s, z == g.lz - 1 ? s - (g.lz - 1) * sz : s + sz,
                      z == 0 ? s + (g.lz - 1) * sz : s - sz);
  hop_dir_t<3, SF, S, KC>(acc, src, U, g.V, s, t == g.lt - 1 ? s - (g.lt - 1) * stt : s + stt,
                      t == 0 ? s + (g.lt - 1) * stt : s - stt);
  hop_dir_t<0, SF, S, KC>(acc, src, U, g.V, s, x == g.lx - 1 ? s - (g.lx - 1) : s + 1, x == 0 ? s + (g.lx - 1) : s - 1);
  hop_dir_t<1, SF, S, KC>(acc, src, U, g.V, s, y == g.ly - 1 ? s - (g.ly - 1) * sy : s + sy,
                      y == 0 ? s + (g.ly - 1) * sy : s - sy);
}

// ---------------------------------------------------------------------------
// Pieces of the t-marching form (batched stencils).  A thread that walks its
// site through consecutive time slices holds the site's full spinor at the
// current and the next slice in registers; the t hops then project those
// registers instead of loading neighbours.
// ---------------------------------------------------------------------------
// all 12 components of this thread's column at site sn
template <typename S, int KC>
__device__ __forceinline__ void load_spinor(cx<typename Store<S>::R> (&p)[12], const S *__restrict__ in, int V,
                                            int sn) {
#pragma unroll
  for (int c = 0; c < 12; ++c) p[c] = Store<S>::ld(in, (size_t(c) * V + sn) * KC);
}
// the t projector (1 + SG gamma_t) of a spinor in registers (the MU = 3 case of load_project)
template <int SG, typename R>
__device__ __forceinline__ void project_t(cx<R> (&h)[6], const cx<R> (&p)[12]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    h[a] = p[a] + sgn<SG>(p[6 + a]);
    h[3 + a] = p[3 + a] + sgn<SG>(p[9 + a]);
  }
}
// u = U_t h (ADJ: U_t^+ h) at site sl, the half spinor not yet reconstructed
template <bool ADJ, typename S>
__device__ __forceinline__ void mult_t(cx<typename Store<S>::R> (&u)[6], const cx<typename Store<S>::R> (&h)[6],
                                       const S *__restrict__ U, int V, int sl) {
  using R = typename Store<S>::R;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cx<R> t0, t1;
    if constexpr (!ADJ) {
      const cx<R> u0 = Store<S>::ld(U, size_t(27 + a * 3 + 0) * V + sl);
      const cx<R> u1 = Store<S>::ld(U, size_t(27 + a * 3 + 1) * V + sl);
      const cx<R> u2 = Store<S>::ld(U, size_t(27 + a * 3 + 2) * V + sl);
      t0 = u0 * h[0];
      cfma(t0, u1, h[1]);
      cfma(t0, u2, h[2]);
      t1 = u0 * h[3];
      cfma(t1, u1, h[4]);
      cfma(t1, u2, h[5]);
    } else {
      const cx<R> u0 = Store<S>::ld(U, size_t(27 + 0 + a) * V + sl);
      const cx<R> u1 = Store<S>::ld(U, size_t(27 + 3 + a) * V + sl);
      const cx<R> u2 = Store<S>::ld(U, size_t(27 + 6 + a) * V + sl);
      t0 = cmulc(u0, h[0]);
      cfmac(t0, u1, h[1]);
      cfmac(t0, u2, h[2]);
      t1 = cmulc(u0, h[3]);
      cfmac(t1, u1, h[4]);
      cfmac(t1, u2, h[5]);
    }
    u[a] = t0;
    u[3 + a] = t1;
  }
}
// acc += the spin reconstruction of a t half spinor with projector sign SG
template <int SG, typename R>
__device__ __forceinline__ void recon_t(cx<R> (&acc)[12], const cx<R> (&u)[6]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    acc[a] = acc[a] + u[a];
    acc[3 + a] = acc[3 + a] + u[3 + a];
    acc[6 + a] = acc[6 + a] + sgn<SG>(u[a]);
    acc[9 + a] = acc[9 + a] + sgn<SG>(u[3 + a]);
  }
}

}  // namespace ebicg
