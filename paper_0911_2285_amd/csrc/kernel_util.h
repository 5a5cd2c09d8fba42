// Launch geometry, reduction-scratch regions and small scalar helpers shared
// by the kernel files (kernels.hip, batch.hip, eo.hip).
#pragma once

#include <type_traits>

#include "device_common.h"
#include "kernels.h"

namespace ebicg {
namespace {

// Partial-sum regions of the reduction scratch, one per producer so that a
// record is never overwritten before its consumer has read it.
enum Region : int { RG_SIGMA = 0, RG_RR, RG_V, RG_T, RG_XR, RG_INIT, RG_RES, RG_GEN };
constexpr size_t kRegion = kRegionDoubles;
inline double *region(const RedScratch &rs, Region r) { return rs.partials + size_t(r) * kRegion; }

inline int nblocks_for(size_t n, int per_thread = 1) {
  size_t t = (n + per_thread - 1) / per_thread;
  return int((t + kBlock - 1) / kBlock);
}
// grid of the streaming kernels with reductions: a function of n only
inline int red_grid(size_t n) {
  int nb = nblocks_for(n, 4);
  return nb < 1 ? 1 : (nb > kMaxRedBlocks ? kMaxRedBlocks : nb);
}
// stencil kernels with reductions: one block per kBlock sites, capped at
// stencil_block_cap(); the kernels loop over site blocks beyond the cap
inline int stencil_grid(int V) {
  int nb = nblocks_for(size_t(V));
  const int cap = stencil_block_cap();
  return nb > cap ? cap : nb;
}
// the BiCG matvec: one work item per (tile, pass)
inline int matvec_grid(int V) { return 2 * stencil_grid(V); }
inline int stream_grid(size_t n) {
  int nb = nblocks_for(n, 4);
  return nb < 1 ? 1 : (nb > 8192 ? 8192 : nb);
}

// grids: records of KC * NV doubles per block must fit one scratch region
inline int batch_stencil_grid(int V, int kc, int nv) {
  int nb = nblocks_for(size_t(V) * kc);
  const int cap = int(kRegion / size_t(kc * nv));
  const int scap = stencil_block_cap();
  nb = nb > scap ? scap : nb;
  return nb > cap ? cap : nb;
}
inline int batch_red_grid(size_t n, int kc, int nv) {
  int nb = red_grid(n);
  const int cap = int(kRegion / size_t(kc * nv));
  return nb > cap ? cap : nb;
}

template <typename F>
void dispatch_kc(int kc, F &&f) {
  switch (kc) {
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 8: f(std::integral_constant<int, 8>{}); break;
    case 16: f(std::integral_constant<int, 16>{}); break;
    default: break;  // the host validates kc
  }
}

__device__ __forceinline__ bool skip_iter(const KrylovState *S, int j) { return S->stopped && j > S->stop_at; }

__device__ __forceinline__ cx<double> cdiv(cx<double> a, cx<double> b) {
  const double d = b.x * b.x + b.y * b.y;
  return {(a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d};
}
__device__ __forceinline__ cx<double> c2(double2 v) { return {v.x, v.y}; }
__device__ __forceinline__ double2 d2(cx<double> v) { return make_double2(v.x, v.y); }

}  // namespace
}  // namespace ebicg
