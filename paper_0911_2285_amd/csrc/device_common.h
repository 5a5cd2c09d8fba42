// Device-side building blocks shared by the kernels: complex arithmetic,
// storage formats (FP64, FP32, BF16 pairs), wave64/block reductions with a
// deterministic last-block finish, and the XCD-aware block remap.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ebicg {

constexpr int kBlock = 256;   // threads per block of the streaming kernels
constexpr int kWave = 64;     // CDNA wavefront width
constexpr int kNumXcd = 8;    // MI355X: 8 XCDs, each with its own L2

// ----------------------------------------------------------------- complex
template <typename R>
struct cx {
  R x, y;
};

template <typename R>
__device__ __forceinline__ cx<R> mk(R a, R b) {
  return cx<R>{a, b};
}
template <typename R>
__device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) {
  return {a.x + b.x, a.y + b.y};
}
template <typename R>
__device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) {
  return {a.x - b.x, a.y - b.y};
}
template <typename R>
__device__ __forceinline__ cx<R> operator-(cx<R> a) {
  return {-a.x, -a.y};
}
template <typename R>
__device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename R>
__device__ __forceinline__ cx<R> operator*(R s, cx<R> a) {
  return {s * a.x, s * a.y};
}
template <typename R>
__device__ __forceinline__ cx<R> cconj(cx<R> a) {
  return {a.x, -a.y};
}
// conj(a) * b
template <typename R>
__device__ __forceinline__ cx<R> cmulc(cx<R> a, cx<R> b) {
  return {a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}
// i * a
template <typename R>
__device__ __forceinline__ cx<R> ci(cx<R> a) {
  return {-a.y, a.x};
}
// acc += a * b
template <typename R>
__device__ __forceinline__ void cfma(cx<R> &acc, cx<R> a, cx<R> b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}
// acc += conj(a) * b
template <typename R>
__device__ __forceinline__ void cfmac(cx<R> &acc, cx<R> a, cx<R> b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(-a.y, b.x, acc.y);
}

// ----------------------------------------------------------------- storage
// One complex number per element.  bf16c packs (re, im) as two bfloat16.
struct bf16c {
  uint32_t v;
};

__device__ __forceinline__ float bf16_to_f32(uint32_t h) { return __uint_as_float(h << 16); }
__device__ __forceinline__ uint32_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  uint32_t lsb = (u >> 16) & 1u;  // round to nearest even
  return (u + 0x7fffu + lsb) >> 16;
}

template <typename S>
struct Store;
template <>
struct Store<double2> {
  using R = double;
  static __device__ __forceinline__ cx<double> ld(const double2 *p, size_t i) {
    double2 v = p[i];
    return {v.x, v.y};
  }
  static __device__ __forceinline__ void st(double2 *p, size_t i, cx<double> a) { p[i] = make_double2(a.x, a.y); }
};
template <>
struct Store<float2> {
  using R = float;
  static __device__ __forceinline__ cx<float> ld(const float2 *p, size_t i) {
    float2 v = p[i];
    return {v.x, v.y};
  }
  template <typename T>
  static __device__ __forceinline__ void st(float2 *p, size_t i, cx<T> a) {
    p[i] = make_float2(float(a.x), float(a.y));
  }
};
template <>
struct Store<bf16c> {
  using R = float;
  static __device__ __forceinline__ cx<float> ld(const bf16c *p, size_t i) {
    uint32_t v = p[i].v;
    return {bf16_to_f32(v & 0xffffu), bf16_to_f32(v >> 16)};
  }
  template <typename T>
  static __device__ __forceinline__ void st(bf16c *p, size_t i, cx<T> a) {
    bf16c o;
    o.v = f32_to_bf16(float(a.x)) | (f32_to_bf16(float(a.y)) << 16);
    p[i] = o;
  }
};

// ----------------------------------------------------------------- launch geometry
// Workgroups are dispatched round-robin over the XCDs (block b -> XCD b % 8).
// Remap so that each XCD walks one contiguous range of logical blocks: the
// stencil's neighbours and the reuse between consecutive blocks then stay in
// that XCD's L2.  The map is a bijection on [0, nb).
__device__ __forceinline__ int xcd_remap(int bid, int nb) {
  const int q = nb / kNumXcd, r = nb % kNumXcd;
  const int x = bid % kNumXcd, slot = bid / kNumXcd;
  return x * q + (x < r ? x : r) + slot;
}

// ----------------------------------------------------------------- reductions
template <int NV>
__device__ __forceinline__ void wave_sum(double (&v)[NV]) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] += __shfl_xor(v[i], off, kWave);
  }
}

// Block-wide sum (fixed order); the result is valid in thread 0.
template <int NV, int BS>
__device__ __forceinline__ void block_sum(double (&v)[NV]) {
  __shared__ double sm[BS / kWave][NV];
  wave_sum<NV>(v);
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  __syncthreads();
  if (l == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) sm[w][i] = v[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double s = 0;
      for (int k = 0; k < BS / kWave; ++k) s += sm[k][i];
      v[i] = s;
    }
  }
}

// Write this block's partial sums (record of NV doubles at part[bid * NV]).
template <int NV, int BS>
__device__ __forceinline__ void block_partial(double (&v)[NV], double *__restrict__ part, int bid) {
  block_sum<NV, BS>(v);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) part[size_t(bid) * NV + i] = v[i];
  }
}

// Per-column block sums for KC right-hand sides interleaved as the fastest
// index: thread t of a block always carries column t % KC.  The wave sum runs
// over the lanes of one column (xor offsets >= KC), then over the waves; the
// record of KC * NV doubles [col][i] goes to part[bid * KC * NV].
template <int NV, int KC, int BS>
__device__ __forceinline__ void block_partial_cols(double (&v)[NV], double *__restrict__ part, int bid) {
  static_assert(KC >= 1 && KC <= kWave && (KC & (KC - 1)) == 0, "KC must be a power of two <= 64");
  __shared__ double sm[BS / kWave][KC][NV];
#pragma unroll
  for (int off = kWave / 2; off >= KC; off >>= 1) {
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] += __shfl_xor(v[i], off, kWave);
  }
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  __syncthreads();
  if (l < KC) {
#pragma unroll
    for (int i = 0; i < NV; ++i) sm[w][l][i] = v[i];
  }
  __syncthreads();
  if (threadIdx.x < KC * NV) {
    const int col = threadIdx.x / NV, i = threadIdx.x % NV;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < BS / kWave; ++k) s += sm[k][col][i];
    part[size_t(bid) * KC * NV + threadIdx.x] = s;
  }
}

// Sum of the nblk partial records written by the previous kernel, in a fixed
// order, so every block of the consuming kernel obtains the same totals (in
// every thread).  Kernel boundaries make the partials visible: no fences and
// no atomics are needed.
template <int NV, int BS>
__device__ __forceinline__ void sum_partials(const double *__restrict__ part, int nblk, double (&out)[NV]) {
  __shared__ double sm[BS / kWave][NV];
  double v[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = 0.0;
  for (int b = threadIdx.x; b < nblk; b += BS) {
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] += part[size_t(b) * NV + i];
  }
  wave_sum<NV>(v);
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  __syncthreads();
  if (l == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) sm[w][i] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double s = 0;
    for (int k = 0; k < BS / kWave; ++k) s += sm[k][i];
    out[i] = s;
  }
}

}  // namespace ebicg
