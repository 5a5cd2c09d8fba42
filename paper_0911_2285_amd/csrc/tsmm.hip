// Tall-skinny complex products.
//
//   gram:    out = X^+ Y              X: N x nx, Y: N x ny, out: nx x ny  (FP64 matrix cores)
//   combine: out = [out +] In C       In: N x nin, C: nin x nout, out: N x nout  (FP64 VALU;
//            rotations into more than 24 columns on the matrix cores, FP32 for FP32 windows)
//
// N is the length of a spinor (12 V complex entries) and the other sizes are
// at most 128, so both products are long contractions into small tiles or
// small contractions of long columns.  They carry the projections of the
// deflation space (Alg. Incremental eigBiCG: biorthogonalisation of new pairs,
// extension of H = U_l^+ A U_r) and the window rotation of Alg. BiCG-eigen
// (V <- V Y, W <- W Z).
//
// Complex arithmetic on the real matrix cores: with x = xr + i xi,
//   conj(x) y = (xr yr + xi yi) + i (xr yi - xi yr)
//   x c       = (xr cr - xi ci) + i (xr ci + xi cr)
// so every complex entry of the contraction is two real k-steps, feeding the
// real and the imaginary accumulator tiles with permuted/negated operands.
//
// v_mfma_f64_16x16x4f64 (one wave): D(16x16) += A(16x4) B(4x16); lane l
// holds A[l % 16][l / 16], B[l / 16][l % 16] and D[l / 16 + 4 v][l % 16]
// in component v of its 4-double accumulator (checked by a lane probe).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_common.h"
#include "kernels.h"

namespace ebicg {
namespace {

typedef double dx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ dx4 mfma16(double a, double b, dx4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// FP32: v_mfma_f32_16x16x4f32 (one block) takes A and B as the FP64 form does,
// but lane l holds D[4 (l / 16) + v][l % 16] in component v (a lane probe).
typedef float fx4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ fx4 mfma16(float a, float b, fx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

constexpr int kTile = 16;                    // MFMA tile edge
constexpr int kTileRec = 2 * kTile * kTile;  // doubles of one complex 16 x 16 tile

// ---------------------------------------------------------------------------
// gram: partial tiles of X^+ Y.  Block = 4 waves over one 16-column group of Y
// (blockIdx.y) and all TA 16-column groups of X; the waves take 16-entry
// chunks in turn.  In a chunk, lane (r = l % 16, q = l / 16) reads entries
// 16 c + 4 u + q (u = 0..3) of X column 16 ta + r and of Y column 16 tb + r,
// so each load instruction reads 64 contiguous bytes of 16 columns.  The
// block sums its waves' tiles in LDS and writes one record of TA tiles.
// ---------------------------------------------------------------------------
template <int TA>
__global__ void __launch_bounds__(kBlock)
    k_gram_mfma(const double2 *__restrict__ X, size_t ldx, int nx, const double2 *__restrict__ Y, size_t ldy,
                int ny, size_t N, double *__restrict__ part) {
  __shared__ double sm[kBlock / kWave][kTileRec];
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int r = lane % kTile, q = lane / kTile;
  const int b = blockIdx.y * kTile + r;
  const bool hb = b < ny;
  const double2 *yb = Y + size_t(hb ? b : 0) * ldy;
  const double2 *xa[TA];
  bool ha[TA];
#pragma unroll
  for (int t = 0; t < TA; ++t) {
    const int a = t * kTile + r;
    ha[t] = a < nx;
    xa[t] = X + size_t(ha[t] ? a : 0) * ldx;
  }
  dx4 re[TA], im[TA];
#pragma unroll
  for (int t = 0; t < TA; ++t) re[t] = im[t] = dx4{0.0, 0.0, 0.0, 0.0};

  const size_t nch = (N + kTile - 1) / kTile;
  const size_t stride = size_t(gridDim.x) * (kBlock / kWave);
  for (size_t c = size_t(blockIdx.x) * (kBlock / kWave) + w; c < nch; c += stride) {
    double2 yv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const size_t i = c * kTile + 4 * u + q;
      yv[u] = (hb && i < N) ? yb[i] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int t = 0; t < TA; ++t) {
      double2 xv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const size_t i = c * kTile + 4 * u + q;
        xv[u] = (ha[t] && i < N) ? xa[t][i] : make_double2(0.0, 0.0);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        re[t] = mfma16(xv[u].x, yv[u].x, re[t]);
        im[t] = mfma16(xv[u].x, yv[u].y, im[t]);
        re[t] = mfma16(xv[u].y, yv[u].y, re[t]);
        im[t] = mfma16(xv[u].y, -yv[u].x, im[t]);
      }
    }
  }
  // Block sum of the waves' tiles, one tile at a time; record layout
  // [(a_local * 16 + b_local) * 2 + {re, im}], a_local = q + 4 v, b_local = r.
#pragma unroll
  for (int t = 0; t < TA; ++t) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int e = ((q + 4 * v) * kTile + r) * 2;
      sm[w][e] = re[t][v];
      sm[w][e + 1] = im[t][v];
    }
    __syncthreads();
    double *rec = part + ((size_t(blockIdx.y) * TA + t) * gridDim.x + blockIdx.x) * kTileRec;
    for (int e = threadIdx.x; e < kTileRec; e += kBlock) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < kBlock / kWave; ++k) s += sm[k][e];
      rec[e] = s;
    }
    __syncthreads();
  }
}

// out[a + b nx] = sum of the records of tile (ta, tb), blocks in order.
// Grid: (TA * TB tiles, 16 slices of 16 tile entries); in a block, thread
// (e = t % 16, s = t / 16) sums records s, s + 16, ... of entry e, then the 16
// sums of each entry are added in order of s.
__global__ void __launch_bounds__(kBlock)
    k_gram_finish(double2 *out, const double *__restrict__ part, int nblk, int TA, int nx, int ny) {
  __shared__ double sm[kTile][kTile][2];
  const int tile = blockIdx.x;  // tb * TA + ta
  const int e = blockIdx.y * kTile + threadIdx.x % kTile, s = threadIdx.x / kTile;
  const double *rec = part + size_t(tile) * nblk * kTileRec + 2 * e;
  double sr = 0.0, si = 0.0;
  for (int k = s; k < nblk; k += kTile) {
    sr += rec[size_t(k) * kTileRec];
    si += rec[size_t(k) * kTileRec + 1];
  }
  sm[s][threadIdx.x % kTile][0] = sr;
  sm[s][threadIdx.x % kTile][1] = si;
  __syncthreads();
  if (threadIdx.x < kTile) {
    double tr = 0.0, ti = 0.0;
    for (int k = 0; k < kTile; ++k) {
      tr += sm[k][threadIdx.x][0];
      ti += sm[k][threadIdx.x][1];
    }
    const int ta = tile % TA, tb = tile / TA;
    const int a = ta * kTile + e / kTile, b = tb * kTile + e % kTile;
    if (a < nx && b < ny) out[a + size_t(b) * nx] = make_double2(tr, ti);
  }
}

// ---------------------------------------------------------------------------
// combine: out_k = [out_k +] sgn sum_c in_c C[c + k nin] for the NT output
// columns k0 = NT blockIdx.y .. of this block, one entry per thread.  The
// coefficient C[c, k] is the same for every lane, so it reaches the FMAs
// through scalar loads and no tile is padded: on this chip the FP64 matrix
// cores sustain about half the FP64 vector rate on these shapes, and padding
// 20 output columns to a 32-wide tile wastes another third.  DOTS: one
// element per thread, and the block's partial dots of g with the new outputs,
// g^+ out_k (conj_out = 0) or out_k^+ g (conj_out = 1), as element-major
// records part[(blockIdx.y 2NT + e) gridDim.x + blockIdx.x].
// ---------------------------------------------------------------------------
// G5IN: an input slot -(slot + 1) is read as gamma5 times that column (spinor
// columns of length N = 12 V: the second half, components 6..11, flips sign).
// TI, TO: storage of the input and output columns (double2, or float2 for an
// FP32 window); coefficients, accumulation and dots stay FP64.
template <typename TI, typename TO, int NT, bool ADD, bool DOTS, bool G5IN>
__global__ void __launch_bounds__(kBlock)
    k_combine(TO *out_base, SlotList out_slots, size_t ldo, const TI *in_base, SlotList in_slots,
              size_t ldi, const double2 *__restrict__ C, double sgn, size_t N, const double2 *__restrict__ g,
              int conj_out, double *__restrict__ part, int jtag, const KrylovState *S) {
  if (S && S->stopped && jtag > S->stop_at) return;
  const int nin = in_slots.n, nout = out_slots.n;
  const int k0 = blockIdx.y * NT;
  const int nk = nout - k0 < NT ? nout - k0 : NT;
  const double2 *__restrict__ Ck = C + size_t(k0) * nin;  // coefficient (c, k0 + k) at Ck[c + k nin]
  const size_t half = N / 2;
  auto load_in = [&](int c, size_t i) -> cx<double> {
    int sc = in_slots.idx[c];
    if constexpr (G5IN) {
      const bool flip = sc < 0;
      if (flip) sc = -sc - 1;
      const TI t = in_base[size_t(sc) * ldi + i];
      return (flip && i >= half) ? cx<double>{-double(t.x), -double(t.y)} : cx<double>{double(t.x), double(t.y)};
    } else {
      const TI t = in_base[size_t(sc) * ldi + i];
      return {double(t.x), double(t.y)};
    }
  };
  cx<double> acc[NT];
  auto element = [&](size_t i) {
#pragma unroll
    for (int k = 0; k < NT; ++k) acc[k] = {0.0, 0.0};
    int c = 0;
    for (; c + 2 <= nin; c += 2) {
      const cx<double> v0 = load_in(c, i), v1 = load_in(c + 1, i);
#pragma unroll
      for (int k = 0; k < NT; ++k)
        if (k < nk) {
          const double2 w0 = Ck[c + size_t(k) * nin], w1 = Ck[c + 1 + size_t(k) * nin];
          cfma(acc[k], v0, cx<double>{w0.x, w0.y});
          cfma(acc[k], v1, cx<double>{w1.x, w1.y});
        }
    }
    if (c < nin) {
      const cx<double> v0 = load_in(c, i);
#pragma unroll
      for (int k = 0; k < NT; ++k)
        if (k < nk) {
          const double2 w0 = Ck[c + size_t(k) * nin];
          cfma(acc[k], v0, cx<double>{w0.x, w0.y});
        }
    }
#pragma unroll
    for (int k = 0; k < NT; ++k) {
      if (k >= nk) continue;
      TO *oc = out_base + size_t(out_slots.idx[k0 + k]) * ldo;
      cx<double> o = {sgn * acc[k].x, sgn * acc[k].y};
      if constexpr (ADD) {
        const TO old = oc[i];
        o = {double(old.x) + o.x, double(old.y) + o.y};
      }
      if constexpr (std::is_same<TO, double2>::value)
        oc[i] = make_double2(o.x, o.y);
      else
        oc[i] = make_float2(float(o.x), float(o.y));
      acc[k] = o;
    }
  };
  if constexpr (!DOTS) {
    for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < N; i += size_t(gridDim.x) * kBlock) element(i);
  } else {
    // one element per thread: the dots are formed from the finished outputs
    // in place and reduced four outputs at a time, so they add few live
    // registers to the contraction
    const size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x;
#pragma unroll
    for (int k = 0; k < NT; ++k) acc[k] = {0.0, 0.0};
    double2 gv = make_double2(0.0, 0.0);
    if (i < N) {
      element(i);
      gv = g[i];
    }
#pragma unroll
    for (int k4 = 0; k4 < NT; k4 += 4) {
      double t[8];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const cx<double> o = acc[k4 + q];
        if (conj_out) {  // conj(o) g
          t[2 * q] = o.x * gv.x + o.y * gv.y;
          t[2 * q + 1] = o.x * gv.y - o.y * gv.x;
        } else {  // conj(g) o
          t[2 * q] = gv.x * o.x + gv.y * o.y;
          t[2 * q + 1] = gv.x * o.y - gv.y * o.x;
        }
      }
      block_sum<8, kBlock>(t);
      if (threadIdx.x == 0)
#pragma unroll
        for (int e = 0; e < 8; ++e)
          part[(size_t(blockIdx.y) * 2 * NT + 2 * k4 + e) * gridDim.x + blockIdx.x] = t[e];
    }
  }
}

// ---------------------------------------------------------------------------
// rotate on the matrix cores: out_k = sgn sum_c in_c C[c + k nin] for all
// nout <= 16 OT output columns in one pass over the inputs (the window
// rotation of Alg. BiCG-eigen at large windows, e.g. 60 columns into 50).
// The transposed product out^T = C^T in^T is tiled: a wave takes 16 entries
// i and 16 outputs k per tile, K over the input columns in steps of 4, so that
// lane (r = l % 16, q = l / 16) loads entry i0 + r of input column c0 + q
// (16 consecutive entries per column: one 256-byte read) and holds the
// results for entry i0 + r of outputs q + 4 v (16 consecutive entries per
// output column in one store).  C^T sits in LDS ([c][k], k fastest), the
// slot lists too.  A complex product is four real MFMAs into a real and an
// imaginary tile.  With FP32 inputs and outputs (the FP32 window) the
// products and sums run in FP32 on the FP32 matrix instructions (twice the
// FP64 rate on gfx950); otherwise in FP64.  DOTS: the block's partial dots
// of g with the outputs (g^+ out_k, or out_k^+ g with conj_out), in FP64,
// element-major records part[(2 k + {re, im}) gridDim.x + blockIdx.x] for
// k < 16 OT.
// ---------------------------------------------------------------------------
template <typename TI, typename TO, int OT, bool DOTS, bool G5IN>
__global__ void __launch_bounds__(kBlock)
    k_rotate_mfma(TO *out_base, SlotList out_slots, size_t ldo, const TI *in_base, SlotList in_slots, size_t ldi,
                  const double2 *__restrict__ C, double sgn, size_t N, const double2 *__restrict__ g, int conj_out,
                  double *__restrict__ part, int jtag, const KrylovState *S) {
  if (S && S->stopped && jtag > S->stop_at) return;
  constexpr int KP = kTile * OT;
  constexpr bool F32 = std::is_same<TI, float2>::value && std::is_same<TO, float2>::value;
  using E = typename std::conditional<F32, float, double>::type;  // product and sum type
  using Acc = typename std::conditional<F32, fx4, dx4>::type;
  // output row of component v of lane (r, q) in a 16 x 16 tile
  auto orow = [](int q, int v) { return F32 ? 4 * q + v : q + 4 * v; };
  // C^T: cs[c KP + k], in the product type (FP32 coefficients for the FP32
  // window: half the LDS, so more blocks fit a CU)
  using CS = typename std::conditional<F32, float2, double2>::type;
  extern __shared__ double2 cs_lds[];
  CS *cs = reinterpret_cast<CS *>(cs_lds);
  __shared__ int islot[kMaxCols], oslot[KP];
  __shared__ double sd[DOTS ? kBlock / kWave : 1][DOTS ? 2 * KP : 1];
  const int nin = in_slots.n, nout = out_slots.n, nin4 = (nin + 3) & ~3;
  for (int e = threadIdx.x; e < nin4 * KP; e += kBlock) {
    const int c = e / KP, k = e % KP;
    const double2 a = (c < nin && k < nout) ? C[c + size_t(k) * nin] : make_double2(0.0, 0.0);
    cs[e] = CS{E(a.x), E(a.y)};
  }
  for (int c = threadIdx.x; c < kMaxCols; c += kBlock) islot[c] = c < nin ? in_slots.idx[c] : 0;
  for (int k = threadIdx.x; k < KP; k += kBlock) oslot[k] = k < nout ? out_slots.idx[k] : 0;
  __syncthreads();
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int r = lane % kTile, q = lane / kTile;
  const size_t half = N / 2, nch = (N + kTile - 1) / kTile;
  double dre[OT][4], dim[OT][4];
#pragma unroll
  for (int t = 0; t < OT; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) dre[t][v] = dim[t][v] = 0.0;
  for (size_t ch = size_t(blockIdx.x) * (kBlock / kWave) + w; ch < nch; ch += size_t(gridDim.x) * (kBlock / kWave)) {
    const size_t i = ch * kTile + r;
    const bool in = i < N;
    Acc re[OT], im[OT];
#pragma unroll
    for (int t = 0; t < OT; ++t) re[t] = im[t] = Acc{E(0), E(0), E(0), E(0)};
    // entry i of input column c.  Past the inputs (c >= nin) the first input
    // column is read instead, and past N its entry 0: the padded rows of C^T
    // are zero, and rows past N are neither stored nor dotted (g is taken as
    // 0 there), so every load is unconditional and nothing but the products
    // reads its value
    const size_t ii = in ? i : 0;
    auto load = [&](int c, E &br, E &bi) {
      int sc = islot[c < nin ? c : 0];
      if constexpr (G5IN) {
        if (sc < 0) sc = -sc - 1;
      }
      const TI x = in_base[size_t(sc) * ldi + ii];
      br = E(x.x);
      bi = E(x.y);
    };
    // the products of input columns c0 .. c0 + 3 (this lane's column c0 + q);
    // gamma5 is applied here, where the entry is used, not where it is loaded
    auto step = [&](int c0, E br, E bi) {
      const int c = c0 + q;
      if constexpr (G5IN) {
        if (islot[c < nin ? c : 0] < 0 && i >= half) {
          br = -br;
          bi = -bi;
        }
      }
#pragma unroll
      for (int t = 0; t < OT; ++t) {
        const CS a = cs[c * KP + kTile * t + r];
        const E ax = a.x, ay = a.y;
        re[t] = mfma16(ax, br, re[t]);
        re[t] = mfma16(-ay, bi, re[t]);
        im[t] = mfma16(ax, bi, im[t]);
        im[t] = mfma16(ay, br, im[t]);
      }
    };
    // two input buffers: the next step's entry is requested before this
    // step's products, so a load is in flight while the matrix instructions
    // run (the scheduling barriers keep the compiler from gathering the loads
    // at the top of the loop, where each would be waited for at once)
    if (nin > 0) {
      E ar, ai, br, bi;
      load(q, ar, ai);
      int c0 = 0;
      for (; c0 + 8 <= nin4; c0 += 8) {
        load(c0 + 4 + q, br, bi);
        __builtin_amdgcn_sched_barrier(0);
        step(c0, ar, ai);
        __builtin_amdgcn_sched_barrier(0);
        load(c0 + 8 + q, ar, ai);
        __builtin_amdgcn_sched_barrier(0);
        step(c0 + 4, br, bi);
        __builtin_amdgcn_sched_barrier(0);
      }
      if (c0 < nin4) step(c0, ar, ai);  // the last 4 columns when nin4 is not a multiple of 8
    }
    double2 gv = make_double2(0.0, 0.0);
    if (DOTS && in) gv = g[i];
#pragma unroll
    for (int t = 0; t < OT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = kTile * t + orow(q, v);
        const double ox = sgn * double(re[t][v]), oy = sgn * double(im[t][v]);
        if (in && k < nout) {
          TO *oc = out_base + size_t(oslot[k]) * ldo;
          if constexpr (std::is_same<TO, double2>::value)
            oc[i] = make_double2(ox, oy);
          else
            oc[i] = make_float2(float(ox), float(oy));
        }
        if constexpr (DOTS) {
          if (conj_out) {  // conj(o) g
            dre[t][v] += ox * gv.x + oy * gv.y;
            dim[t][v] += ox * gv.y - oy * gv.x;
          } else {  // conj(g) o
            dre[t][v] += gv.x * ox + gv.y * oy;
            dim[t][v] += gv.x * oy - gv.y * ox;
          }
        }
      }
  }
  if constexpr (DOTS) {
    // sum over the 16 lanes of each q (the entries), then over the waves
#pragma unroll
    for (int t = 0; t < OT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
#pragma unroll
        for (int off = kTile / 2; off > 0; off >>= 1) {
          dre[t][v] += __shfl_xor(dre[t][v], off, kWave);
          dim[t][v] += __shfl_xor(dim[t][v], off, kWave);
        }
        if (r == 0) {
          const int k = kTile * t + orow(q, v);
          sd[w][2 * k] = dre[t][v];
          sd[w][2 * k + 1] = dim[t][v];
        }
      }
    __syncthreads();
    for (int e = threadIdx.x; e < 2 * KP; e += kBlock) {
      double s = 0.0;
#pragma unroll
      for (int ww = 0; ww < kBlock / kWave; ++ww) s += sd[ww][e];
      part[size_t(e) * gridDim.x + blockIdx.x] = s;
    }
  }
}

// Partial dots of g with NT output columns of a rotation (column group
// blockIdx.y): g^+ out_k (conj_out = 0) or out_k^+ g (conj_out = 1); records
// element-major, part[(blockIdx.y 2NT + e) gridDim.x + blockIdx.x].
template <typename TO, int NT>
__global__ void __launch_bounds__(kBlock)
    k_slot_dots(const TO *base, SlotList slots, size_t ld, const double2 *__restrict__ g, size_t N, int conj_out,
                int jtag, const KrylovState *S, double *__restrict__ part) {
  if (S && S->stopped && jtag > S->stop_at) return;
  const int k0 = blockIdx.y * NT;
  const int nk = slots.n - k0 < NT ? slots.n - k0 : NT;
  double dv[2 * NT];
#pragma unroll
  for (int e = 0; e < 2 * NT; ++e) dv[e] = 0.0;
  for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < N; i += size_t(gridDim.x) * kBlock) {
    const double2 gv = g[i];
#pragma unroll
    for (int k = 0; k < NT; ++k) {
      if (k >= nk) continue;
      const TO ov = base[size_t(slots.idx[k0 + k]) * ld + i];
      const double2 o = make_double2(double(ov.x), double(ov.y));
      if (conj_out) {  // conj(o) g
        dv[2 * k] += o.x * gv.x + o.y * gv.y;
        dv[2 * k + 1] += o.x * gv.y - o.y * gv.x;
      } else {  // conj(g) o
        dv[2 * k] += gv.x * o.x + gv.y * o.y;
        dv[2 * k + 1] += gv.x * o.y - gv.y * o.x;
      }
    }
  }
  block_sum<2 * NT, kBlock>(dv);
  if (threadIdx.x == 0)
    for (int e = 0; e < 2 * NT; ++e) part[(size_t(blockIdx.y) * 2 * NT + e) * gridDim.x + blockIdx.x] = dv[e];
}

// One block per record element (blockIdx.x = group * 2KW + e): thread t sums
// the blocks t, t + 256, ... and the block adds the 256 sums in a fixed tree.
template <int KW>
__global__ void __launch_bounds__(kBlock)
    k_combine_dots(const double *__restrict__ part, int nblk, int nout, double2 *dots, int jtag,
                   const KrylovState *S) {
  if (S && S->stopped && jtag > S->stop_at) return;
  const double *rec = part + size_t(blockIdx.x) * nblk;
  double v[1] = {0.0};
  for (int k = threadIdx.x; k < nblk; k += kBlock) v[0] += rec[k];
  block_sum<1, kBlock>(v);
  const int grp = blockIdx.x / (2 * KW), e = blockIdx.x % (2 * KW);
  const int kk = grp * KW + e / 2;
  if (threadIdx.x == 0 && kk < nout) reinterpret_cast<double *>(dots)[2 * kk + e % 2] = v[0];
}

}  // namespace

void launch_gram_mfma(double2 *out, const double2 *X, size_t ldx, int nx, const double2 *Y, size_t ldy, int ny,
                      size_t N, double *part, size_t part_cap, hipStream_t st) {
  const int TA = (nx + kTile - 1) / kTile, TB = (ny + kTile - 1) / kTile;
  if (TA < 1 || TA > 8 || TB < 1 || N == 0) return;
  // about 2 blocks per CU in total, bounded by the chunks and the record space
  const size_t nch = (N + kTile - 1) / kTile;
  size_t nb = (512 + TB - 1) / TB;
  const size_t by_chunks = (nch + 3) / 4;
  const size_t by_space = part_cap / (size_t(TA) * TB * kTileRec);
  nb = nb < by_chunks ? nb : by_chunks;
  nb = nb < by_space ? nb : by_space;
  if (nb < 1) nb = 1;
  const dim3 grid = dim3(unsigned(nb), unsigned(TB));
  auto go = [&](auto ta_tag) {
    constexpr int T = decltype(ta_tag)::value;
    EB_LAUNCH(k_gram_mfma<T>, grid, dim3(kBlock), 0, st, X, ldx, nx, Y, ldy, ny, N, part);
  };
  switch (TA) {
    case 1: go(std::integral_constant<int, 1>{}); break;
    case 2: go(std::integral_constant<int, 2>{}); break;
    case 3: go(std::integral_constant<int, 3>{}); break;
    case 4: go(std::integral_constant<int, 4>{}); break;
    case 5: go(std::integral_constant<int, 5>{}); break;
    case 6: go(std::integral_constant<int, 6>{}); break;
    case 7: go(std::integral_constant<int, 7>{}); break;
    default: go(std::integral_constant<int, 8>{}); break;
  }
  EB_LAUNCH(k_gram_finish, dim3(TA * TB, kTile), dim3(kBlock), 0, st, out, part, int(nb), TA, nx, ny);
}

template <typename TI, typename TO>
void launch_combine_t(TO *out_base, const SlotList &out_slots, size_t ldo, const TI *in_base,
                      const SlotList &in_slots, size_t ldi, const double2 *C, double sgn, bool add, size_t N,
                      const double2 *g, int conj_out, double2 *dots, int jtag, const KrylovState *S, double *part,
                      size_t part_cap, hipStream_t st) {
  const int nin = in_slots.n, nout = out_slots.n;
  if (nin < 1 || nout < 1 || N == 0) return;
  if (!add && nout > 24 && nout <= 4 * kTile && sgn == 1.0) {
    // a rotation into more than 24 columns: the matrix cores, the inputs read once
    bool g5in = false;
    for (int c = 0; c < nin; ++c) g5in = g5in || in_slots.idx[c] < 0;
    const int OT = (nout + kTile - 1) / kTile;
    const size_t nch = (N + kTile - 1) / kTile;
    size_t nb = (nch + 3) / 4;
    nb = nb < 2048 ? nb : 2048;
    if (g) {  // the dot records of 2 KW rows, KW = 16 OT
      const size_t rcap = part_cap / (2 * size_t(kTile) * OT);
      nb = nb < rcap ? nb : rcap;
    }
    if (nb < 1) nb = 1;
    auto go = [&](auto ot_tag, auto dots_tag, auto g5_tag) {
      constexpr int T = decltype(ot_tag)::value;
      constexpr bool D = decltype(dots_tag)::value, G = decltype(g5_tag)::value;
      constexpr bool F32 = std::is_same<TI, float2>::value && std::is_same<TO, float2>::value;
      const size_t lds = size_t((nin + 3) & ~3) * kTile * T * (F32 ? sizeof(float2) : sizeof(double2));
      // the kernel's static LDS (slot lists, dot sums) comes on top of this; past 64 KB in
      // all a workgroup needs the larger limit set (gfx950 holds 160 KB per workgroup)
      (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_rotate_mfma<TI, TO, T, D, G>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));  // a failure shows at launch
      EB_LAUNCH((k_rotate_mfma<TI, TO, T, D, G>), dim3(unsigned(nb)), dim3(kBlock), lds, st, out_base, out_slots, ldo,
                in_base, in_slots, ldi, C, sgn, N, g, conj_out, part, jtag, S);
      if constexpr (D)
        EB_LAUNCH(k_combine_dots<kTile * T>, dim3(2 * kTile * T), dim3(kBlock), 0, st, part, int(nb), nout, dots,
                  jtag, S);
    };
    using Tt = std::true_type;
    using Ff = std::false_type;
    auto by_flags = [&](auto ot_tag) {
      if (g && g5in)
        go(ot_tag, Tt{}, Tt{});
      else if (g)
        go(ot_tag, Tt{}, Ff{});
      else if (g5in)
        go(ot_tag, Ff{}, Tt{});
      else
        go(ot_tag, Ff{}, Ff{});
    };
    if (OT == 2)
      by_flags(std::integral_constant<int, 2>{});
    else if (OT == 3)
      by_flags(std::integral_constant<int, 3>{});
    else
      by_flags(std::integral_constant<int, 4>{});
    return;
  }
  auto go = [&](auto nt_tag) {
    constexpr int NT = decltype(nt_tag)::value;
    const int groups = (nout + NT - 1) / NT;
    size_t nb = (N + kBlock - 1) / kBlock;
    const size_t cap = (4096 + groups - 1) / groups;
    nb = nb < cap ? nb : cap;
    const dim3 grid = dim3(unsigned(nb), unsigned(groups));
    bool g5in = false;
    for (int c = 0; c < nin; ++c) g5in = g5in || in_slots.idx[c] < 0;
    auto launch = [&](auto add_tag, auto dots_tag, auto g5_tag, dim3 gr) {
      constexpr bool A = decltype(add_tag)::value, D = decltype(dots_tag)::value, G = decltype(g5_tag)::value;
      if constexpr (A && !std::is_same<TO, double2>::value) {
        return;  // accumulating outputs are FP64 only (the host never asks for FP32 ones)
      } else {
        EB_LAUNCH((k_combine<TI, TO, NT, A, D, G>), gr, dim3(kBlock), 0, st, out_base, out_slots, ldo, in_base,
                  in_slots, ldi, C, sgn, N, g, conj_out, part, jtag, S);
      }
    };
    using T = std::true_type;
    using F = std::false_type;
    // a rotation with dots: one element per thread when the dot records fit
    const size_t nfull = (N + kBlock - 1) / kBlock;
    if (g && !add && nfull * groups * 2 * NT <= part_cap && nfull <= 0x7fffffff) {
      const dim3 gfull = dim3(unsigned(nfull), unsigned(groups));
      if (g5in)
        launch(F{}, T{}, T{}, gfull);
      else
        launch(F{}, T{}, F{}, gfull);
      EB_LAUNCH(k_combine_dots<NT>, dim3(groups * 2 * NT), dim3(kBlock), 0, st, part, int(nfull), nout, dots, jtag, S);
      return;
    }
    if (add && g5in)
      launch(T{}, F{}, T{}, grid);
    else if (add)
      launch(T{}, F{}, F{}, grid);
    else if (g5in)
      launch(F{}, F{}, T{}, grid);
    else
      launch(F{}, F{}, F{}, grid);
    if (g) {
      // dots of the fresh outputs with g, a light second pass (nout + 1 columns)
      size_t nd = (N + kBlock - 1) / kBlock;
      size_t dcap = part_cap / (size_t(groups) * 2 * NT);
      dcap = dcap < 1024 ? dcap : 1024;
      nd = nd < dcap ? nd : dcap;
      if (nd < 1) nd = 1;
      EB_LAUNCH((k_slot_dots<TO, NT>), dim3(unsigned(nd), unsigned(groups)), dim3(kBlock), 0, st, out_base,
                out_slots, ldo, g, N, conj_out, jtag, S, part);
      EB_LAUNCH(k_combine_dots<NT>, dim3(groups * 2 * NT), dim3(kBlock), 0, st, part, int(nd), nout, dots, jtag, S);
    }
  };
  if (nout <= 4)
    go(std::integral_constant<int, 4>{});
  else if (nout <= 8)
    go(std::integral_constant<int, 8>{});
  else if (nout <= 12)
    go(std::integral_constant<int, 12>{});
  else if (nout <= 16)
    go(std::integral_constant<int, 16>{});
  else if (nout <= 20)
    go(std::integral_constant<int, 20>{});
  else
    go(std::integral_constant<int, 24>{});
}

void launch_combine(double2 *out_base, const SlotList &out_slots, size_t ldo, const double2 *in_base,
                    const SlotList &in_slots, size_t ldi, const double2 *C, double sgn, bool add, size_t N,
                    const double2 *g, int conj_out, double2 *dots, int jtag, const KrylovState *S, double *part,
                    size_t part_cap, hipStream_t st) {
  launch_combine_t(out_base, out_slots, ldo, in_base, in_slots, ldi, C, sgn, add, N, g, conj_out, dots, jtag, S, part,
                   part_cap, st);
}
void launch_combine(float2 *out_base, const SlotList &out_slots, size_t ldo, const float2 *in_base,
                    const SlotList &in_slots, size_t ldi, const double2 *C, size_t N, const double2 *g, int conj_out,
                    double2 *dots, int jtag, const KrylovState *S, double *part, size_t part_cap, hipStream_t st) {
  launch_combine_t(out_base, out_slots, ldo, in_base, in_slots, ldi, C, 1.0, false, N, g, conj_out, dots, jtag, S,
                   part, part_cap, st);
}
void launch_combine(double2 *out_base, const SlotList &out_slots, size_t ldo, const float2 *in_base,
                    const SlotList &in_slots, size_t ldi, const double2 *C, size_t N, const double2 *g, int conj_out,
                    double2 *dots, int jtag, const KrylovState *S, double *part, size_t part_cap, hipStream_t st) {
  launch_combine_t(out_base, out_slots, ldo, in_base, in_slots, ldi, C, 1.0, false, N, g, conj_out, dots, jtag, S,
                   part, part_cap, st);
}

}  // namespace ebicg
