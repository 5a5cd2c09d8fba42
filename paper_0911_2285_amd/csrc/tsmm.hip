// Tall-skinny complex products on the FP64 matrix cores (gfx950 MFMA).
//
//   gram:    out = X^+ Y              X: N x nx, Y: N x ny, out: nx x ny
//   combine: out = [out +] In C       In: N x nin, C: nin x nout, out: N x nout
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
// combine: out_k = [out_k +] sum_c in_c C[c + k nin] over the output columns
// 16 TB blockIdx.y .. + 16 TB.  A wave owns RT row tiles of 16 entries and
// TB column tiles; lane (r, q) reads entry e0 + 16 t + r of input column
// c0 + q (64 lanes: four 256-byte runs) and coefficient C[c0 + q][k0 + 16 u + r]
// from LDS.  With g: partial dots g^+ out_k (conj_out = 0) or out_k^+ g
// (conj_out = 1), one record of 32 TB doubles per block.
// ---------------------------------------------------------------------------
template <int RT, int TB, bool ADD>
__global__ void __launch_bounds__(kBlock)
    k_combine_mfma(double2 *out_base, SlotList out_slots, size_t ldo, const double2 *in_base, SlotList in_slots,
                   size_t ldi, const double2 *__restrict__ C, double sgn, size_t N, const double2 *__restrict__ g,
                   int conj_out, int jtag, const KrylovState *S, double *__restrict__ part) {
  if (S && S->stopped && jtag > S->stop_at) return;
  extern __shared__ double2 sB[];  // [nin padded to 4][16 TB]
  __shared__ double sd[kBlock / kWave][2 * kTile * TB];
  constexpr int KW = kTile * TB;
  const int nin = in_slots.n, nout = out_slots.n;
  const int nin4 = (nin + 3) & ~3;
  const int k0 = blockIdx.y * KW;
  for (int e = threadIdx.x; e < nin4 * KW; e += kBlock) {
    const int c = e / KW, kk = e % KW;
    double2 v = make_double2(0.0, 0.0);
    if (c < nin && k0 + kk < nout) {
      const double2 cc = C[c + size_t(k0 + kk) * nin];
      v = make_double2(sgn * cc.x, sgn * cc.y);
    }
    sB[e] = v;
  }
  __syncthreads();
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int r = lane % kTile, q = lane / kTile;
  constexpr int ENT = RT * kTile;  // entries per wave tile
  const size_t ntile = (N + ENT - 1) / ENT;
  double dr[TB], di[TB];
#pragma unroll
  for (int u = 0; u < TB; ++u) dr[u] = di[u] = 0.0;

  for (size_t tile = size_t(blockIdx.x) * (kBlock / kWave) + w; tile < ntile;
       tile += size_t(gridDim.x) * (kBlock / kWave)) {
    const size_t e0 = tile * ENT;
    dx4 re[RT][TB], im[RT][TB];
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int u = 0; u < TB; ++u) re[t][u] = im[t][u] = dx4{0.0, 0.0, 0.0, 0.0};
    // groups of CS k-steps: all loads of a group are issued before its MFMAs
    constexpr int CS = 4;
    for (int cg = 0; cg < nin4; cg += 4 * CS) {
      double2 av[CS][RT];
#pragma unroll
      for (int s = 0; s < CS; ++s) {
        const int c = cg + 4 * s + q;
        const double2 *col = in_base + size_t(c < nin ? in_slots.idx[c] : 0) * ldi;
#pragma unroll
        for (int t = 0; t < RT; ++t) {
          const size_t i = e0 + t * kTile + r;
          av[s][t] = (c < nin && i < N) ? col[i] : make_double2(0.0, 0.0);
        }
      }
#pragma unroll
      for (int s = 0; s < CS; ++s) {
        const int c = cg + 4 * s + q;
        if (cg + 4 * s >= nin4) break;
        double2 bv[TB];
#pragma unroll
        for (int u = 0; u < TB; ++u) bv[u] = sB[c * KW + u * kTile + r];
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
          for (int u = 0; u < TB; ++u) {
            re[t][u] = mfma16(av[s][t].x, bv[u].x, re[t][u]);
            im[t][u] = mfma16(av[s][t].x, bv[u].y, im[t][u]);
            re[t][u] = mfma16(av[s][t].y, -bv[u].y, re[t][u]);
            im[t][u] = mfma16(av[s][t].y, bv[u].x, im[t][u]);
          }
      }
    }
    // lane holds entries e0 + 16 t + q + 4 v of output column k0 + 16 u + r
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      double2 gv[4];
      if (g) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const size_t i = e0 + t * kTile + q + 4 * v;
          gv[v] = i < N ? g[i] : make_double2(0.0, 0.0);
        }
      }
#pragma unroll
      for (int u = 0; u < TB; ++u) {
        const int k = k0 + u * kTile + r;
        if (k >= nout) continue;
        double2 *oc = out_base + size_t(out_slots.idx[k]) * ldo;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const size_t i = e0 + t * kTile + q + 4 * v;
          if (i >= N) continue;
          double2 o = make_double2(re[t][u][v], im[t][u][v]);
          if (ADD) {
            const double2 old = oc[i];
            o = make_double2(old.x + o.x, old.y + o.y);
          }
          oc[i] = o;
          if (g) {
            // conj(g) o, or conj(o) g
            const double gx = gv[v].x, gy = gv[v].y;
            if (conj_out) {
              dr[u] += o.x * gx + o.y * gy;
              di[u] += o.x * gy - o.y * gx;
            } else {
              dr[u] += gx * o.x + gy * o.y;
              di[u] += gx * o.y - gy * o.x;
            }
          }
        }
      }
    }
  }
  if (!g) return;
  // sum over the four lanes of a column (q), then over the block's waves
#pragma unroll
  for (int u = 0; u < TB; ++u) {
    dr[u] += __shfl_xor(dr[u], 16, kWave);
    di[u] += __shfl_xor(di[u], 16, kWave);
    dr[u] += __shfl_xor(dr[u], 32, kWave);
    di[u] += __shfl_xor(di[u], 32, kWave);
  }
  if (q == 0) {
#pragma unroll
    for (int u = 0; u < TB; ++u) {
      sd[w][2 * (u * kTile + r)] = dr[u];
      sd[w][2 * (u * kTile + r) + 1] = di[u];
    }
  }
  __syncthreads();
  if (threadIdx.x < 2 * KW) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kBlock / kWave; ++k) s += sd[k][threadIdx.x];
    // element-major records: element e of column group y at part[(y 2KW + e) nblk + block]
    part[(size_t(blockIdx.y) * 2 * KW + threadIdx.x) * gridDim.x + blockIdx.x] = s;
  }
}

// One block per record element (blockIdx.x = group * 2KW + e): thread t sums
// the blocks t, t + 256, ... and the block adds the 256 sums in a fixed tree.
template <int TB>
__global__ void __launch_bounds__(kBlock)
    k_combine_dots(const double *__restrict__ part, int nblk, int nout, double2 *dots, int jtag,
                   const KrylovState *S) {
  if (S && S->stopped && jtag > S->stop_at) return;
  constexpr int KW = kTile * TB;
  const double *rec = part + size_t(blockIdx.x) * nblk;
  double v[1] = {0.0};
  for (int k = threadIdx.x; k < nblk; k += kBlock) v[0] += rec[k];
  block_sum<1, kBlock>(v);
  const int grp = blockIdx.x / (2 * KW), e = blockIdx.x % (2 * KW);
  const int kk = grp * KW + e / 2;
  if (threadIdx.x == 0 && kk < nout) reinterpret_cast<double *>(dots)[2 * kk + e % 2] = v[0];
}

}  // namespace

#define EB_LAUNCH(kernel, grid, block, shmem, st, ...) hipLaunchKernelGGL(kernel, grid, block, shmem, st, __VA_ARGS__)

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

void launch_combine_mfma(double2 *out_base, const SlotList &out_slots, size_t ldo, const double2 *in_base,
                         const SlotList &in_slots, size_t ldi, const double2 *C, double sgn, bool add, size_t N,
                         const double2 *g, int conj_out, double2 *dots, int jtag, const KrylovState *S, double *part,
                         size_t part_cap, hipStream_t st) {
  const int nin = in_slots.n, nout = out_slots.n;
  if (nin < 1 || nout < 1 || N == 0) return;
  const int nin4 = (nin + 3) & ~3;
  // two column tiles per wave when the coefficient block fits in 48 KB of LDS
  const bool two = nout > kTile && size_t(nin4) * 2 * kTile * sizeof(double2) <= 48 * 1024;
  auto go = [&](auto rt_tag, auto tb_tag) {
    constexpr int RT = decltype(rt_tag)::value, TB = decltype(tb_tag)::value;
    constexpr int KW = kTile * TB;
    const int groups = (nout + KW - 1) / KW;
    const size_t ntile = (N + RT * kTile - 1) / (RT * kTile);
    size_t nb = (ntile + 3) / 4;
    size_t cap = (2048 + groups - 1) / groups;
    if (g) {
      const size_t by_space = part_cap / (size_t(groups) * 2 * KW);
      cap = cap < by_space ? cap : by_space;
    }
    nb = nb < cap ? nb : cap;
    if (nb < 1) nb = 1;
    const dim3 grid = dim3(unsigned(nb), unsigned(groups));
    const size_t sh = size_t(nin4) * KW * sizeof(double2);
    if (add)
      EB_LAUNCH((k_combine_mfma<RT, TB, true>), grid, dim3(kBlock), sh, st, out_base, out_slots, ldo, in_base,
                in_slots, ldi, C, sgn, N, g, conj_out, jtag, S, part);
    else
      EB_LAUNCH((k_combine_mfma<RT, TB, false>), grid, dim3(kBlock), sh, st, out_base, out_slots, ldo, in_base,
                in_slots, ldi, C, sgn, N, g, conj_out, jtag, S, part);
    if (g) EB_LAUNCH(k_combine_dots<TB>, dim3(groups * 2 * KW), dim3(kBlock), 0, st, part, int(nb), nout, dots, jtag, S);
  };
  if (two)
    go(std::integral_constant<int, 2>{}, std::integral_constant<int, 2>{});
  else
    go(std::integral_constant<int, 4>{}, std::integral_constant<int, 1>{});
}

}  // namespace ebicg
