// Device dense linear algebra for the window eigenproblems of eigBiCG, run by
// one workgroup of kWinThreads threads (one wavefront): eig(C) of Sec. 1 (end)
// for the m x m window matrices of Alg. BiCG-eigen, with the conventions of
// the host solver (hostla.h): right vectors y_i with ||y_i|| = 1, left
// vectors z_i with z_i^+ C = lambda_i z_i^+ and z_i^+ y_i = 1, sorted by a
// criterion (|lambda| ascending by default; ties: imaginary part descending).
//
// Method, as on the host: Householder reduction to Hessenberg form, complex
// single-shift QR with Wilkinson shifts (an exceptional shift every tenth
// sweep) to the Schur form T = Q^+ C Q, and eigenvectors of T by triangular
// substitution, mapped back with Q.  Every step is a chain of small dependent
// updates, so latency decides the time: the working matrices (T, Q and the
// right and left eigenvectors of T) live in a 150 KB LDS pool when it holds
// all four (n <= 48), or T and Q alone (n <= 69); the rest go to the
// workgroup's global scratch.  In LDS
// the leading dimension is odd, so that the lanes of a row-wise sweep (one
// column per lane) fall in different banks.  Every lane computes each Givens
// rotation of the QR chase itself from the same entries, with no broadcast.
// Every thread of the workgroup calls these functions; they synchronise
// internally.
#pragma once

#include "device_common.h"

namespace ebicg {

constexpr int kWinThreads = 64;      // one wavefront
constexpr int kWinMaxN = 128;        // largest matrix
constexpr int kWinLdsEntries = 9600;  // complex entries of the LDS matrix pool (150 KB)

// The workgroup's LDS: the matrix pool and three vectors of kWinMaxN.  One
// variable at namespace scope, so that every access compiles to an LDS
// instruction (a pointer handed through a call would be a generic one).
struct WinLds {
  double2 pool[kWinLdsEntries];
  double2 vec[kWinMaxN];  // Householder vector
  double2 lm[kWinMaxN];   // unsorted eigenvalues
  int ord[kWinMaxN];      // sort order
};
namespace {
__shared__ WinLds win_lds;
}

using wcx = cx<double>;

__device__ __forceinline__ double wabs(wcx a) { return hypot(a.x, a.y); }
__device__ __forceinline__ double wabs1(wcx a) { return fabs(a.x) + fabs(a.y); }
__device__ __forceinline__ wcx wdiv(wcx a, wcx b) {
  // Smith's division
  if (fabs(b.x) >= fabs(b.y)) {
    const double r = b.y / b.x, d = b.x + b.y * r;
    return {(a.x + a.y * r) / d, (a.y - a.x * r) / d};
  }
  const double r = b.x / b.y, d = b.y + b.x * r;
  return {(a.x * r + a.y) / d, (a.y * r - a.x) / d};
}
__device__ __forceinline__ wcx wsqrt(wcx z) {
  const double m = wabs(z);
  if (m == 0.0) return {0.0, 0.0};
  const double re = sqrt(0.5 * (m + z.x));
  const double im = sqrt(0.5 * (m - z.x));
  return {re, z.y < 0.0 ? -im : im};
}
__device__ __forceinline__ wcx ld2(const double2 *p) {
  const double2 v = *p;
  return {v.x, v.y};
}
__device__ __forceinline__ void st2(double2 *p, wcx v) { *p = make_double2(v.x, v.y); }

// Sum over the workgroup (one wavefront); every lane gets the total.
__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int off = kWinThreads / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWinThreads);
  return v;
}

// Householder reduction A = Q Hs Q^+ (A overwritten by Hs, Q set); leading
// dimension ld for both.  v: scratch of n.
__device__ __forceinline__ void win_hessenberg(double2 *A, double2 *Q, int n, int ld, double2 *v) {
  const int t = threadIdx.x;
  for (int j = 0; j < n; ++j)
    for (int i = t; i < n; i += kWinThreads) Q[i + j * ld] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  __syncthreads();
  for (int k = 0; k + 2 < n; ++k) {
    double xs = 0.0;
    for (int i = k + 1 + t; i < n; i += kWinThreads) {
      const wcx a = ld2(A + i + k * ld);
      xs += a.x * a.x + a.y * a.y;
    }
    const double xn = sqrt(wsum(xs));
    if (xn == 0.0) continue;
    const wcx x0 = ld2(A + (k + 1) + k * ld);
    const double ax0 = wabs(x0);
    const wcx ph = ax0 == 0.0 ? wcx{1.0, 0.0} : wcx{x0.x / ax0, x0.y / ax0};
    const wcx alpha = {-ph.x * xn, -ph.y * xn};
    double vs = 0.0;
    wcx vi[2];  // this lane's entries of v (n <= 128)
    for (int r = 0; r < 2; ++r) {
      const int i = k + 1 + t + r * kWinThreads;
      vi[r] = {0.0, 0.0};
      if (i < n) {
        wcx a = ld2(A + i + k * ld);
        if (i == k + 1) a = a - alpha;
        vi[r] = a;
        vs += a.x * a.x + a.y * a.y;
      }
    }
    const double vn = sqrt(wsum(vs));
    if (vn == 0.0) continue;
    for (int r = 0; r < 2; ++r) {
      const int i = k + 1 + t + r * kWinThreads;
      if (i < n) st2(v + i, wcx{vi[r].x / vn, vi[r].y / vn});
    }
    __syncthreads();
    // A <- (I - 2 v v^+) A, one column per lane
    for (int j = t; j < n; j += kWinThreads) {
      wcx s = {0.0, 0.0};
#pragma unroll 4
      for (int i = k + 1; i < n; ++i) cfmac(s, ld2(v + i), ld2(A + i + j * ld));
      s = 2.0 * s;
      for (int i = k + 1; i < n; ++i) st2(A + i + j * ld, ld2(A + i + j * ld) - ld2(v + i) * s);
    }
    __syncthreads();
    // A <- A (I - 2 v v^+), Q <- Q (I - 2 v v^+), one row per lane
    for (int i = t; i < n; i += kWinThreads) {
      wcx s = {0.0, 0.0}, u = {0.0, 0.0};
#pragma unroll 4
      for (int j = k + 1; j < n; ++j) {
        const wcx vj = ld2(v + j);
        cfma(s, ld2(A + i + j * ld), vj);
        cfma(u, ld2(Q + i + j * ld), vj);
      }
      s = 2.0 * s;
      u = 2.0 * u;
      for (int j = k + 1; j < n; ++j) {
        const wcx vc = cconj(ld2(v + j));
        st2(A + i + j * ld, ld2(A + i + j * ld) - s * vc);
        st2(Q + i + j * ld, ld2(Q + i + j * ld) - u * vc);
      }
    }
    for (int i = k + 2 + t; i < n; i += kWinThreads) st2(A + i + k * ld, wcx{0.0, 0.0});
    __syncthreads();
  }
}

// Givens rotation G = [[c, s], [-conj(s), c]] with G [x; y] = [r; 0]:
// c = |x| / r, s = (x / |x|) conj(y) / r, r = sqrt(|x|^2 + |y|^2).  The
// rotation lies on the serial path of the QR chase, so it is formed from the
// squares of the entries (two square roots and one reciprocal, no hypot);
// entries whose squares would leave the FP64 range are first scaled by the
// largest component.  Every lane takes the same branch.
__device__ __forceinline__ void win_givens(wcx x, wcx y, double &c, wcx &s) {
  double ax2 = x.x * x.x + x.y * x.y, ay2 = y.x * y.x + y.y * y.y;
  const double r2 = ax2 + ay2;
  if (!(r2 > 1e-280 && r2 < 1e280)) {  // rare: rescale (or y = 0 among tiny entries)
    const double sc = fmax(fmax(fabs(x.x), fabs(x.y)), fmax(fabs(y.x), fabs(y.y)));
    if (sc == 0.0) {
      c = 1.0;
      s = {0.0, 0.0};
      return;
    }
    const double is = 1.0 / sc;
    x = is * x;
    y = is * y;
    ax2 = x.x * x.x + x.y * x.y;
    ay2 = y.x * y.x + y.y * y.y;
  }
  if (ay2 == 0.0) {
    c = 1.0;
    s = {0.0, 0.0};
    return;
  }
  if (ax2 == 0.0) {
    const double iay = 1.0 / sqrt(ay2);
    c = 0.0;
    s = {y.x * iay, -y.y * iay};
    return;
  }
  const double ax = sqrt(ax2), r = sqrt(ax2 + ay2);
  const double inv = 1.0 / (ax * r);
  c = ax2 * inv;
  s = inv * (x * cconj(y));
}

// Lane l's value of v (l uniform across the wave).
__device__ __forceinline__ double win_readlane(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(int(b), lane), hi = __builtin_amdgcn_readlane(int(b >> 32), lane);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}
__device__ __forceinline__ wcx win_readlane(wcx v, int lane) { return {win_readlane(v.x, lane), win_readlane(v.y, lane)}; }

// 1 / sqrt(v) for v in [1e-280, 1e280]: the hardware estimate and two Newton
// steps r <- r (3/2 - v r^2 / 2).
__device__ __forceinline__ double win_rsq(double v) {
  double r = __builtin_amdgcn_rsq(v);
  const double h = 0.5 * v;
  r = r * fma(-h * r, r, 1.5);
  r = r * fma(-h * r, r, 1.5);
  return r;
}

// The rotation of win_givens on the serial path of the QR chase: where |x|^2
// and r^2 lie in [1e-150, 1e150] (every step but the rarest), c = |x|^2 q and
// s = x conj(y) q with q = 1 / (|x| r) from one reciprocal square root of
// |x|^2 r^2 (y = 0 gives c = 1, s = 0); elsewhere win_givens itself.
__device__ __forceinline__ void win_givens_fast(wcx x, wcx y, double &c, wcx &s) {
  const double ax2 = x.x * x.x + x.y * x.y, ay2 = y.x * y.x + y.y * y.y;
  const double r2 = ax2 + ay2;
  if (ax2 > 1e-150 && r2 < 1e150) {
    const double q = win_rsq(ax2 * r2);
    c = ax2 * q;
    s = q * (x * cconj(y));
    return;
  }
  win_givens(x, y, c, s);
}

// One implicit single-shift QR sweep over the active block l..ihi of the
// Hessenberg T (n <= kWinThreads), with the same rotations applied to the
// same entries in the same order as the entry-by-entry chase, but with the
// serial path cut to the rotation and a few products.  The 2 x 2 block of
// rows and columns k, k+1 at step k is held by every lane (uniform values),
// so the next rotation follows from it without a round trip through LDS or
// across lanes.  Lane j > k+1 owns column j and carries in a register the
// entry of its column in the row that the next row rotation mixes; the row
// below is original (untouched by earlier steps) and read one step ahead.
// The column rotations of the entries above the block (rows < k) and of Z
// commute with the rest of the chase and are applied after it, one row per
// lane, from the rotations kept in LDS.
__device__ __forceinline__ void win_sweep_lanes(double2 *T, double2 *Z, int n, int ld, int l, int ihi, wcx mu) {
  const int j = threadIdx.x;
  const bool own = j < n;
  // uniform: ua0 = T(k,k), ua1 = T(k,k+1), ub0 = T(k+1,k), ub1 = T(k+1,k+1), current
  wcx ua0 = ld2(T + l + l * ld), ua1 = ld2(T + l + (l + 1) * ld);
  wcx ub0 = ld2(T + (l + 1) + l * ld), ub1 = ld2(T + (l + 1) + (l + 1) * ld);
  wcx cur = {0.0, 0.0}, bnx = {0.0, 0.0};  // lane j > k+1: T(k, j) current, T(k+1, j) original
  if (own && j >= l + 2) {
    cur = ld2(T + l + j * ld);
    bnx = ld2(T + (l + 1) + j * ld);
  }
  wcx x = ua0 - mu, y = ub0;
  double rc = 1.0;  // this lane's rotation of the sweep (lane i: rotation l + i)
  wcx rs = {0.0, 0.0};
  for (int k = l; k < ihi; ++k) {
    const bool more = k + 2 <= ihi;
    // original entries of row k+2 (F = T(k+2,k+1), G = T(k+2,k+2), lanes: T(k+2, j))
    wcx F = {0.0, 0.0}, G = {0.0, 0.0}, bn2 = {0.0, 0.0};
    if (more) {
      F = ld2(T + (k + 2) + (k + 1) * ld);
      G = ld2(T + (k + 2) + (k + 2) * ld);
    }
    if (own && k + 2 < n) bn2 = ld2(T + (k + 2) + j * ld);
    double c;
    wcx s;
    win_givens_fast(x, y, c, s);
    const wcx sc = cconj(s);
    // row rotation k: the 2 x 2 block (every lane) and the far columns (own lane)
    const wcx A = c * ua0 + s * ub0, C = c * ub0 - sc * ua0;
    const wcx B = c * ua1 + s * ub1, D = c * ub1 - sc * ua1;
    if (own && j >= k + 2) {
      const wcx top = c * cur + s * bnx;
      cur = c * bnx - sc * cur;
      st2(T + k + j * ld, top);
    }
    // column rotation k on rows k, k+1 and k+2 of columns k, k+1
    const wcx xn = c * C + D * sc, dn = c * D - C * s;
    if (j == k - l) {  // rotation k - l of the sweep, kept by lane k - l
      rc = c;
      rs = s;
    }
    if (j == 0) {
      if (k > l) {  // the bulge column k-1: T(k,k-1) final, T(k+1,k-1) = 0
        st2(T + k + (k - 1) * ld, c * x + s * y);
        st2(T + (k + 1) + (k - 1) * ld, wcx{0.0, 0.0});
      }
      st2(T + k + k * ld, c * A + B * sc);
      st2(T + k + (k + 1) * ld, c * B - A * s);
    }
    x = xn;
    ua0 = dn;
    if (more) {
      y = F * sc;
      ub0 = c * F;
      ub1 = G;
      ua1 = win_readlane(cur, k + 2);  // T(k+1, k+2) after this row rotation
    }
    bnx = bn2;
  }
  if (j == 0) {
    st2(T + ihi + (ihi - 1) * ld, x);
    st2(T + ihi + ihi * ld, ua0);
  }
  if (own && j > ihi) st2(T + ihi + j * ld, cur);
  __syncthreads();
  // deferred column rotations: rows i < k of columns k, k+1 for every k (T),
  // and every row of Z.  The rotations come from the lanes that kept them
  // (readlane); the row entries are read four steps at a time ahead of use
  // (each is the value from before the pass: step k reads column k + 1 and
  // writes column k).
  const int k0 = l > j + 1 ? l : j + 1;
  const bool tdo = j <= ihi && k0 < ihi;
  if (own) {
    wcx tc = tdo ? ld2(T + j + k0 * ld) : wcx{0.0, 0.0};
    wcx zc = ld2(Z + j + l * ld);
    for (int kb = l; kb < ihi; kb += 4) {
      wcx zb[4], tb[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = kb + u;
        zb[u] = tb[u] = wcx{0.0, 0.0};
        if (k < ihi) {
          zb[u] = ld2(Z + j + (k + 1) * ld);
          if (tdo && k >= k0) tb[u] = ld2(T + j + (k + 1) * ld);
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = kb + u;
        if (k < ihi) {
          const double c = win_readlane(rc, k - l);
          const wcx s = win_readlane(rs, k - l), sc = cconj(s);
          st2(Z + j + k * ld, c * zc + zb[u] * sc);
          zc = c * zb[u] - zc * s;
          if (tdo && k >= k0) {
            st2(T + j + k * ld, c * tc + tb[u] * sc);
            tc = c * tb[u] - tc * s;
          }
        }
      }
    }
    st2(Z + j + ihi * ld, zc);
    if (tdo) st2(T + j + ihi * ld, tc);
  }
  __syncthreads();
}

// Complex Schur form of the Hessenberg T (upper triangular on return), the
// similarity accumulated into Z (A = Z T Z^+); leading dimension ld for both.
// Returns false if the iteration did not converge.  Every lane takes the
// same decisions from the same (settled) entries.
__device__ __forceinline__ bool win_schur(double2 *T, double2 *Z, int n, int ld) {
  const int t = threadIdx.x;
  const double eps = 2.220446049250313e-16;
  double anorm = 0.0;
  for (int j = 0; j < n; ++j)
    for (int i = t; i < n; i += kWinThreads) anorm = fmax(anorm, wabs1(ld2(T + i + j * ld)));
#pragma unroll
  for (int off = kWinThreads / 2; off > 0; off >>= 1) anorm = fmax(anorm, __shfl_xor(anorm, off, kWinThreads));
  if (anorm == 0.0) anorm = 1.0;
  int ihi = n - 1, its = 0, total = 0;
  const int max_total = 100 * (n > 1 ? n : 1);
  bool ok = true;
  while (ihi > 0) {
    // deflation point: the largest k <= ihi with a negligible T(k, k-1), one
    // k per lane and a ballot per 64 of them
    int l = 0;
    for (int base = 0; base < ihi; base += kWinThreads) {
      const int k = base + 1 + t;
      bool small = false;
      if (k <= ihi) {
        double tst = wabs1(ld2(T + (k - 1) + (k - 1) * ld)) + wabs1(ld2(T + k + k * ld));
        if (tst == 0.0) tst = anorm;
        small = wabs1(ld2(T + k + (k - 1) * ld)) <= eps * tst;
      }
      const unsigned long long mask = __ballot(small);
      if (mask) l = base + 1 + (63 - __clzll(mask));
    }
    __syncthreads();
    if (l > 0 && t == 0) st2(T + l + (l - 1) * ld, wcx{0.0, 0.0});
    __syncthreads();
    if (l == ihi) {
      --ihi;
      its = 0;
      continue;
    }
    if (++total > max_total) {
      ok = false;
      break;
    }
    ++its;
    wcx mu;
    if (its % 10 == 0) {
      mu = ld2(T + ihi + ihi * ld);
      mu.x += fabs(ld2(T + ihi + (ihi - 1) * ld).x) + (ihi >= 2 ? fabs(ld2(T + (ihi - 1) + (ihi - 2) * ld).x) : 0.0);
    } else {
      const wcx a = ld2(T + (ihi - 1) + (ihi - 1) * ld), b = ld2(T + (ihi - 1) + ihi * ld);
      const wcx c = ld2(T + ihi + (ihi - 1) * ld), d = ld2(T + ihi + ihi * ld);
      const wcx hm = 0.5 * (a - d);
      const wcx disc = wsqrt(hm * hm + b * c);
      const wcx avg = 0.5 * (a + d);
      const wcx m1 = avg + disc, m2 = avg - disc;
      mu = wabs(m1 - d) < wabs(m2 - d) ? m1 : m2;
    }
    if (n <= kWinThreads) {
      win_sweep_lanes(T, Z, n, ld, l, ihi, mu);
      continue;
    }
    for (int k = l; k < ihi; ++k) {
      double c;
      wcx s;
      {
        const int col = k == l ? k : k - 1;  // the first rotation makes the bulge
        wcx x = ld2(T + k + col * ld);
        if (k == l) x = x - mu;
        win_givens(x, ld2(T + (k + 1) + col * ld), c, s);
      }
      const wcx sc = cconj(s);
      // rows k, k+1 (every lane has read the entries above: nobody writes them before the barrier)
      __syncthreads();
      const int j0 = k == l ? k : k - 1;
      for (int j = j0 + t; j < n; j += kWinThreads) {
        const wcx a = ld2(T + k + j * ld), b = ld2(T + (k + 1) + j * ld);
        st2(T + k + j * ld, c * a + s * b);
        st2(T + (k + 1) + j * ld, c * b - sc * a);
      }
      __syncthreads();
      if (k > l && t == 0) st2(T + (k + 1) + (k - 1) * ld, wcx{0.0, 0.0});
      // columns k, k+1 of T and of Z
      const int i1 = k + 2 < ihi ? k + 2 : ihi;
      for (int i = t; i <= i1; i += kWinThreads) {
        const wcx a = ld2(T + i + k * ld), b = ld2(T + i + (k + 1) * ld);
        st2(T + i + k * ld, c * a + b * sc);
        st2(T + i + (k + 1) * ld, c * b - a * s);
      }
      for (int i = t; i < n; i += kWinThreads) {
        const wcx a = ld2(Z + i + k * ld), b = ld2(Z + i + (k + 1) * ld);
        st2(Z + i + k * ld, c * a + b * sc);
        st2(Z + i + (k + 1) * ld, c * b - a * s);
      }
      __syncthreads();
    }
  }
  __syncthreads();
  for (int j = 0; j < n; ++j)
    for (int i = j + 1 + t; i < n; i += kWinThreads) st2(T + i + j * ld, wcx{0.0, 0.0});
  __syncthreads();
  return ok;
}

// [y, z, lam] = eig(C) with the first PL of T, Q, X, W in the LDS pool and
// the rest in ws (leading dimension n | 1 for all four).
template <int PL>
__device__ __attribute__((noinline)) bool win_eig_pl(const double2 *C, int n, int ld, double2 *lam, double2 *y,
                                                     double2 *z, double2 *ws, int which) {
  // the same on every lane: scalar registers, uniform loops and branches
  n = __builtin_amdgcn_readfirstlane(n);
  ld = __builtin_amdgcn_readfirstlane(ld);
  which = __builtin_amdgcn_readfirstlane(which);
  const int t = threadIdx.x;
  const int lw = n | 1;  // odd leading dimension
  const size_t nn = size_t(lw) * n;
  double2 *A, *Q, *X, *W;
  if constexpr (PL >= 1) A = win_lds.pool; else A = ws;
  if constexpr (PL >= 2) Q = win_lds.pool + nn; else Q = ws + nn;
  if constexpr (PL >= 3) X = win_lds.pool + 2 * nn; else X = ws + 2 * nn;
  if constexpr (PL >= 4) W = win_lds.pool + 3 * nn; else W = ws + 3 * nn;
  double2 *lm = win_lds.lm;
  int *ord = win_lds.ord;
  for (int j = 0; j < n; ++j)
    for (int i = t; i < n; i += kWinThreads) A[i + j * lw] = C[i + j * ld];
  __syncthreads();
  win_hessenberg(A, Q, n, lw, win_lds.vec);
  if (!win_schur(A, Q, n, lw)) return false;
  double tmax = 0.0;
  for (int j = 0; j < n; ++j)
    for (int i = t; i <= j && i < n; i += kWinThreads) tmax = fmax(tmax, wabs(ld2(A + i + j * lw)));
#pragma unroll
  for (int off = kWinThreads / 2; off > 0; off >>= 1) tmax = fmax(tmax, __shfl_xor(tmax, off, kWinThreads));
  const double smin = fmax(2.220446049250313e-16 * tmax, 2.2250738585072014e-308);
  // eigenvectors of T, one per lane: right x (x_k = 1, x_j = 0 for j > k) in
  // column k of X, left w (w_k = 1, w_j = 0 for j < k) in column k of W
  for (int k = t; k < n; k += kWinThreads) {
    const wcx lk = ld2(A + k + k * lw);
    lm[k] = make_double2(lk.x, lk.y);
    double2 *x = X + size_t(k) * lw, *w = W + size_t(k) * lw;
    x[k] = make_double2(1.0, 0.0);
    for (int i = k - 1; i >= 0; --i) {
      wcx s = {0.0, 0.0};
#pragma unroll 4
      for (int j = i + 1; j <= k; ++j) cfma(s, ld2(A + i + j * lw), ld2(x + j));
      wcx d = ld2(A + i + i * lw) - lk;
      if (wabs(d) < smin) d = {smin, 0.0};
      st2(x + i, -wdiv(s, d));
    }
    w[k] = make_double2(1.0, 0.0);
    for (int i = k + 1; i < n; ++i) {
      wcx s = {0.0, 0.0};
#pragma unroll 4
      for (int j = k; j < i; ++j) cfmac(s, ld2(A + j + i * lw), ld2(w + j));
      wcx d = cconj(ld2(A + i + i * lw) - lk);
      if (wabs(d) < smin) d = {smin, 0.0};
      st2(w + i, -wdiv(s, d));
    }
  }
  __syncthreads();
  // sort order: the criterion's key ascending, ties (to 1e-12 of the larger
  // modulus) by imaginary part descending, then by index; an insertion sort
  // (the order the host solver produces, also where near-ties make the
  // comparison intransitive).  Does entry (kp, mp, ip, op) come after (kk, mk, ik, ok)?
  auto after = [](double kp, double mp, double ip, int op, double kk, double mk, double ik, int ok) {
    if (fabs(kp - kk) > 1e-12 * fmax(fmax(mp, mk), 1e-300)) return kp > kk;
    if (ip != ik) return ip < ik;
    return op > ok;
  };
  if (n <= kWinThreads) {
    // lane p holds sorted position p; each insertion finds its place with a
    // ballot (the highest p whose entry does not come after the new one, as
    // the scan from the right stops there) and shifts the tail up one lane
    double key = 0.0, mod = 0.0, im = 0.0;
    if (t < n) {
      const wcx li = ld2(lm + t);
      mod = wabs(li);
      key = which == 1 ? li.x : (which == 2 ? -mod : mod);
      im = li.y;
    }
    double sk = key, sm = mod, si = im;
    int so = t;
    for (int i = 1; i < n; ++i) {
      const double kk = win_readlane(key, i), mk = win_readlane(mod, i), ik = win_readlane(im, i);
      const bool stay = t < i && !after(sk, sm, si, so, kk, mk, ik, i);
      const unsigned long long m = __ballot(stay);
      const int pos = m ? 64 - __clzll(m) : 0;
      const double uk = __shfl_up(sk, 1), um = __shfl_up(sm, 1), ui = __shfl_up(si, 1);
      const int uo = __shfl_up(so, 1);
      if (t == pos) {
        sk = kk;
        sm = mk;
        si = ik;
        so = i;
      } else if (t > pos && t <= i) {
        sk = uk;
        sm = um;
        si = ui;
        so = uo;
      }
    }
    if (t < n) ord[t] = so;
  } else {
    // keys and moduli first, one value per lane (vec is free here); lane 0 sorts
    for (int i = t; i < n; i += kWinThreads) {
      const wcx li = ld2(lm + i);
      const double a = wabs(li);
      win_lds.vec[i] = make_double2(which == 1 ? li.x : (which == 2 ? -a : a), a);
    }
    __syncthreads();
    if (t == 0) {
      const double2 *km = win_lds.vec;
      for (int i = 0; i < n; ++i) ord[i] = i;
      for (int i = 1; i < n; ++i) {
        const int key = ord[i];
        const double2 kk = km[key];
        const double lky = lm[key].y;
        int p = i - 1;
        while (p >= 0) {
          const int op = ord[p];
          const double2 kp = km[op];
          if (!after(kp.x, kp.y, lm[op].y, op, kk.x, kk.y, lky, key)) break;
          ord[p + 1] = op;
          --p;
        }
        ord[p + 1] = key;
      }
    }
  }
  __syncthreads();
  // back to the original basis: y = Q x, z = Q w, one output column per lane;
  // a first pass for ||y|| and z^+ y, a second that writes the normalised
  // vectors (||y|| = 1, z^+ y = 1)
  for (int c = t; c < n; c += kWinThreads) {
    const int k = ord[c];
    lam[c] = lm[k];
    const double2 *x = X + size_t(k) * lw, *w = W + size_t(k) * lw;
    double yn = 0.0;
    wcx d = {0.0, 0.0};
    for (int i = 0; i < n; ++i) {
      wcx sy = {0.0, 0.0}, sz = {0.0, 0.0};
#pragma unroll 4
      for (int j = 0; j <= k; ++j) cfma(sy, ld2(Q + i + j * lw), ld2(x + j));
#pragma unroll 4
      for (int j = k; j < n; ++j) cfma(sz, ld2(Q + i + j * lw), ld2(w + j));
      yn += sy.x * sy.x + sy.y * sy.y;
      cfmac(d, sz, sy);
    }
    yn = sqrt(yn);
    const double inv = 1.0 / yn;
    const wcx dc = cconj(inv * d);  // conj(z^+ y) after y is scaled by 1 / ||y||
    for (int i = 0; i < n; ++i) {
      wcx sy = {0.0, 0.0}, sz = {0.0, 0.0};
#pragma unroll 4
      for (int j = 0; j <= k; ++j) cfma(sy, ld2(Q + i + j * lw), ld2(x + j));
#pragma unroll 4
      for (int j = k; j < n; ++j) cfma(sz, ld2(Q + i + j * lw), ld2(w + j));
      st2(y + i + c * ld, inv * sy);
      st2(z + i + c * ld, wdiv(sz, dc));
    }
  }
  __syncthreads();
  return true;
}

// [y, z, lam] = eig(C) for the n x n matrix C (column-major, leading dimension
// ld, global; 1 <= n <= kWinMaxN).  Workspace ws (global):
// window_eig_ws_entries(n) complex, for the matrices the LDS pool does not
// hold (all four fit up to n = 48, T and Q up to n = 69).  Outputs y, z: n x n
// (leading dimension ld), lam: n, in the order of the criterion which (0
// |lambda| ascending, 1 real part ascending, 2 |lambda| descending).  Returns
// false on a QR failure (on every lane).
__device__ bool win_eig(const double2 *C, int n, int ld, double2 *lam, double2 *y, double2 *z, double2 *ws,
                        int which) {
  if (n <= 0) return true;
  const size_t nn = size_t(n | 1) * n;
  if (4 * nn <= size_t(kWinLdsEntries)) return win_eig_pl<4>(C, n, ld, lam, y, z, ws, which);
  if (2 * nn <= size_t(kWinLdsEntries)) return win_eig_pl<2>(C, n, ld, lam, y, z, ws, which);
  return win_eig_pl<0>(C, n, ld, lam, y, z, ws, which);
}

}  // namespace ebicg
