// Device dense linear algebra for the window eigenproblems of eigBiCG, run by
// one workgroup of kWinThreads threads (one wavefront): eig(C) of Sec. 1 (end)
// for the m x m window matrices of Alg. BiCG-eigen, with the conventions of
// the host solver (hostla.h): right vectors y_i with ||y_i|| = 1, left
// vectors z_i with z_i^+ C = lambda_i z_i^+ and z_i^+ y_i = 1, sorted by
// |lambda| ascending (ties: imaginary part descending).
//
// Method, as on the host: Householder reduction to Hessenberg form, complex
// single-shift QR with Wilkinson shifts (an exceptional shift every tenth
// sweep) to the Schur form T = Q^+ C Q, and eigenvectors of T by triangular
// substitution, mapped back with Q.  Matrices are column-major with leading
// dimension ld in global memory (the workgroup's own scratch); the Schur
// chase keeps T in LDS when it fits (n <= kWinLdsN).  Every thread of the
// workgroup calls these functions; they synchronise internally.
#pragma once

#include "device_common.h"

namespace ebicg {

constexpr int kWinThreads = 64;  // one wavefront
constexpr int kWinLdsN = 56;     // largest n whose Schur chase runs on an LDS copy of T

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

// Householder reduction A = Q Hs Q^+ (A overwritten by Hs, Q set).  v: scratch of n.
__device__ void win_hessenberg(double2 *A, double2 *Q, int n, int ld, double2 *v) {
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
    for (int i = k + 1 + t; i < n; i += kWinThreads) {
      wcx a = ld2(A + i + k * ld);
      if (i == k + 1) a = a - alpha;
      st2(v + i, a);
      vs += a.x * a.x + a.y * a.y;
    }
    const double vn = sqrt(wsum(vs));
    __syncthreads();
    if (vn == 0.0) continue;
    for (int i = k + 1 + t; i < n; i += kWinThreads) {
      const wcx a = ld2(v + i);
      st2(v + i, wcx{a.x / vn, a.y / vn});
    }
    __syncthreads();
    // A <- (I - 2 v v^+) A, one column per lane
    for (int j = t; j < n; j += kWinThreads) {
      wcx s = {0.0, 0.0};
      for (int i = k + 1; i < n; ++i) cfmac(s, ld2(v + i), ld2(A + i + j * ld));
      s = 2.0 * s;
      for (int i = k + 1; i < n; ++i) st2(A + i + j * ld, ld2(A + i + j * ld) - ld2(v + i) * s);
    }
    __syncthreads();
    // A <- A (I - 2 v v^+), Q <- Q (I - 2 v v^+), one row per lane
    for (int i = t; i < n; i += kWinThreads) {
      wcx s = {0.0, 0.0}, u = {0.0, 0.0};
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
    __syncthreads();
    for (int i = k + 2 + t; i < n; i += kWinThreads) st2(A + i + k * ld, wcx{0.0, 0.0});
    __syncthreads();
  }
}

// Complex Schur form of the Hessenberg T (upper triangular on return), the
// similarity accumulated into Z (A = Z T Z^+).  T is column-major with leading
// dimension ldt (in LDS or global memory).  Returns false if the iteration did
// not converge.  Control decisions are taken by lane 0 and broadcast through
// `ctl` (LDS).
template <typename TP>
__device__ bool win_schur(TP T, int ldt, double2 *Z, int ldz, int n, double *ctl) {
  const int t = threadIdx.x;
  const double eps = 2.220446049250313e-16;
  double anorm = 0.0;
  for (int j = 0; j < n; ++j)
    for (int i = t; i < n; i += kWinThreads) anorm = fmax(anorm, wabs1(ld2(T + i + j * ldt)));
#pragma unroll
  for (int off = kWinThreads / 2; off > 0; off >>= 1) anorm = fmax(anorm, __shfl_xor(anorm, off, kWinThreads));
  if (anorm == 0.0) anorm = 1.0;
  int ihi = n - 1, its = 0, total = 0;
  const int max_total = 100 * (n > 1 ? n : 1);
  bool ok = true;
  while (ihi > 0) {
    // deflation point: every lane reads the same (settled) entries
    int l = 0;
    for (int k = ihi; k >= 1; --k) {
      double tst = wabs1(ld2(T + (k - 1) + (k - 1) * ldt)) + wabs1(ld2(T + k + k * ldt));
      if (tst == 0.0) tst = anorm;
      if (wabs1(ld2(T + k + (k - 1) * ldt)) <= eps * tst) {
        l = k;
        break;
      }
    }
    __syncthreads();
    if (l > 0 && t == 0) st2(T + l + (l - 1) * ldt, wcx{0.0, 0.0});
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
      mu = ld2(T + ihi + ihi * ldt);
      mu.x += fabs(ld2(T + ihi + (ihi - 1) * ldt).x) + (ihi >= 2 ? fabs(ld2(T + (ihi - 1) + (ihi - 2) * ldt).x) : 0.0);
    } else {
      const wcx a = ld2(T + (ihi - 1) + (ihi - 1) * ldt), b = ld2(T + (ihi - 1) + ihi * ldt);
      const wcx c = ld2(T + ihi + (ihi - 1) * ldt), d = ld2(T + ihi + ihi * ldt);
      const wcx hm = 0.5 * (a - d);
      const wcx disc = wsqrt(hm * hm + b * c);
      const wcx avg = 0.5 * (a + d);
      const wcx m1 = avg + disc, m2 = avg - disc;
      mu = wabs(m1 - d) < wabs(m2 - d) ? m1 : m2;
    }
    __syncthreads();
    for (int k = l; k < ihi; ++k) {
      // rotation G = [[c, s], [-conj(s), c]] with G [x; y] = [r; 0], by lane 0
      if (t == 0) {
        wcx x, y;
        if (k == l) {
          x = ld2(T + k + k * ldt) - mu;
          y = ld2(T + (k + 1) + k * ldt);
        } else {
          x = ld2(T + k + (k - 1) * ldt);
          y = ld2(T + (k + 1) + (k - 1) * ldt);
        }
        const double ax = wabs(x), ay = wabs(y);
        double c;
        wcx s;
        if (ay == 0.0) {
          c = 1.0;
          s = {0.0, 0.0};
        } else if (ax == 0.0) {
          c = 0.0;
          s = {y.x / ay, -y.y / ay};
        } else {
          const double r = hypot(ax, ay);
          c = ax / r;
          const wcx xs = {x.x / ax, x.y / ax};
          s = (1.0 / r) * (xs * cconj(y));
        }
        ctl[0] = c;
        ctl[1] = s.x;
        ctl[2] = s.y;
      }
      __syncthreads();
      const double c = ctl[0];
      const wcx s = {ctl[1], ctl[2]};
      const wcx sc = cconj(s);
      const int j0 = k == l ? k : k - 1;
      for (int j = j0 + t; j < n; j += kWinThreads) {
        const wcx a = ld2(T + k + j * ldt), b = ld2(T + (k + 1) + j * ldt);
        st2(T + k + j * ldt, c * a + s * b);
        st2(T + (k + 1) + j * ldt, c * b - sc * a);
      }
      __syncthreads();
      if (k > l && t == 0) st2(T + (k + 1) + (k - 1) * ldt, wcx{0.0, 0.0});
      const int i1 = k + 2 < ihi ? k + 2 : ihi;
      for (int i = t; i <= i1; i += kWinThreads) {
        const wcx a = ld2(T + i + k * ldt), b = ld2(T + i + (k + 1) * ldt);
        st2(T + i + k * ldt, c * a + b * sc);
        st2(T + i + (k + 1) * ldt, c * b - a * s);
      }
      for (int i = t; i < n; i += kWinThreads) {
        const wcx a = ld2(Z + i + k * ldz), b = ld2(Z + i + (k + 1) * ldz);
        st2(Z + i + k * ldz, c * a + b * sc);
        st2(Z + i + (k + 1) * ldz, c * b - a * s);
      }
      __syncthreads();
    }
  }
  __syncthreads();
  for (int j = 0; j < n; ++j)
    for (int i = j + 1 + t; i < n; i += kWinThreads) st2(T + i + j * ldt, wcx{0.0, 0.0});
  __syncthreads();
  return ok;
}

// [y, z, lam] = eig(C) for the n x n matrix C (column-major, leading dimension
// ld, global).  Workspace ws: 4 ld x ld complex plus 4 ld; tlds: LDS space for
// kWinLdsN^2 complex (used when n <= kWinLdsN); ctl: 4 doubles of LDS.
// Outputs y, z: n x n (leading dimension ld), lam: n.  Returns false on a
// QR failure (on every lane).
__device__ bool win_eig(const double2 *C, int n, int ld, double2 *lam, double2 *y, double2 *z, double2 *ws,
                        double2 *tlds, double *ctl) {
  const int t = threadIdx.x;
  double2 *A = ws, *Q = ws + size_t(ld) * ld, *X = ws + 2 * size_t(ld) * ld, *W = ws + 3 * size_t(ld) * ld;
  double2 *v = ws + 4 * size_t(ld) * ld;  // n
  double2 *lm = v + ld;                   // n unsorted eigenvalues
  int *ord = reinterpret_cast<int *>(lm + ld);  // n
  for (int j = 0; j < n; ++j)
    for (int i = t; i < n; i += kWinThreads) A[i + j * ld] = C[i + j * ld];
  __syncthreads();
  if (n == 0) return true;
  win_hessenberg(A, Q, n, ld, v);
  bool ok;
  if (n <= kWinLdsN) {
    for (int j = 0; j < n; ++j)
      for (int i = t; i < n; i += kWinThreads) tlds[i + j * kWinLdsN] = A[i + j * ld];
    __syncthreads();
    ok = win_schur(tlds, kWinLdsN, Q, ld, n, ctl);
    for (int j = 0; j < n; ++j)
      for (int i = t; i < n; i += kWinThreads) A[i + j * ld] = tlds[i + j * kWinLdsN];
    __syncthreads();
  } else {
    ok = win_schur(A, ld, Q, ld, n, ctl);
  }
  if (!ok) return false;
  double tmax = 0.0;
  for (int j = 0; j < n; ++j)
    for (int i = t; i <= j && i < n; i += kWinThreads) tmax = fmax(tmax, wabs(ld2(A + i + j * ld)));
#pragma unroll
  for (int off = kWinThreads / 2; off > 0; off >>= 1) tmax = fmax(tmax, __shfl_xor(tmax, off, kWinThreads));
  const double smin = fmax(2.220446049250313e-16 * tmax, 2.2250738585072014e-308);
  // eigenvectors of T, one per lane: right x (x_k = 1, x_j = 0 for j > k) in
  // column k of X, left w (w_k = 1, w_j = 0 for j < k) in column k of W
  for (int k = t; k < n; k += kWinThreads) {
    const wcx lk = ld2(A + k + k * ld);
    lm[k] = make_double2(lk.x, lk.y);
    double2 *x = X + size_t(k) * ld, *w = W + size_t(k) * ld;
    for (int i = 0; i < n; ++i) {
      x[i] = make_double2(0.0, 0.0);
      w[i] = make_double2(0.0, 0.0);
    }
    x[k] = make_double2(1.0, 0.0);
    for (int i = k - 1; i >= 0; --i) {
      wcx s = {0.0, 0.0};
      for (int j = i + 1; j <= k; ++j) cfma(s, ld2(A + i + j * ld), ld2(x + j));
      wcx d = ld2(A + i + i * ld) - lk;
      if (wabs(d) < smin) d = {smin, 0.0};
      st2(x + i, -wdiv(s, d));
    }
    w[k] = make_double2(1.0, 0.0);
    for (int i = k + 1; i < n; ++i) {
      wcx s = {0.0, 0.0};
      for (int j = k; j < i; ++j) cfmac(s, ld2(A + j + i * ld), ld2(w + j));
      wcx d = cconj(ld2(A + i + i * ld) - lk);
      if (wabs(d) < smin) d = {smin, 0.0};
      st2(w + i, -wdiv(s, d));
    }
  }
  __syncthreads();
  // sort order (lane 0): |lambda| ascending, ties by imaginary part descending
  if (t == 0) {
    for (int i = 0; i < n; ++i) ord[i] = i;
    for (int i = 1; i < n; ++i) {
      const int key = ord[i];
      const wcx lk = ld2(lm + key);
      const double ak = wabs(lk);
      int p = i - 1;
      while (p >= 0) {
        const wcx lp = ld2(lm + ord[p]);
        const double ap = wabs(lp);
        bool after;  // does ord[p] come after key?
        if (fabs(ap - ak) > 1e-12 * fmax(fmax(ap, ak), 1e-300))
          after = ap > ak;
        else if (lp.y != lk.y)
          after = lp.y < lk.y;
        else
          after = ord[p] > key;
        if (!after) break;
        ord[p + 1] = ord[p];
        --p;
      }
      ord[p + 1] = key;
    }
  }
  __syncthreads();
  // back to the original basis: y = Q x, z = Q w, normalised; one output column per lane
  for (int c = t; c < n; c += kWinThreads) {
    const int k = ord[c];
    lam[c] = lm[k];
    const double2 *x = X + size_t(k) * ld, *w = W + size_t(k) * ld;
    double yn = 0.0;
    for (int i = 0; i < n; ++i) {
      wcx sy = {0.0, 0.0}, sz = {0.0, 0.0};
      for (int j = 0; j <= k; ++j) cfma(sy, ld2(Q + i + j * ld), ld2(x + j));
      for (int j = k; j < n; ++j) cfma(sz, ld2(Q + i + j * ld), ld2(w + j));
      st2(y + i + c * ld, sy);
      st2(z + i + c * ld, sz);
      yn += sy.x * sy.x + sy.y * sy.y;
    }
    yn = sqrt(yn);
    wcx d = {0.0, 0.0};
    for (int i = 0; i < n; ++i) {
      const wcx yi = (1.0 / yn) * ld2(y + i + c * ld);
      st2(y + i + c * ld, yi);
      cfmac(d, ld2(z + i + c * ld), yi);
    }
    const wcx dc = cconj(d);
    for (int i = 0; i < n; ++i) st2(z + i + c * ld, wdiv(ld2(z + i + c * ld), dc));
  }
  __syncthreads();
  return true;
}

}  // namespace ebicg
