// The window eigenproblems of eigBiCG on the device (one workgroup): eig(C)
// with the conventions of Sec. 1 (end), and Alg. BiCG-eigen's restart
// coefficients built from the device-resident BiCG scalars (winla.h).
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "kernels.h"
#include "winla.h"

namespace ebicg {
namespace {

__host__ __device__ constexpr size_t window_eig_ws_entries_dev(int n) { return 4 * size_t(n) * n + 3 * size_t(n) + 8; }

__global__ void __launch_bounds__(kWinThreads)
    k_small_eig(const double2 *C, int n, double2 *lam, double2 *y, double2 *z, double2 *ws, int *status) {
  __shared__ double2 tlds[kWinLdsN * kWinLdsN];
  __shared__ double ctl[4];
  const bool ok = win_eig(C, n, n, lam, y, z, ws, tlds, ctl);
  if (threadIdx.x == 0) *status = ok ? 1 : 0;
}

// The window matrix H^(n) of the columns `cols` (Alg. eigBiCG, the H updates
// from alpha, beta, ||r||, rho; the arrow row and column of the first
// residual after a Ritz block from the raw dots of the last restart), the
// column scales eta, zeta of the stored residuals (v = eta r, w = zeta rhat).
__device__ void win_build_H(double2 *H, int ld, const WinCols &cols, const KrylovHistory &h,
                            const double2 *lam_prev, const double2 *dV, const double2 *dW, double2 *eta,
                            double2 *zeta) {
  const int n = cols.n, t = threadIdx.x;
  for (int j = 0; j < n; ++j)
    for (int i = t; i < n; i += kWinThreads) H[i + j * ld] = make_double2(0.0, 0.0);
  __syncthreads();
  for (int c = t; c < n; c += kWinThreads) {
    if (cols.ritz[c]) {
      H[c + c * ld] = lam_prev[cols.idx[c]];
      eta[c] = zeta[c] = make_double2(1.0, 0.0);
      continue;
    }
    const int i = cols.idx[c];
    const wcx a = ld2(h.alpha + i);
    wcx d = wdiv(wcx{1.0, 0.0}, a);
    if (i >= 1) d = d + wdiv(ld2(h.beta + i - 1), ld2(h.alpha + i - 1));
    st2(H + c + c * ld, d);
    const double rn = h.rn[i];
    eta[c] = make_double2(1.0 / rn, 0.0);
    st2(zeta + c, wdiv(wcx{rn, 0.0}, cconj(ld2(h.rho + i))));
    if (c + 1 < n && !cols.ritz[c + 1]) {
      const wcx be = ld2(h.beta + i);
      const double rn1 = h.rn[i + 1];
      st2(H + c + (c + 1) * ld, -((rn / rn1) * wdiv(be, a)));
      st2(H + (c + 1) + c * ld, -wdiv(wcx{rn1 / rn, 0.0}, a));
    }
    if (c > 0 && cols.ritz[c - 1]) {
      const wcx rho = ld2(h.rho + i);
      const wcx f = wdiv(wcx{rn, 0.0}, rho);
      for (int k = 0; k < c; ++k) {
        const int rk = cols.idx[k];
        st2(H + c + k * ld, f * ld2(dV + rk));
        st2(H + k + c * ld, (1.0 / rn) * ld2(dW + rk));
      }
    }
  }
  __syncthreads();
}

// Alg. BiCG-eigen (mode 0) or the final extraction of Alg. eigBiCG (mode 1)
// on the device.  Mode 0: [y, z] = eig(H^(m)), [y', z'] = eig(H^(m-1)) with a
// zero appended, the 2 nev coefficient vectors biorthogonalised (two-sided
// Gram-Schmidt, twice; a pair with pivot below 1e-12 |y||z| is dropped),
// T = Zt^+ H Yt, [u, q, Lambda] = eig(T), CV = Yt u, CW = Zt q with
// ||CV_k|| = 1, CW_k^+ CV_k = 1, written with the stored residuals' scales
// folded in (cV = diag(eta) CV, cW = diag(zeta) CW), columns >= kept zero,
// lam_out = Lambda, *kept_out = kept.  Mode 1: eig(H^(vs)), the first
// min(nev, vs) pairs, cV = diag(eta) y, cW = diag(zeta) z.  Coefficient blocks
// are n x kout column-major (kout = 2 nev in mode 0, min(nev, n) in mode 1).
__global__ void __launch_bounds__(kWinThreads)
    k_window_eig(WinCols cols, int nev, int mode, KrylovHistory h, const double2 *lam_prev, const double2 *dots_prev,
                 double2 *cV, double2 *cW, double2 *lam_out, int *kept_out, double2 *ws, int jtag,
                 const KrylovState *S) {
  if (S && S->stopped && jtag > S->stop_at) {  // the restart's iteration did not run
    if (threadIdx.x == 0) *kept_out = -2;
    return;
  }
  __shared__ double2 tlds[kWinLdsN * kWinLdsN];
  __shared__ double ctl[4];
  const int n = cols.n, t = threadIdx.x, ld = n;
  const int nn = n * n;
  double2 *H = ws, *eta = H + nn, *zeta = eta + n, *y1 = zeta + n, *z1 = y1 + nn, *lam1 = z1 + nn;
  double2 *ews = lam1 + n;  // eig workspace
  double2 *after_ews = ews + window_eig_ws_entries_dev(n);
  win_build_H(H, ld, cols, h, lam_prev, dots_prev, dots_prev + 2 * nev, eta, zeta);
  if (mode == 1) {
    const bool ok = win_eig(H, n, ld, lam1, y1, z1, ews, tlds, ctl);
    const int k = nev < n ? nev : n;
    for (int c = 0; c < k; ++c)
      for (int i = t; i < n; i += kWinThreads) {
        st2(cV + i + c * n, ld2(eta + i) * ld2(y1 + i + c * ld));
        st2(cW + i + c * n, ld2(zeta + i) * ld2(z1 + i + c * ld));
      }
    for (int c = t; c < k; c += kWinThreads) lam_out[c] = lam1[c];
    if (t == 0) *kept_out = ok ? k : -1;
    return;
  }
  const int m = n, k2 = 2 * nev;
  // eig(H^(m)) and eig(H^(m-1)) (the leading block, same leading dimension)
  double2 *y2 = after_ews, *z2 = y2 + nn, *lam2 = z2 + nn;
  double2 *Y = lam2 + n, *Z = Y + size_t(m) * k2, *HY = Z + size_t(m) * k2;
  double2 *T = HY + size_t(m) * k2, *u = T + k2 * k2, *q = u + k2 * k2, *lamT = q + k2 * k2;
  double2 *yv = lamT + k2, *zv = yv + m;
  bool ok = win_eig(H, m, ld, lam1, y1, z1, ews, tlds, ctl);
  ok = win_eig(H, m - 1, ld, lam2, y2, z2, ews, tlds, ctl) && ok;
  if (!ok) {
    if (t == 0) *kept_out = -1;
    return;
  }
  for (int k = 0; k < nev; ++k)
    for (int i = t; i < m; i += kWinThreads) {
      Y[i + k * m] = y1[i + k * ld];
      Z[i + k * m] = z1[i + k * ld];
      Y[i + (nev + k) * m] = i < m - 1 ? y2[i + k * ld] : make_double2(0.0, 0.0);
      Z[i + (nev + k) * m] = i < m - 1 ? z2[i + k * ld] : make_double2(0.0, 0.0);
    }
  __syncthreads();
  // two-sided Gram-Schmidt (twice) of columns nev.. against the kept ones
  int kept = nev;
  for (int k = nev; k < k2; ++k) {
    for (int i = t; i < m; i += kWinThreads) {
      yv[i] = Y[i + k * m];
      zv[i] = Z[i + k * m];
    }
    __syncthreads();
    for (int pass = 0; pass < 2; ++pass)
      for (int qq = 0; qq < kept; ++qq) {
        double ar = 0, ai = 0, br = 0, bi = 0;
        for (int i = t; i < m; i += kWinThreads) {
          const wcx zq = ld2(Z + i + qq * m), yq = ld2(Y + i + qq * m), yi = ld2(yv + i), zi = ld2(zv + i);
          wcx a = {0, 0}, b = {0, 0};
          cfmac(a, zq, yi);
          cfmac(b, yq, zi);
          ar += a.x;
          ai += a.y;
          br += b.x;
          bi += b.y;
        }
        const wcx a = {wsum(ar), wsum(ai)}, b = {wsum(br), wsum(bi)};
        for (int i = t; i < m; i += kWinThreads) {
          st2(yv + i, ld2(yv + i) - ld2(Y + i + qq * m) * a);
          st2(zv + i, ld2(zv + i) - ld2(Z + i + qq * m) * b);
        }
        __syncthreads();
      }
    double pr = 0, pi = 0, ny = 0, nz = 0;
    for (int i = t; i < m; i += kWinThreads) {
      const wcx yi = ld2(yv + i), zi = ld2(zv + i);
      wcx p = {0, 0};
      cfmac(p, zi, yi);
      pr += p.x;
      pi += p.y;
      ny += yi.x * yi.x + yi.y * yi.y;
      nz += zi.x * zi.x + zi.y * zi.y;
    }
    wcx piv = {wsum(pr), wsum(pi)};
    ny = sqrt(wsum(ny));
    nz = sqrt(wsum(nz));
    if (!(wabs(piv) > 1e-12 * ny * nz)) continue;
    piv = (1.0 / ny) * piv;
    const wcx pc = cconj(piv);
    for (int i = t; i < m; i += kWinThreads) {
      st2(Y + i + kept * m, (1.0 / ny) * ld2(yv + i));
      st2(Z + i + kept * m, wdiv(ld2(zv + i), pc));
    }
    __syncthreads();
    ++kept;
  }
  // T = Zt^+ (H Yt), kept x kept
  for (int e = t; e < m * kept; e += kWinThreads) {
    const int i = e % m, c = e / m;
    wcx s = {0, 0};
    for (int j = 0; j < m; ++j) cfma(s, ld2(H + i + j * ld), ld2(Y + j + c * m));
    st2(HY + i + c * m, s);
  }
  __syncthreads();
  for (int e = t; e < kept * kept; e += kWinThreads) {
    const int p = e % kept, c = e / kept;
    wcx s = {0, 0};
    for (int i = 0; i < m; ++i) cfmac(s, ld2(Z + i + p * m), ld2(HY + i + c * m));
    st2(T + p + c * kept, s);
  }
  __syncthreads();
  if (!win_eig(T, kept, kept, lamT, u, q, ews, tlds, ctl)) {
    if (t == 0) *kept_out = -1;
    return;
  }
  // CV = Yt u, CW = Zt q, ||CV_k|| = 1, CW_k scaled by the same norm; then the scales
  for (int c = 0; c < k2; ++c) {
    double nrm2 = 0.0;
    for (int i = t; i < m; i += kWinThreads) {
      wcx sv = {0, 0}, sw = {0, 0};
      if (c < kept)
        for (int j = 0; j < kept; ++j) {
          cfma(sv, ld2(Y + i + j * m), ld2(u + j + c * kept));
          cfma(sw, ld2(Z + i + j * m), ld2(q + j + c * kept));
        }
      st2(cV + i + c * m, sv);
      st2(cW + i + c * m, sw);
      nrm2 += sv.x * sv.x + sv.y * sv.y;
    }
    const double nrm = sqrt(wsum(nrm2));
    for (int i = t; i < m; i += kWinThreads) {
      if (c < kept) {
        st2(cV + i + c * m, ld2(eta + i) * ((1.0 / nrm) * ld2(cV + i + c * m)));
        st2(cW + i + c * m, ld2(zeta + i) * (nrm * ld2(cW + i + c * m)));
      }
    }
  }
  for (int c = t; c < k2; c += kWinThreads) lam_out[c] = c < kept ? lamT[c] : make_double2(0.0, 0.0);
  if (t == 0) *kept_out = kept;
}

}  // namespace

size_t window_eig_ws_entries(int n) { return window_eig_ws_entries_dev(n); }

size_t window_restart_ws_entries(int m, int nev) {
  const size_t nn = size_t(m) * m, k2 = 2 * size_t(nev);
  return nn + 2 * m + 2 * nn + m + window_eig_ws_entries(m) + 2 * nn + m + 3 * m * k2 + 3 * k2 * k2 + k2 + 2 * m + 64;
}

void launch_window_eig(const WinCols &cols, int nev, int mode, const KrylovHistory &h, const double2 *lam_prev,
                       const double2 *dots_prev, double2 *cV, double2 *cW, double2 *lam_out, int *kept_out,
                       double2 *ws, int jtag, const KrylovState *S, hipStream_t st) {
  EB_LAUNCH(k_window_eig, dim3(1), dim3(kWinThreads), 0, st, cols, nev, mode, h, lam_prev, dots_prev, cV, cW,
            lam_out, kept_out, ws, jtag, S);
}

void launch_small_eig(const double2 *C, int n, double2 *lam, double2 *y, double2 *z, double2 *ws, int *status,
                      hipStream_t st) {
  EB_LAUNCH(k_small_eig, dim3(1), dim3(kWinThreads), 0, st, C, n, lam, y, z, ws, status);
}

}  // namespace ebicg
