// The window eigenproblems of eigBiCG on the device (one workgroup): eig(C)
// with the conventions of Sec. 1 (end), and Alg. BiCG-eigen's restart
// coefficients built from the device-resident BiCG scalars (winla.h).
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "kernels.h"
#include "winla.h"

namespace ebicg {
static_assert(kWinMaxN >= kMaxCols, "the device eigensolver takes every window size");
namespace {

// win_eig's global fallback: four matrices of leading dimension n | 1
__host__ __device__ constexpr size_t window_eig_ws_entries_dev(int n) { return 4 * size_t(n | 1) * n + 8; }

__global__ void __launch_bounds__(kWinThreads)
    k_small_eig(const double2 *C, int n, double2 *lam, double2 *y, double2 *z, double2 *ws, int *status) {
  const bool ok = win_eig(C, n, n, lam, y, z, ws, 0);
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

// Scratch layout of the window kernels (complex entries of ws), for an
// n-column window and k2 = 2 nev: offsets in the order of the members.
struct WinWs {
  double2 *H, *eta, *zeta, *y1, *z1, *lam1, *ews1;     // block 0: H^(n), eig(H^(n)), eig workspace
  double2 *H2, *eta2, *zeta2, *y2, *z2, *lam2, *ews2;  // block 1: its own H, eig(H^(n-1))
  int *ok;                                             // eig status of the two blocks
  double2 *Y, *Z, *HY, *T, *u, *q, *lamT, *yv, *zv;    // the restart's second phase
  // the sizes, in member order; ok takes one entry
  static constexpr int kParts = 25;
  __host__ __device__ static void sizes(int n, int nev, size_t (&sz)[kParts]) {
    const size_t nn = size_t(n) * n, k2 = 2 * size_t(nev), E = window_eig_ws_entries_dev(n);
    const size_t v[kParts] = {nn, size_t(n), size_t(n), nn, nn, size_t(n), E,  // block 0
                              nn, size_t(n), size_t(n), nn, nn, size_t(n), E,  // block 1
                              1,                                               // ok
                              n * k2, n * k2, n * k2, k2 * k2, k2 * k2, k2 * k2, k2, size_t(n), size_t(n), 0};
    for (int i = 0; i < kParts; ++i) sz[i] = v[i];
  }
  __host__ __device__ static size_t total(int n, int nev) {
    size_t sz[kParts], t = 0;
    sizes(n, nev, sz);
    for (int i = 0; i < kParts; ++i) t += sz[i];
    return t;
  }
  __device__ WinWs(double2 *ws, int n, int nev) {
    size_t sz[kParts];
    sizes(n, nev, sz);
    double2 *p[kParts];
    size_t off = 0;
    for (int i = 0; i < kParts; ++i) {
      p[i] = ws + off;
      off += sz[i];
    }
    H = p[0], eta = p[1], zeta = p[2], y1 = p[3], z1 = p[4], lam1 = p[5], ews1 = p[6];
    H2 = p[7], eta2 = p[8], zeta2 = p[9], y2 = p[10], z2 = p[11], lam2 = p[12], ews2 = p[13];
    ok = reinterpret_cast<int *>(p[14]);
    Y = p[15], Z = p[16], HY = p[17], T = p[18], u = p[19], q = p[20], lamT = p[21], yv = p[22], zv = p[23];
  }
};

__device__ __forceinline__ bool win_skipped(const KrylovState *S, int jtag) { return S && S->stopped && jtag > S->stop_at; }

// Alg. BiCG-eigen on the device, first phase: block 0 solves [y, z] =
// eig(H^(m)), block 1 [y', z'] = eig(H^(m-1)) (the leading block of its own
// copy of H); the two run on two CUs at once.  Skipped when the solve stopped
// before iteration jtag.
__global__ void __launch_bounds__(kWinThreads)
    k_window_pair(WinCols cols, int nev, int which, KrylovHistory h, const double2 *lam_prev,
                  const double2 *dots_prev, double2 *ws, int jtag, const KrylovState *S) {
  if (win_skipped(S, jtag)) return;
  const int m = cols.n;
  const WinWs w(ws, m, nev);
  const bool second = blockIdx.x == 1;
  double2 *H = second ? w.H2 : w.H;
  win_build_H(H, m, cols, h, lam_prev, dots_prev, dots_prev + 2 * nev, second ? w.eta2 : w.eta,
              second ? w.zeta2 : w.zeta);
  const bool ok = second ? win_eig(H, m - 1, m, w.lam2, w.y2, w.z2, w.ews2, which)
                         : win_eig(H, m, m, w.lam1, w.y1, w.z1, w.ews1, which);
  if (threadIdx.x == 0) w.ok[blockIdx.x] = ok ? 1 : 0;
}

// Alg. BiCG-eigen, second phase (one block): the 2 nev coefficient vectors
// [y_1..nev, y'_1..nev with a zero appended] biorthogonalised (two-sided
// Gram-Schmidt, twice; a pair with pivot below 1e-12 |y||z| is dropped),
// T = Zt^+ H Yt, [u, q, Lambda] = eig(T), CV = Yt u, CW = Zt q with
// ||CV_k|| = 1, CW_k^+ CV_k = 1, written with the stored residuals' scales
// folded in (cV = diag(eta) CV, cW = diag(zeta) CW; m x 2 nev column-major,
// columns >= kept zero), lam_out = Lambda, *kept_out = kept (-1 if an
// eigenproblem failed, -2 if skipped).
__global__ void __launch_bounds__(kWinThreads)
    k_window_restart(WinCols cols, int nev, int which, double2 *cV, double2 *cW, double2 *lam_out, int *kept_out,
                     double2 *ws, int jtag, const KrylovState *S) {
  if (win_skipped(S, jtag)) {  // the restart's iteration did not run
    if (threadIdx.x == 0) *kept_out = -2;
    return;
  }
  const int m = cols.n, t = threadIdx.x, ld = m, k2 = 2 * nev;
  const WinWs w(ws, m, nev);
  if (!(w.ok[0] == 1 && w.ok[1] == 1)) {
    if (t == 0) *kept_out = -1;
    return;
  }
  double2 *H = w.H, *eta = w.eta, *zeta = w.zeta, *y1 = w.y1, *z1 = w.z1, *y2 = w.y2, *z2 = w.z2;
  double2 *Y = w.Y, *Z = w.Z, *HY = w.HY, *T = w.T, *u = w.u, *q = w.q, *lamT = w.lamT, *yv = w.yv, *zv = w.zv;
  double2 *ews = w.ews1;
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
  if (!win_eig(T, kept, kept, lamT, u, q, ews, which)) {
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

// The final extraction of Alg. eigBiCG on the device (one block):
// eig(H^(vs)) of the n-column window, the first min(nev, n) pairs, cV =
// diag(eta) y, cW = diag(zeta) z (n x kout column-major), lam_out, *kept_out
// (-1 if the eigenproblem failed).
__global__ void __launch_bounds__(kWinThreads)
    k_window_final(WinCols cols, int nev, int which, KrylovHistory h, const double2 *lam_prev,
                   const double2 *dots_prev, double2 *cV, double2 *cW, double2 *lam_out, int *kept_out, double2 *ws) {
  const int n = cols.n, t = threadIdx.x, ld = n;
  const WinWs w(ws, n, nev);
  win_build_H(w.H, ld, cols, h, lam_prev, dots_prev, dots_prev + 2 * nev, w.eta, w.zeta);
  const bool ok = win_eig(w.H, n, ld, w.lam1, w.y1, w.z1, w.ews1, which);
  const int k = nev < n ? nev : n;
  for (int c = 0; c < k; ++c)
    for (int i = t; i < n; i += kWinThreads) {
      st2(cV + i + c * n, ld2(w.eta + i) * ld2(w.y1 + i + c * ld));
      st2(cW + i + c * n, ld2(w.zeta + i) * ld2(w.z1 + i + c * ld));
    }
  for (int c = t; c < k; c += kWinThreads) lam_out[c] = w.lam1[c];
  if (t == 0) *kept_out = ok ? k : -1;
}

}  // namespace

size_t window_eig_ws_entries(int n) { return window_eig_ws_entries_dev(n); }

size_t window_restart_ws_entries(int m, int nev) { return WinWs::total(m, nev) + 64; }

void launch_window_eig(const WinCols &cols, int nev, int mode, int which, const KrylovHistory &h,
                       const double2 *lam_prev, const double2 *dots_prev, double2 *cV, double2 *cW, double2 *lam_out,
                       int *kept_out, double2 *ws, int jtag, const KrylovState *S, hipStream_t st) {
  if (mode == 1) {
    EB_LAUNCH(k_window_final, dim3(1), dim3(kWinThreads), 0, st, cols, nev, which, h, lam_prev, dots_prev, cV, cW,
              lam_out, kept_out, ws);
    return;
  }
  EB_LAUNCH(k_window_pair, dim3(2), dim3(kWinThreads), 0, st, cols, nev, which, h, lam_prev, dots_prev, ws, jtag, S);
  EB_LAUNCH(k_window_restart, dim3(1), dim3(kWinThreads), 0, st, cols, nev, which, cV, cW, lam_out, kept_out, ws,
            jtag, S);
}

void launch_small_eig(const double2 *C, int n, double2 *lam, double2 *y, double2 *z, double2 *ws, int *status,
                      hipStream_t st) {
  EB_LAUNCH(k_small_eig, dim3(1), dim3(kWinThreads), 0, st, C, n, lam, y, z, ws, status);
}

}  // namespace ebicg
