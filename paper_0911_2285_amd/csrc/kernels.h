// Host-side launch interface of the HIP kernels (kernels.hip) used by the
// solver drivers (api.hip).  All launches are asynchronous on `st`.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace ebicg {

struct bf16c;

// Lattice geometry; V = lx*ly*lz*lt, N = 12 V complex entries per spinor.
struct Geom {
  int lx, ly, lz, lt;
  int V;
};

// Scalars of one Krylov solve, resident in device memory and updated by the
// last block of each reducing kernel (so the iteration needs no host round
// trip).  Kernels tagged with iteration j do nothing once stopped && j > stop_at.
struct KrylovState {
  double2 rho;    // BiCG: rho_{j-1} = (rhat_{j-1}, r_{j-1});  BiCGStab: (rhat_0, r)
  double2 alpha;  // BiCG: alpha_{j-1}
  double2 beta;   // BiCG: beta_{j-1}
  double2 omega;  // BiCGStab
  double rnorm;   // recursive residual norm
  double bnorm;   // ||b||
  double tol_abs; // stop when rnorm <= tol_abs
  double def_thr; // BiCGStab: stop (reason 3) when rnorm < def_thr; 0 = off
  int stopped;    // 1 once the iteration has stopped
  int stop_at;    // last iteration whose updates count
  int reason;     // 1 converged, 2 breakdown, 3 DefTol threshold, 4 maxiter
  int maxiter;
};

// Per-iteration BiCG scalars (the window matrix H is built from them on the host).
struct KrylovHistory {
  double2 *alpha;  // alpha[i] = alpha_i
  double2 *beta;   // beta[i]  = beta_i = rho_{i+1} / rho_i
  double2 *rho;    // rho[i]   = (rhat_i, r_i)
  double *rn;      // rn[i]    = ||r_i||
};

// Scratch for grid-wide reductions: partial sums and tickets.  Tickets must
// start at zero; every reducing kernel returns its ticket to zero.
struct RedScratch {
  double *partials;   // >= kMaxPartials doubles
  unsigned *tickets;  // >= kMaxTickets
};
constexpr size_t kMaxPartials = size_t(1) << 22;
constexpr int kMaxTickets = 1024;

constexpr int kMaxCols = 128;  // columns addressed by one rotation / projection launch
struct SlotList {
  int n;
  int idx[kMaxCols];
};

// ---- layouts --------------------------------------------------------------
// canonical [V][12] complex128 <-> internal SoA [12][V] (FP64 / FP32 / BF16)
void launch_to_soa_f64(double2 *dst, const double2 *src, const Geom &g, hipStream_t st);
void launch_from_soa_f64(double2 *dst, const double2 *src, const Geom &g, hipStream_t st);
void launch_to_soa_f32(float2 *dst, const float2 *src, const Geom &g, hipStream_t st);
void launch_from_soa_f32(float2 *dst, const float2 *src, const Geom &g, hipStream_t st);
void launch_to_soa_bf16(bf16c *dst, const bf16c *src, const Geom &g, hipStream_t st);
void launch_from_soa_bf16(bf16c *dst, const bf16c *src, const Geom &g, hipStream_t st);
// canonical gauge [4][V][3][3] complex128 -> SoA [4][9][V], t-boundary sign folded in
void launch_pack_gauge_f64(double2 *dst, const double2 *src, const Geom &g, int bc_t, hipStream_t st);
// precision conversions of SoA fields (n complex entries)
void launch_convert_f64_f32(float2 *dst, const double2 *src, size_t n, hipStream_t st);
void launch_convert_f64_bf16(bf16c *dst, const double2 *src, size_t n, hipStream_t st);
void launch_convert_f32_f64(double2 *dst, const float2 *src, size_t n, hipStream_t st);
void launch_convert_bf16_f64(double2 *dst, const bf16c *src, size_t n, hipStream_t st);

// ---- operator ---------------------------------------------------------------
// out = D in, or D^+ in when dagger; internal SoA layout.
void launch_dslash_f64(double2 *out, const double2 *in, const double2 *U, const Geom &g, double kappa, bool dagger,
                       hipStream_t st);
void launch_dslash_f32(float2 *out, const float2 *in, const float2 *U, const Geom &g, double kappa, bool dagger,
                       hipStream_t st);
void launch_dslash_bf16(bf16c *out, const bf16c *in, const bf16c *U, const Geom &g, double kappa, bool dagger,
                        hipStream_t st);
// r = b - D x (FP64); res[0] = ||r||^2, res[1] = ||b||^2 (device)
void launch_residual_f64(double2 *r, const double2 *b, const double2 *x, const double2 *U, const Geom &g, double kappa,
                         double *res, const RedScratch &rs, hipStream_t st);

// ---- BiCG (FP64, window slots) ------------------------------------------------
// Initial state: rhat_0 = r_0 (rhat_mode 0) or gamma5 r_0 (1); p = r_0, phat = rhat_0;
// rho_0 and ||r_0|| into state/history; res = {||r0||^2, ||b||^2} from launch_residual.
void launch_bicg_init(double2 *rhat, double2 *p, double2 *phat, const double2 *r, const double *res, size_t N,
                      int rhat_mode, const Geom &g, double tol, int maxiter, KrylovState *S, KrylovHistory h,
                      const RedScratch &rs, hipStream_t st);
// Ap = D p, Adp = D^+ phat; sigma = (phat, Ap); alpha = rho / sigma.
void launch_bicg_matvec(double2 *Ap, double2 *Adp, const double2 *p, const double2 *phat, const double2 *U,
                        const Geom &g, double kappa, int j, KrylovState *S, KrylovHistory h, const RedScratch &rs,
                        hipStream_t st);
// r_out = r_in - alpha Ap; rhat_out = rhat_in - conj(alpha) Adp; rho_j, ||r_j||, beta_{j-1}.
void launch_bicg_update_r(double2 *r_out, double2 *rh_out, const double2 *r_in, const double2 *rh_in,
                          const double2 *Ap, const double2 *Adp, size_t N, int j, KrylovState *S, KrylovHistory h,
                          const RedScratch &rs, hipStream_t st);
// x += alpha p; p = r + beta p; phat = rhat + conj(beta) phat.
void launch_bicg_update_p(double2 *x, double2 *p, double2 *ph, const double2 *r, const double2 *rh, size_t N, int j,
                          const KrylovState *S, hipStream_t st);
// GA = Adp - conj(beta_{j-2}) s ; GB = Ap - beta_{j-2} q  (the arrow vectors of a restart)
void launch_arrow_vectors(double2 *GA, double2 *GB, const double2 *Adp, const double2 *s, const double2 *Ap,
                          const double2 *q, size_t N, int j, const KrylovState *S, KrylovHistory h, hipStream_t st);
// out[k] = sum_c in[c] C[c + k*nin] for k < nout (out-of-place, slots into one base each).
// If g != null: dots[k] = g^+ out[k] (conj_out = 0) or out[k]^+ g (conj_out = 1).
void launch_rotate(double2 *out_base, const SlotList &out_slots, const double2 *in_base, const SlotList &in_slots,
                   const double2 *C, size_t N, const double2 *g, int conj_out, double2 *dots, int jtag,
                   const KrylovState *S, const RedScratch &rs, hipStream_t st);

// ---- tall-skinny projections (FP64) ------------------------------------------------
// out[a + b*nx] = sum_i conj(X_a[i]) Y_b[i];  X_a = X + a*ldx, Y_b = Y + b*ldy.
void launch_ts_dot(double2 *out, const double2 *X, size_t ldx, int nx, const double2 *Y, size_t ldy, int ny, size_t N,
                   const RedScratch &rs, hipStream_t st);
// Y_b += sgn * sum_a X_a C[a + b*nx]
void launch_ts_update(double2 *Y, size_t ldy, int ny, const double2 *X, size_t ldx, int nx, const double2 *C,
                      double sgn, size_t N, hipStream_t st);

// ---- BLAS-1 (FP64) ---------------------------------------------------------------
void launch_copy_f64(double2 *dst, const double2 *src, size_t n, hipStream_t st);
void launch_scale_f64(double2 *x, double2 a, size_t n, hipStream_t st);
// y += x
void launch_add_f64(double2 *y, const double2 *x, size_t n, hipStream_t st);

// ---- BiCGStab (storage S: FP64, FP32 or BF16; reductions in FP64) -------------------
template <typename S>
void launch_stab_init(S *rhat, S *p, const S *r, size_t N, double tol_abs, double def_thr, int maxiter,
                      KrylovState *K, const RedScratch &rs, hipStream_t st);
template <typename S>
void launch_stab_v(S *v, const S *p, const S *rhat, const S *U, const Geom &g, double kappa, int j, KrylovState *K,
                   const RedScratch &rs, hipStream_t st);
template <typename S>
void launch_stab_s(S *s, const S *r, const S *v, size_t N, int j, const KrylovState *K, hipStream_t st);
template <typename S>
void launch_stab_t(S *t, const S *s, const S *U, const Geom &g, double kappa, int j, KrylovState *K,
                   const RedScratch &rs, hipStream_t st);
template <typename S>
void launch_stab_xr(S *x, S *r, const S *p, const S *s, const S *t, const S *rhat, size_t N, int j, KrylovState *K,
                    const RedScratch &rs, hipStream_t st);
template <typename S>
void launch_stab_p(S *p, const S *r, const S *v, size_t N, int j, const KrylovState *K, hipStream_t st);

}  // namespace ebicg
