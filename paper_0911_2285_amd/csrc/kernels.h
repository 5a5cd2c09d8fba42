// Host-side launch interface of the HIP kernels (kernels.hip) used by the
// solver drivers (api.hip).  All launches are asynchronous on `st`.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "device_common.h"  // storage types (double2, float2, bf16c)

namespace ebicg {

// Kernel-stamped timing.  While `stop` is set on this host thread, every
// launch through EB_LAUNCH takes its timestamps from the dispatch itself
// (hipExtLaunchKernel): the first launch stamps `start`, each launch stamps
// `stop`, so the interval runs from the first kernel's start to the last
// kernel's end and leaves out the queue gaps that stream events include.
struct LaunchStamp {
  hipEvent_t start = nullptr, stop = nullptr;
  bool started = false;
};
LaunchStamp &launch_stamp();

// Grid cap of the stencil kernels that carry reductions (their blocks loop
// over the site tiles beyond it); per host thread, set from the operator by
// every entry point before its launches.  Default kDefaultStencilCap.
constexpr int kDefaultStencilCap = 1024;
int &stencil_block_cap();

#define EB_LAUNCH(kernel, grid, block, shmem, st, ...)                                                       \
  do {                                                                                                       \
    ::ebicg::LaunchStamp &eb_ls_ = ::ebicg::launch_stamp();                                                 \
    if (eb_ls_.stop) {                                                                                       \
      hipExtLaunchKernelGGL(kernel, grid, block, shmem, st, eb_ls_.started ? nullptr : eb_ls_.start, eb_ls_.stop, \
                            0, __VA_ARGS__);                                                                 \
      eb_ls_.started = true;                                                                                 \
    } else {                                                                                                 \
      hipLaunchKernelGGL(kernel, grid, block, shmem, st, __VA_ARGS__);                                       \
    }                                                                                                        \
  } while (0)

// Lattice geometry; V = lx*ly*lz*lt, N = 12 V complex entries per spinor.
struct Geom {
  int lx, ly, lz, lt;
  int V;
};

// Flags of one Krylov solve in device memory.  The scalars of iteration j
// live in KrylovHistory at index j; the kernel that reduces a quantity's
// partial sums (the consumer, in its prologue) writes them, so no kernel ever
// reads a slot that another block of the same launch writes.  Kernels tagged
// with iteration j do nothing once stopped && j > stop_at.
struct KrylovState {
  double bnorm;    // ||b||
  double tol_abs;  // stop when the recursive residual norm <= tol_abs
  double def_thr;  // BiCGStab: stop (reason 3) when it drops below def_thr; 0 = off
  double rnorm;    // last recursive residual norm
  int stopped;     // 1 once the iteration has stopped
  int stop_at;     // last iteration whose updates count
  int reason;      // 1 converged, 2 breakdown, 3 DefTol threshold, 4 maxiter
  int maxiter;
};

// Per-iteration scalars.  BiCG: alpha[i] = alpha_i, beta[i] = rho_{i+1}/rho_i,
// rho[i] = (rhat_i, r_i), rn[i] = ||r_i||.  BiCGStab (iteration j = 1, 2, ...):
// rho[j] = (rhat_0, r_j), alpha[j], omega[j], beta[j] (for p_{j+1}), rn[j].
struct KrylovHistory {
  double2 *alpha;
  double2 *beta;
  double2 *rho;
  double2 *omega;
  double *rn;
};

// Scratch for reductions: per-block partial sums written by a producing
// kernel and summed, in a fixed order, by the kernel that consumes them.
struct RedScratch {
  double *partials;  // >= kMaxPartials doubles
};
constexpr size_t kMaxPartials = size_t(1) << 23;
constexpr int kMaxRedBlocks = 2048;         // grid cap of the streaming reducing kernels
constexpr size_t kRegionDoubles = 1 << 17;  // partial records per producer region (doubles)
// Largest volume the library accepts: the window rotation keeps one partial
// record of up to 40 doubles per block of 256 entries of a spinor (12 V
// entries) in the general region of the scratch.
constexpr long long kMaxVolume = 4LL << 20;

constexpr int kMaxCols = 128;  // columns addressed by one rotation / projection launch
struct SlotList {
  int n;
  int idx[kMaxCols];
};

// ---- layouts --------------------------------------------------------------
// canonical [V][12] complex <-> internal SoA [12][V] (FP64 / FP32 / BF16)
void launch_to_soa_f64(double2 *dst, const double2 *src, const Geom &g, hipStream_t st);
void launch_from_soa_f64(double2 *dst, const double2 *src, const Geom &g, hipStream_t st);
void launch_to_soa_f32(float2 *dst, const float2 *src, const Geom &g, hipStream_t st);
void launch_from_soa_f32(float2 *dst, const float2 *src, const Geom &g, hipStream_t st);
// canonical gauge [4][V][3][3] complex128 -> SoA [4][9][V], t-boundary sign folded in
void launch_pack_gauge_f64(double2 *dst, const double2 *src, const Geom &g, int bc_t, hipStream_t st);
// precision conversions of SoA fields (n complex entries)
void launch_convert_f64_f32(float2 *dst, const double2 *src, size_t n, hipStream_t st);
void launch_convert_f32_f64(double2 *dst, const float2 *src, size_t n, hipStream_t st);
// BF16 storage: (re, im) as two bfloat16 (round to nearest even), arithmetic in FP32
void launch_to_soa_bf16(bf16c *dst, const bf16c *src, const Geom &g, hipStream_t st);
void launch_from_soa_bf16(bf16c *dst, const bf16c *src, const Geom &g, hipStream_t st);
void launch_convert_f64_bf16(bf16c *dst, const double2 *src, size_t n, hipStream_t st);
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
// g5 selects the gamma5-Hermitian form (Sec. 4, rhat_mode 2): the shadow
// vectors rhat_j = gamma5 r_j and phat_j = gamma5 p_j are never formed, the
// rhat/phat/Adp/s arguments are not touched (they may be null) and each
// iteration applies D once.
//
// Initial state: rhat_0 = r_0 (rhat_mode 0) or gamma5 r_0 (1, 2); p = r_0, phat = rhat_0
// (not written in mode 2); rho_0, ||r_0||, ||b|| into state/history; res = {||r0||^2, ||b||^2}
// from launch_residual.
void launch_bicg_init(double2 *rhat, double2 *p, double2 *phat, const double2 *r, const double *res, size_t N,
                      int rhat_mode, const Geom &g, double tol, int maxiter, KrylovState *S, KrylovHistory h,
                      const RedScratch &rs, hipStream_t st);
// Ap = D p, Adp = D^+ phat; partials of sigma = (phat, Ap).
void launch_bicg_matvec(double2 *Ap, double2 *Adp, const double2 *p, const double2 *phat, const double2 *U,
                        const Geom &g, double kappa, int j, KrylovState *S, KrylovHistory h, const RedScratch &rs,
                        bool g5, hipStream_t st);
// alpha_{j-1} = rho_{j-1} / sigma; r_out = r_in - alpha Ap; rhat_out = rhat_in - conj(alpha) Adp;
// partials of rho_j and ||r_j||^2.  w32r / w32rh (may be null): FP32 copies of
// r_out / rhat_out (the window of an FP32-window eigBiCG).  nrec: the sigma
// records of the matvec (0: those of launch_bicg_matvec).
void launch_bicg_update_r(double2 *r_out, double2 *rh_out, const double2 *r_in, const double2 *rh_in,
                          const double2 *Ap, const double2 *Adp, size_t N, int j, KrylovState *S, KrylovHistory h,
                          const RedScratch &rs, bool g5, hipStream_t st, float2 *w32r = nullptr,
                          float2 *w32rh = nullptr, int nrec = 0);
// beta_{j-1}, rho_j, ||r_j|| and the stop test; x += alpha p; p = r + beta p; phat = rhat + conj(beta) phat.
void launch_bicg_update_p(double2 *x, double2 *p, double2 *ph, const double2 *r, const double2 *rh, size_t N, int j,
                          KrylovState *S, KrylovHistory h, const RedScratch &rs, bool g5, hipStream_t st);
// GA = Adp - conj(beta_{j-2}) s ; GB = Ap - beta_{j-2} q  (the arrow vectors of a restart);
// g5: GA = gamma5 (Ap - conj(beta_{j-2}) q).
void launch_arrow_vectors(double2 *GA, double2 *GB, const double2 *Adp, const double2 *s, const double2 *Ap,
                          const double2 *q, size_t N, int j, const KrylovState *S, KrylovHistory h, bool g5,
                          hipStream_t st);
// out[k] = sum_c in[c] C[c + k*nin] for k < nout (out-of-place, slots into one base each).
// An input slot given as -(slot + 1) is read as gamma5 in[slot] (spinor columns,
// N = 12 V: components 6..11 flip sign).
// If g != null: dots[k] = g^+ out[k] (conj_out = 0) or out[k]^+ g (conj_out = 1).
void launch_rotate(double2 *out_base, const SlotList &out_slots, const double2 *in_base, const SlotList &in_slots,
                   const double2 *C, size_t N, const double2 *g, int conj_out, double2 *dots, int jtag,
                   const KrylovState *S, const RedScratch &rs, hipStream_t st);
// The same for an FP32 window: FP32 columns in, FP32 (window) or FP64 (the
// deflation space) columns out; coefficients, sums and dots in FP64.
void launch_rotate(float2 *out_base, const SlotList &out_slots, const float2 *in_base, const SlotList &in_slots,
                   const double2 *C, size_t N, const double2 *g, int conj_out, double2 *dots, int jtag,
                   const KrylovState *S, const RedScratch &rs, hipStream_t st);
void launch_rotate(double2 *out_base, const SlotList &out_slots, const float2 *in_base, const SlotList &in_slots,
                   const double2 *C, size_t N, const double2 *g, int conj_out, double2 *dots, int jtag,
                   const KrylovState *S, const RedScratch &rs, hipStream_t st);

// ---- even-odd (Schur) form, FP64 (eo.hip) -------------------------------------
// Half-lattice spinors: SoA [12][V/2] of one parity, sites in increasing order
// (index s / 2; every extent even).  Links: [parity][4][9][V/2] (pack_gauge_eo).
// Dhat = 1 - kappa^2 H_eo H_oe on the even sites; tmp is an odd-site scratch spinor.
bool eo_geometry_ok(const Geom &g);
void launch_to_eo(double2 *e, double2 *o, const double2 *canon, const Geom &g, hipStream_t st);
// o may be null: the odd sites of the canonical output are zero
void launch_from_eo(double2 *canon, const double2 *e, const double2 *o, const Geom &g, hipStream_t st);
void launch_pack_gauge_eo(double2 *Ueo, const double2 *canon, const Geom &g, int bc_t, hipStream_t st);
// out = Dhat in (dagger: Dhat^+ in)
void launch_schur_eo(double2 *out, const double2 *in, double2 *tmp, const double2 *Ueo, const Geom &g, double kappa,
                     bool dagger, hipStream_t st);
// out = id + kappa H_{P,1-P} in, P = out_parity: b_hat = b_e + kappa H_eo b_o (P = 0),
// x_o = b_o + kappa H_oe x_e (P = 1)
void launch_prep_eo(double2 *out, const double2 *id, const double2 *in, const Geom &g, const double2 *Ueo,
                    double kappa, int out_parity, hipStream_t st);
// r = b - Dhat x; res = {||r||^2, ||b||^2} (device)
void launch_residual_eo(double2 *r, const double2 *b, const double2 *x, double2 *tmp, const double2 *Ueo,
                        const Geom &g, double kappa, double *res, const RedScratch &rs, hipStream_t st);
// the BiCG matvec pair on Dhat with the sigma records (as launch_bicg_matvec)
void launch_bicg_matvec_eo(double2 *Ap, double2 *Adp, const double2 *p, const double2 *ph, double2 *tmp,
                           const double2 *Ueo, const Geom &g, double kappa, int j, KrylovState *S,
                           const RedScratch &rs, bool g5, hipStream_t st);
// BiCGStab v = Dhat p with (rhat, v), t = Dhat s with (t, s), ||t||^2 (as launch_stab_v/t);
// storage S = double2, float2 or bf16c (links in the same storage), FP64 partials.
template <typename S>
void launch_stab_v_eo(S *v, const S *p, const S *rhat, S *tmp, const S *Ueo, const Geom &g, double kappa, int j,
                      KrylovState *K, const RedScratch &rs, hipStream_t st);
template <typename S>
void launch_stab_t_eo(S *t, const S *sv, S *tmp, const S *Ueo, const Geom &g, double kappa, int j, KrylovState *K,
                      const RedScratch &rs, hipStream_t st);
// out = Dhat in (dagger: Dhat^+ in) in storage S
template <typename S>
void launch_schur_eo_s(S *out, const S *in, S *tmp, const S *Ueo, const Geom &g, double kappa, bool dagger,
                       hipStream_t st);
// Multi-RHS on Dhat: kc half-lattice spinors in the batch layout (element
// (c, h, col) at (c V/2 + h) kc + col), tmp the same size.  out = Dhat in per
// column; the BiCGStab forms as launch_bstab_v/t, with records for the batched
// BiCGStab passes called with a geometry of V/2 sites.
// stage: tile form of the batched hops (1: the input tile staged in LDS, 0:
// neighbours read from global memory, < 0: the built-in rule; the bricked
// forms are for the full-lattice stencil only).
template <typename S>
void launch_bschur_eo(S *out, const S *in, S *tmp, const S *Ueo, const Geom &g, double kappa, bool dagger, int kc,
                      hipStream_t st, int stage = -1);
template <typename S>
void launch_bstab_v_eo(S *v, const S *p, const S *rhat, S *tmp, const S *Ueo, const Geom &g, double kappa, int j,
                       int kc, KrylovState *K, const RedScratch &rs, hipStream_t st, int stage = -1);
template <typename S>
void launch_bstab_t_eo(S *t, const S *sv, S *tmp, const S *Ueo, const Geom &g, double kappa, int j, int kc,
                       KrylovState *K, const RedScratch &rs, hipStream_t st, int stage = -1);

// ---- tall-skinny projections (FP64) ------------------------------------------------
// out[a + b*nx] = sum_i conj(X_a[i]) Y_b[i];  X_a = X + a*ldx, Y_b = Y + b*ldy.
void launch_ts_dot(double2 *out, const double2 *X, size_t ldx, int nx, const double2 *Y, size_t ldy, int ny, size_t N,
                   const RedScratch &rs, hipStream_t st);
// Y_b += sgn * sum_a X_a C[a + b*nx]  (nx, ny <= kMaxCols)
void launch_ts_update(double2 *Y, size_t ldy, int ny, const double2 *X, size_t ldx, int nx, const double2 *C,
                      double sgn, size_t N, hipStream_t st);

// Tall-skinny forms (tsmm.hip).  gram (matrix cores): out = X^+ Y for nx <= 128 (any ny);
// part: scratch for per-block records, part_cap doubles.
void launch_gram_mfma(double2 *out, const double2 *X, size_t ldx, int nx, const double2 *Y, size_t ldy, int ny,
                      size_t N, double *part, size_t part_cap, hipStream_t st);
// combine: out_k (+)= sgn sum_c in_c C[c + k*nin], column c at in_base + in_slots.idx[c]*ldi and
// out_k at out_base + out_slots.idx[k]*ldo; with g, dots[k] = g^+ out_k (conj_out 0) or out_k^+ g (1).
// Skipped when S && S->stopped && jtag > S->stop_at.
void launch_combine(double2 *out_base, const SlotList &out_slots, size_t ldo, const double2 *in_base,
                    const SlotList &in_slots, size_t ldi, const double2 *C, double sgn, bool add, size_t N,
                    const double2 *g, int conj_out, double2 *dots, int jtag, const KrylovState *S, double *part,
                    size_t part_cap, hipStream_t st);
void launch_combine(float2 *out_base, const SlotList &out_slots, size_t ldo, const float2 *in_base,
                    const SlotList &in_slots, size_t ldi, const double2 *C, size_t N, const double2 *g, int conj_out,
                    double2 *dots, int jtag, const KrylovState *S, double *part, size_t part_cap, hipStream_t st);
void launch_combine(double2 *out_base, const SlotList &out_slots, size_t ldo, const float2 *in_base,
                    const SlotList &in_slots, size_t ldi, const double2 *C, size_t N, const double2 *g, int conj_out,
                    double2 *dots, int jtag, const KrylovState *S, double *part, size_t part_cap, hipStream_t st);

// ---- BLAS-1 (FP64) ---------------------------------------------------------------
void launch_copy_f64(double2 *dst, const double2 *src, size_t n, hipStream_t st);
void launch_scale_f64(double2 *x, double2 a, size_t n, hipStream_t st);
// y += x
void launch_add_f64(double2 *y, const double2 *x, size_t n, hipStream_t st);

// ---- BiCGStab (storage S: FP64 or FP32; reductions and scalars in FP64) -----------
// rhat = p = r; rho_0 = ||r||^2; flags.
template <typename S>
void launch_stab_init(S *rhat, S *p, const S *r, size_t N, double tol_abs, double def_thr, int maxiter,
                      KrylovState *K, KrylovHistory h, const RedScratch &rs, hipStream_t st);
// v = D p; partials of (rhat, v)
template <typename S>
void launch_stab_v(S *v, const S *p, const S *rhat, const S *U, const Geom &g, double kappa, int j, KrylovState *K,
                   KrylovHistory h, const RedScratch &rs, hipStream_t st);
// alpha_j = rho_{j-1} / (rhat, v); s = r - alpha v.  nrec: the records of the
// v pass (launch_stab_v: 0; the t-marching pass: march_records(g, 1)).
template <typename S>
void launch_stab_s(S *s, const S *r, const S *v, size_t N, int j, KrylovState *K, KrylovHistory h,
                   const RedScratch &rs, hipStream_t st, int nrec = 0);
// t = D s; partials of (t, s), (t, t)
template <typename S>
void launch_stab_t(S *t, const S *s, const S *U, const Geom &g, double kappa, int j, KrylovState *K, KrylovHistory h,
                   const RedScratch &rs, hipStream_t st);
// omega_j; x += alpha p + omega s; r = s - omega t; partials of (rhat, r), ||r||^2.
// nrec: the records of the t pass, as for launch_stab_s.
template <typename S>
void launch_stab_xr(S *x, S *r, const S *p, const S *s, const S *t, const S *rhat, size_t N, int j, KrylovState *K,
                    KrylovHistory h, const RedScratch &rs, hipStream_t st, int nrec = 0);
// rho_j, beta_j, the stop tests; p = r + beta (p - omega v)
template <typename S>
void launch_stab_p(S *p, const S *r, const S *v, size_t N, int j, KrylovState *K, KrylovHistory h,
                   const RedScratch &rs, hipStream_t st);

// ---- window eigenproblems on the device (winrestart.hip) -----------------------------
// eig(C) of an n x n column-major matrix by one workgroup (conventions of the
// host eig_small); ws: window_eig_ws_entries(n) complex; *status = 1 on success.
size_t window_eig_ws_entries(int n);
void launch_small_eig(const double2 *C, int n, double2 *lam, double2 *y, double2 *z, double2 *ws, int *status,
                      hipStream_t st);
// The columns of an eigBiCG window: column c is Ritz vector idx[c] of the last
// restart (ritz[c] = 1) or the stored residual r_idx[c] (ritz[c] = 0).
struct WinCols {
  int n;
  int idx[kMaxCols];
  unsigned char ritz[kMaxCols];
};
// Alg. BiCG-eigen (mode 0) or the final extraction (mode 1) of the window
// `cols` by one workgroup, from the device history h, the last restart's Ritz
// values lam_prev and raw arrow dots dots_prev (dV at [0, 2nev), dW at [2nev,
// 4nev)).  Outputs: cV, cW (cols.n x kout coefficient blocks with the stored
// residuals' scales folded in; kout = 2 nev, or min(nev, n) in mode 1), lam_out,
// *kept_out (-1 if an eigenproblem failed).  Skipped when the solve stopped
// before iteration jtag.  which: the sort criterion of every eig() (0
// |lambda| ascending, 1 real part ascending, 2 |lambda| descending).  ws:
// window_restart_ws_entries(cols.n, nev) complex.
size_t window_restart_ws_entries(int m, int nev);
void launch_window_eig(const WinCols &cols, int nev, int mode, int which, const KrylovHistory &h,
                       const double2 *lam_prev, const double2 *dots_prev, double2 *cV, double2 *cW, double2 *lam_out,
                       int *kept_out, double2 *ws, int jtag, const KrylovState *S, hipStream_t st);

// ---- multi-RHS batches (batch.hip) ------------------------------------------------
// A batch holds kc right-hand sides interleaved as the fastest index: element
// (component c, site s, column col) at (c V + s) kc + col; kc in {1, 2, 4, 8, 16}.
// Per-column solver state K[col], history entries at j kc + col.
constexpr int kMaxBatch = 16;
bool batch_size_ok(int kc);
// Tile forms of the multi-RHS stencil (the `stage` argument of the batched
// launchers): 0 global neighbour reads in site order, 1 each block's tile
// staged in LDS, 2, 3 and 4 global reads with the sites visited in bricks of
// 8 x 8 x 4 x 4, 8 x 8 x 8 x 8 and 4 x 4 x 4 x 4 sites (full-lattice operator,
// extents divisible by the brick), 5 global reads in site order with the
// loads of several hops in flight (no fence between hops; full-lattice
// operator), 6 t-marching (boxes of sites walked through a chunk of time
// slices, the t neighbours in registers; full-lattice operator, a box of a
// whole number of blocks for k); < 0 the built-in rule (LDS staging for k = 1
// and for BF16).
constexpr int kTileForms = 7;
constexpr int kMarchTile = 6;
bool batch_tile_ok(const Geom &g, bool eo, int stage, int kc);
// Records (blocks) of a t-marching pass on kc columns (the form must fit).
int march_records(const Geom &g, int kc);
// The BiCG matvec pair (as launch_bicg_matvec) in the t-marching form with one
// column (full-lattice operator, batch_tile_ok(g, false, kMarchTile, 1)); it
// writes bicg_matvec_march_records(g, g5) sigma records.
void launch_bicg_matvec_march(double2 *Ap, double2 *Adp, const double2 *p, const double2 *ph, const double2 *U,
                              const Geom &g, double kappa, int j, KrylovState *S, const RedScratch &rs, bool g5,
                              hipStream_t st);
int bicg_matvec_march_records(const Geom &g, bool g5);
// stage: tile form of the batched stencils (kTileForms above)
template <typename S>
void launch_bdslash(S *out, const S *in, const S *U, const Geom &g, double kappa, bool dagger, int kc, hipStream_t st,
                    int stage = -1);
// rhat = p = r; rho_0, ||r_0|| per column; column col stops at once if ||r_0|| <= tol_abs[col] (device)
template <typename S>
void launch_bstab_init(S *rhat, S *p, const S *r, size_t N, int kc, const double *tol_abs, int maxiter,
                       KrylovState *K, KrylovHistory h, const RedScratch &rs, hipStream_t st);
template <typename S>
void launch_bstab_v(S *v, const S *p, const S *rhat, const S *U, const Geom &g, double kappa, int j, int kc,
                    KrylovState *K, const RedScratch &rs, hipStream_t st, int stage = -1);
// stage: the tile form of the v pass whose records this pass sums
template <typename S>
void launch_bstab_s(S *s, const S *r, const S *v, const Geom &g, int j, int kc, KrylovState *K, KrylovHistory h,
                    const RedScratch &rs, hipStream_t st, int stage);
template <typename S>
void launch_bstab_t(S *t, const S *s, const S *U, const Geom &g, double kappa, int j, int kc, KrylovState *K,
                    const RedScratch &rs, hipStream_t st, int stage = -1);
// stage: the tile form of the t pass whose records this pass sums
template <typename S>
void launch_bstab_xr(S *x, S *r, const S *p, const S *s, const S *t, const S *rhat, const Geom &g, int j, int kc,
                     KrylovState *K, KrylovHistory h, const RedScratch &rs, hipStream_t st, int stage);
template <typename S>
void launch_bstab_p(S *p, const S *r, const S *v, const Geom &g, int j, int kc, KrylovState *K, KrylovHistory h,
                    const RedScratch &rs, hipStream_t st);
// kc FP64 SoA columns (column col at src + col N) -> batch in storage S; x_col += batch column col
template <typename S>
void launch_pack_batch(S *dst, const double2 *src, size_t N, int kc, hipStream_t st);
template <typename S>
void launch_unpack_add_batch(double2 *x, const S *e, size_t N, int kc, hipStream_t st);
// canonical spinors back to back [kc][V][12] <-> batch
template <typename S>
void launch_to_batch(S *dst, const S *src, const Geom &g, int kc, hipStream_t st);
template <typename S>
void launch_from_batch(S *dst, const S *src, const Geom &g, int kc, hipStream_t st);

}  // namespace ebicg
