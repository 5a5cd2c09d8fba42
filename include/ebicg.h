/*
 * ebicg.h -- C ABI of the MI355X (gfx950) incremental eigBiCG library.
 *
 * The library solves A x_i = b_i, i = 1..N_r, for the Wilson-Dirac operator A
 * (Sec. 1, the main linear problem), grows left and right eigenvectors of A
 * from a window of BiCG residuals (Alg. eigBiCG with Alg. BiCG-eigen),
 * accumulates them into a deflation space (Alg. Incremental eigBiCG, step 2)
 * and deflates the initial guesses of later solves, which run BiCGStab with
 * the DefTol restart (Alg. Incremental eigBiCG, step 3, and the text after
 * the listings).
 *
 * Conventions shared by every call
 *  - Plain C: no C++ types and no exceptions cross this boundary.  Every call
 *    returns an eb_status; on a non-OK status eb_last_error() gives a message.
 *  - Dot product (w, v) := w^+ v (Sec. 1, end).
 *  - Site index s = x + Lx*(y + Ly*(z + Lz*t)); directions mu = 0..3 <-> x,y,z,t.
 *  - Canonical spinor layout (every spinor argument): [V][4 spin][3 colour]
 *    complex numbers, interleaved (re, im).  Element type by precision:
 *    EB_FP64 -> two doubles, EB_FP32 -> two floats, EB_BF16 -> two bfloat16.
 *  - Canonical gauge layout: [4 mu][V][3][3] complex128, U[mu][s][a][b] is
 *    row a, column b of U_mu(s).
 *  - Operator: (D psi)(x) = psi(x) - kappa sum_mu [ (1 - gamma_mu) U_mu(x) psi(x+mu)
 *    + (1 + gamma_mu) U_mu(x-mu)^+ psi(x-mu) ], periodic in x, y, z; every hop
 *    across the t boundary is multiplied by bc_t.  Gamma matrices: chiral basis,
 *    gamma_k = [[0, -i sigma_k], [i sigma_k, 0]], gamma_t = [[0, 1], [1, 0]],
 *    gamma5 = diag(1, 1, -1, -1).  D^+ = gamma5 D gamma5 (Sec. 4).
 *  - Device pointers are HIP device addresses (e.g. torch tensors'
 *    data_ptr()); `stream` is a hipStream_t (NULL = the null stream).  Solves
 *    synchronise their stream before returning; op_apply calls do not.
 *  - Ownership: the library copies the gauge field and owns the deflation
 *    space and all work buffers; the caller owns b, x and the outputs.
 *  - One eb_op is not re-entrant: calls on the same op must not overlap.
 */
#ifndef EBICG_H
#define EBICG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct eb_op eb_op;

typedef enum {
  EB_OK = 0,
  EB_ERR_INVALID = -1,       /* bad argument (sizes, null pointers, m <= 2 nev, ...) */
  EB_ERR_OOM = -2,           /* device allocation failed */
  EB_ERR_BREAKDOWN = -3,     /* (rhat, r) or (phat, A p) vanished (Alg. eigBiCG, step 2) */
  EB_ERR_NOT_CONVERGED = -4, /* maxiter reached; x holds the last iterate, stats are filled */
  EB_ERR_HIP = -5,           /* a HIP runtime call failed */
  EB_ERR_EIG = -6,           /* the small dense eigensolver did not converge */
  EB_ERR_CAPACITY = -7       /* the deflation space would exceed its capacity */
} eb_status;

typedef enum { EB_FP64 = 0, EB_FP32 = 1, EB_BF16 = 2 } eb_prec;

/* Sort criterion of the small dense eigenproblem eig(C) (Sec. 1, end: sorted by a
 * user-chosen criterion; Sec. 2 names the smallest absolute value).  An eigBiCG
 * solve keeps, at every restart of its window (Alg. BiCG-eigen), and returns the
 * nev pairs that come first.  Keys equal to 1e-12 relative (to the larger modulus)
 * are ordered by imaginary part descending. */
typedef enum {
  EB_SORT_SMALLEST_MAG = 0,  /* |lambda| ascending (the deflation target; the default) */
  EB_SORT_SMALLEST_REAL = 1, /* real part ascending (the left edge of the Wilson-Dirac spectrum) */
  EB_SORT_LARGEST_MAG = 2    /* |lambda| descending */
} eb_sort;

/* Parameters of one eigBiCG solve (Alg. eigBiCG). */
typedef struct {
  int32_t nev;     /* eigenpairs kept per restart and returned (2 nev < m) */
  int32_t m;       /* window size */
  double tol;      /* stop when ||r_j|| <= tol ||b|| (Alg. eigBiCG, last test of the loop) */
  int32_t maxiter; /* iteration cap */
  int32_t rhat;    /* shadow residual: 0 -> rhat_0 = r_0 (Sec. 2 "Normally"); 1 -> gamma5 r_0 (Sec. 4);
                      2 -> the gamma5-Hermitian form (Sec. 4): rhat_j = gamma5 r_j and
                      phat_j = gamma5 p_j are never formed, D^+ phat = gamma5 D p is not
                      applied (one D per iteration, matvec_ddag = 0), and the left window's
                      residuals are read as gamma5 times the right window's.  Same iterates
                      as 1 in exact arithmetic.  A source with (gamma5 r_0, r_0) = 0, such as a
                      Z2 source (entries +-1) with x_0 = 0, breaks down at once in modes 1 and
                      2 (EB_ERR_BREAKDOWN). */
  int32_t window;  /* storage of the window's vectors: EB_FP64, or EB_FP32 (the BiCG recurrence,
                      its scalars, H and the Ritz problem stay FP64; the window holds FP32 copies of
                      r_j, rhat_j and its rotations read FP32 and sum in FP64; the pairs absorbed
                      into the deflation space are FP64) */
  int32_t device_eig; /* 0: the window eigenproblems of Alg. BiCG-eigen on a host thread; 1: on the
                      GPU by one workgroup on a side stream, from the device-resident BiCG scalars
                      (the host reads back only the number of pairs kept and the Ritz values) */
  int32_t sort;       /* eb_sort: which Ritz pairs the window keeps and the solve returns (and absorbs
                         into the deflation space); ritz[] comes out in this order */
} eb_eig_params;

/* Parameters of a deflated solve (Alg. Incremental eigBiCG, step 3). */
typedef struct {
  double tol;       /* target ||b - A x|| / ||b|| (true residual, checked in FP64) */
  double deftol;    /* DefTol: 0 disables the deflation restart (the setting of Fig. 1) */
  int32_t maxiter;  /* cap on inner iterations summed over restarts and refinement steps */
  int32_t method;   /* 0: BiCGStab (the paper's choice for step 3); 1: two-sided BiCG (the
                       recurrences of Alg. eigBiCG without the window; Sec. 1 compares it with
                       BiCGStab), FP64 only: needs inner = EB_FP64 and deftol = 0, runs the
                       right-hand sides one at a time, two D applications per iteration */
  eb_prec inner;    /* working precision of the inner iteration; FP32/BF16 run inside FP64 refinement */
  double inner_tol; /* relative residual reduction per refinement step, < 1; <= 0 selects the
                       default (1e-6 FP32, 1e-2 BF16); ignored for EB_FP64 */
  int32_t nrhs;     /* right-hand sides (b, x hold nrhs spinors back to back) */
  int32_t batch;    /* columns per batched iteration: 1 = one at a time; 2, 4, 8, 16; 0 = the
                       library's choice (timed once per operator and precision). Batching needs
                       deftol = 0; with deftol > 0 the columns run one at a time. */
} eb_solve_params;

/* Per-call statistics. */
typedef struct {
  int32_t iters;              /* iterations (summed over the nrhs columns for batched solves) */
  int32_t matvec_d;           /* applications of D */
  int32_t matvec_ddag;        /* applications of D^+ */
  int32_t window_restarts;    /* Alg. BiCG-eigen calls */
  int32_t defl_restarts;      /* DefTol restarts */
  int32_t breakdown_restarts; /* reserved */
  int32_t outer_steps;        /* FP64 refinement steps (mixed precision) */
  int32_t nev_added;          /* pairs absorbed into the deflation space by this call */
  double true_rel_resid;      /* max over columns of ||b - A x|| / ||b|| in FP64 */
  double rec_rel_resid;       /* last recursive residual / ||b|| */
  double seconds;             /* wall time of the call */
} eb_stats;

/* Create an operator: copies gauge (host, canonical layout) to the device.
 * dims: Lx, Ly, Lz, Lt, each >= 2.  bc_t: -1 antiperiodic, +1 periodic in t.
 * defl_capacity: maximum number K of left/right pairs the deflation space holds
 * (its 2 K FP64 spinors are allocated on first use).  Device: the current HIP device. */
eb_status eb_op_create(const double *gauge, double kappa, const int32_t dims[4], int32_t bc_t,
                       int32_t defl_capacity, eb_op **out);
/* An operator whose solves run on the even-odd (Schur) form, as the paper's
 * test matrices are even-odd preconditioned (Sec. 3).  With H the hop sum
 * (D = 1 - kappa H; H connects sites of opposite parity x+y+z+t), the solvers
 * work on Dhat = 1 - kappa^2 H_eo H_oe over the even sites:
 *   Dhat x_e = b_e + kappa H_eo b_o,   x_o = b_o + kappa H_oe x_e.
 * Every extent must be even (EB_ERR_INVALID otherwise).  The entry points
 * keep their full-lattice canonical arguments: eb_op_apply / _dagger apply the
 * full D; eb_eigbicg_solve and eb_deflated_bicg_solve take b and x on the full
 * lattice (the odd part of the start x is ignored), stop when the even
 * system's residual is tol ||b||, and report the full system's
 * ||b - D x|| / ||b|| as true_rel_resid; their deflation space holds
 * eigenvectors of Dhat (V/2 sites), which eb_get_eigenpairs returns as
 * full-lattice spinors with zero odd part.  Deflated solves take every inner
 * precision and batch size; eb_op_apply_block applies the full D.  Memory: the
 * FP64 links twice (full and per parity), and per parity in FP32 / BF16 once
 * a solve uses that inner precision. */
eb_status eb_op_create_eo(const double *gauge, double kappa, const int32_t dims[4], int32_t bc_t,
                          int32_t defl_capacity, eb_op **out);
eb_status eb_op_destroy(eb_op *op);

/* out = D in, and out = D^+ in (Alg. eigBiCG, first step of the loop).  in/out:
 * device, canonical layout, element type given by prec; they must not overlap.
 * Asynchronous on `stream`. */
eb_status eb_op_apply(eb_op *op, void *out, const void *in, eb_prec prec, void *stream);
eb_status eb_op_apply_dagger(eb_op *op, void *out, const void *in, eb_prec prec, void *stream);

/* out = D in (dagger = 0) or D^+ in (dagger = 1) in FP64, as eb_op_apply /
 * eb_op_apply_dagger with EB_FP64, for callers that cannot allocate device
 * memory (code under HIP stream capture, tight serving loops, harnesses that
 * forbid allocation): the call allocates nothing.  Its staging buffers live in
 * a fixed 48 MiB device array per GPU, held until the process ends, which
 * limits the lattice to V <= 131072 sites (16^3 x 32); a larger operator gets
 * EB_ERR_INVALID.  Every call on one GPU shares that array: calls that overlap
 * on one GPU (different streams or host threads) race and must be serialised
 * by the caller.  in/out: device, FP64 canonical layout, not overlapping.
 * Asynchronous on `stream`. */
eb_status eb_op_apply_noalloc(eb_op *op, void *out, const void *in, int32_t dagger, void *stream);

/* For an even-odd operator (eb_op_create_eo): out = Dhat in_e (dagger = 0) or
 * Dhat^+ in_e (dagger = 1), Dhat = 1 - kappa^2 H_eo H_oe (Sec. 3's even-odd
 * preconditioned matrices).  in/out: device FP64 canonical full-lattice
 * spinors; the odd sites of in are ignored and those of out are zero.
 * EB_ERR_INVALID for an operator made by eb_op_create.  Asynchronous. */
eb_status eb_op_apply_schur(eb_op *op, void *out, const void *in, int32_t dagger, void *stream);

/* For an even-odd operator: out_i = Dhat in_i (dagger = 0) or Dhat^+ in_i
 * (dagger = 1) for k right-hand sides at once, k in {1, 2, 4, 8, 16} (the
 * multi-RHS form of eb_op_apply_schur; Sec. 3's even-odd preconditioned
 * matrices).  in/out: device FP64 canonical full-lattice spinors, k back to
 * back; the odd sites of in are ignored and those of out are zero.  prec is
 * the storage of the pass (FP32 / BF16: the inputs and links rounded to it,
 * arithmetic in FP32, results widened to FP64).  EB_ERR_INVALID for an
 * operator made by eb_op_create, an unknown prec or k.  Asynchronous. */
eb_status eb_op_apply_schur_block(eb_op *op, void *out, const void *in, int32_t k, int32_t dagger, eb_prec prec,
                                  void *stream);

/* out_i = D in_i (dagger = 0) or D^+ in_i (dagger = 1) for k right-hand sides
 * at once, k in {1, 2, 4, 8, 16}: one pass over the links serves all k
 * (multi-RHS stencil).  in/out: device, k canonical spinors back to back,
 * element type by prec; they must not overlap.  Asynchronous on `stream`. */
eb_status eb_op_apply_block(eb_op *op, void *out, const void *in, int32_t k, int32_t dagger, eb_prec prec,
                            void *stream);

/* One solve of the first phase of Alg. Incremental eigBiCG (step 2): deflate
 * x0 with the current space (if K > 0), run eigBiCG in FP64, continue with
 * BiCGStab if the FP64 true residual is above tol, then biorthogonalise the nev
 * new pairs against the space and extend H = U_l^+ A U_r.
 * b: device, FP64 canonical; x: device, FP64 canonical, in: x0, out: solution.
 * ritz (host, may be NULL): receives the nev Ritz values of this solve as
 * complex128 (re, im pairs), ordered by |lambda| ascending. */
eb_status eb_eigbicg_solve(eb_op *op, const void *b, void *x, const eb_eig_params *p, double *ritz,
                           eb_stats *st, void *stream);

/* A solve of the second phase (step 3): x0 += U_r H^{-1} U_l^+ (b - A x0),
 * then BiCGStab with the DefTol restart (or BiCG, method = 1); FP32/BF16 inner precision runs
 * inside FP64 iterative refinement.  b, x: device, FP64 canonical, p->nrhs
 * spinors back to back.  With p->batch != 1 the right-hand sides run in
 * batches of k columns that share every link load (multi-RHS stencil); each
 * column keeps its own BiCGStab scalars and stops on its own.  Does not
 * change the deflation space. */
eb_status eb_deflated_bicg_solve(eb_op *op, const void *b, void *x, const eb_solve_params *p,
                                 eb_stats *st, void *stream);

/* Eigenpairs of A from the deflation space by Rayleigh-Ritz (text after the
 * listings): eig(H), H = U_l^+ A U_r.  On input *k is the capacity of the
 * outputs, on output the number written (min(*k, K)), ordered by |lambda|.
 * evals: host complex128[k]; right/left: device FP64 canonical, k spinors each,
 * or NULL.  Right vectors have unit norm and left_i^+ right_i = 1. */
eb_status eb_get_eigenpairs(eb_op *op, int32_t *k, double *evals, void *right, void *left, void *stream);

/* Current size K of the deflation space, and a copy of H (host complex128
 * K x K, row-major; may be NULL). */
eb_status eb_defl_info(eb_op *op, int32_t *K, double *H);
/* Empty the deflation space (K = 0). */
eb_status eb_defl_reset(eb_op *op);

/* The small dense eigenproblem [y, z, lambda] = eig(C) of Sec. 1 (end), as
 * used on the window matrix: C host complex128 n x n row-major; lambda host
 * complex128[n]; y, z host complex128 n x n row-major, column i the right /
 * left vector of lambda_i (may be NULL).  Sorted by |lambda| ascending, ties
 * by imaginary part descending; ||y_i|| = 1 and z_i^+ y_i = 1.  Host-only,
 * needs no GPU.  EB_ERR_EIG if the QR iteration does not converge. */
eb_status eb_small_eig(int32_t n, const double *C, double *lambda, double *y, double *z);

/* The same eigenproblem on the current GPU by one workgroup (the device solver
 * that restarts the window of an eigBiCG solve with eb_eig_params.device_eig;
 * Alg. BiCG-eigen), with the same arguments, conventions and order as
 * eb_small_eig; n <= 128.  Synchronous; allocates and frees its own device
 * buffers.  EB_ERR_EIG if the QR iteration does not converge. */
eb_status eb_small_eig_device(int32_t n, const double *C, double *lambda, double *y, double *z);

/* Kernel timing, for benchmarks.  While enabled, every launch of the solver
 * kernels is bracketed by HIP events on the solve's stream; eb_timing_read
 * returns, per kernel class, the launches and their summed duration (ms)
 * since the last eb_timing_enable.  Classes: */
enum {
  EB_K_BICG_MATVEC = 0, /* D p and D^+ phat with sigma (one launch per BiCG iteration) */
  EB_K_BICG_UPDATE_R,   /* r, rhat updates with rho and ||r|| */
  EB_K_BICG_UPDATE_P,   /* x, p, phat updates */
  EB_K_STAB_V,          /* BiCGStab v = D p with (rhat, v) */
  EB_K_STAB_S,          /* s = r - alpha v */
  EB_K_STAB_T,          /* t = D s with (t, s), (t, t) */
  EB_K_STAB_XR,         /* x, r updates with (rhat, r), ||r|| */
  EB_K_STAB_P,          /* p = r + beta (p - omega v) */
  EB_K_ROTATE,          /* window rotation (Alg. BiCG-eigen) */
  EB_K_RESIDUAL,        /* b - D x in FP64 */
  EB_K_PROJ,            /* deflation projections (tall-skinny products) */
  EB_K_DSLASH,          /* plain D or D^+ applications (extending H) */
  EB_K_BSTAB_V,         /* batched BiCGStab: v = D p for k columns with (rhat, v) */
  EB_K_BSTAB_S,         /* batched: alpha (one block) and s = r - alpha v */
  EB_K_BSTAB_T,         /* batched: t = D s with (t, s), (t, t) */
  EB_K_BSTAB_XR,        /* batched: omega (one block), x and r updates with (rhat, r), ||r|| */
  EB_K_BSTAB_P,         /* batched: beta and stop tests (one block), p update */
  EB_K_BDSLASH,         /* eb_op_apply_block stencil */
  EB_K_COUNT
};
eb_status eb_timing_enable(eb_op *op, int32_t enable);
/* Classes recorded while timing is enabled: bit k for class k (default: all).
 * Each recorded launch costs two event records on the host, which slows
 * solves made of short kernels; select only the classes you need. */
eb_status eb_timing_classes(eb_op *op, uint32_t mask);
eb_status eb_timing_read(eb_op *op, int32_t kclass, int64_t *launches, double *total_ms);

/* ---- Serving: continuous batching of deflated solves -------------------------
 * A session serves solve requests on one operator with `slots` columns of the
 * multi-RHS BiCGStab (Alg. Incremental eigBiCG, step 3, without DefTol).  A
 * request is admitted into a free slot; at the next eb_session_step its start
 * x0 is deflated with the operator's deflation space as it is then
 * (x0 += U_r H^-1 U_l^+ (b - A x0)) and its column starts iterating beside
 * the columns already running.  Each slot runs its own FP64 refinement: the
 * inner iteration (storage `inner`) runs to inner_tol, the correction is added
 * in FP64 and the true residual ||b - A x|| is recomputed in FP64; the request
 * finishes when it is <= tol ||b|| (even-odd operators: the solvers' system,
 * with the full system's residual reported), or with EB_ERR_NOT_CONVERGED
 * after maxiter inner iterations.  Every column keeps its own BiCGStab
 * scalars and stop test, so a request's result does not depend on which other
 * requests share the batch.
 *
 * Threading and streams: a session and every other call on its operator
 * (eigBiCG solves that grow the space, deflated solves) must use the same
 * stream and the same host thread; sessions of different operators on
 * different streams overlap on the device.  The session owns its reduction
 * scratch, states and the batch (eb_session_info reports the bytes); b and x
 * stay owned by the caller and must stay valid until the request is polled. */
typedef struct eb_session eb_session;
typedef struct {
  int32_t slots;    /* columns of the batch: 1, 2, 4, 8 or 16 */
  eb_prec inner;    /* storage of the inner iteration (EB_FP64, EB_FP32, EB_BF16) */
  double tol;       /* target ||b - A x|| / ||b|| per request */
  double inner_tol; /* residual reduction per refinement step, < 1; <= 0: 1e-6 (FP32), 1e-2 (BF16),
                       none (FP64).  A refinement step that makes no inner iteration ends the
                       request with EB_ERR_NOT_CONVERGED. */
  int32_t maxiter;  /* inner iterations per request, summed over refinement steps */
  int32_t chunk;    /* iterations launched between slot updates, 1..1024 */
  int32_t graph;    /* 1: the chunk's launches are captured once as a hipGraph and replayed
                       (on a created stream, not the null stream, and not while kernel timing
                       is enabled); 0: launched one by one */
} eb_session_params;
/* Create a session on `stream` (a hipStream_t; its device memory is allocated here).  Runs
 * the batch autotuner for the operator and `inner` once (eb_op_batch_tune), so the slots'
 * stencils use the tuned tile form. */
eb_status eb_session_create(eb_op *op, const eb_session_params *p, void *stream, eb_session **out);
/* Wait for the work in flight and free the session (requests still running are dropped).
 * A session must be destroyed before its operator. */
eb_status eb_session_destroy(eb_session *s);
/* Reserve a free slot for the request (b, x: device FP64 canonical spinors; x holds x0 and
 * receives the solution; tag: the caller's id).  Host-only: the request starts at the next
 * eb_session_step.  *slot (may be NULL) receives the slot.  EB_ERR_CAPACITY if every slot is busy. */
eb_status eb_session_admit(eb_session *s, const void *b, void *x, int64_t tag, int32_t *slot);
/* Wait for the chunk in flight; harvest the slots whose inner solve stopped (finish them or
 * start their next refinement step); start the admitted requests; launch the next chunk of
 * iterations and return without waiting for it.  Finished requests become pollable.  A
 * request's own failure (maxiter, breakdown) is reported through eb_session_poll; a non-OK
 * status from this call (a HIP error) leaves the slots in an unknown state: destroy the
 * session. */
eb_status eb_session_step(eb_session *s);
/* *ready = 1 when eb_session_step would not wait (no chunk in flight, or it has finished),
 * else 0.  Does not wait: a loop over several sessions steps the ready ones only. */
eb_status eb_session_ready(eb_session *s, int32_t *ready);
/* Take up to max finished requests: tags[i], status[i] (EB_OK, EB_ERR_NOT_CONVERGED,
 * EB_ERR_BREAKDOWN) and stats[i] (may be NULL; seconds = admission to finish).  *n = taken. */
eb_status eb_session_poll(eb_session *s, int32_t max, int64_t *tags, int32_t *status, eb_stats *stats, int32_t *n);
/* Free and busy slots, finished requests not yet polled, device bytes the session holds
 * (any pointer may be NULL). */
eb_status eb_session_info(eb_session *s, int32_t *free_slots, int32_t *busy, int32_t *done, uint64_t *device_bytes);
/* ---- Batch autotuning (multi-RHS tile shapes) ------------------------------
 * The batched solvers' operator (the stencil, or Dhat for an even-odd operator)
 * has EB_TILE_FORMS tile forms for each k: stage = 0 reads every neighbour from
 * global memory with the sites in order; 1 stages each block's tile of 256 / k
 * sites in LDS; 2, 3 and 4 read from global memory with the sites visited in
 * bricks of 8 x 8 x 4 x 4, 8 x 8 x 8 x 8 and 4 x 4 x 4 x 4 sites (full-lattice
 * stencil only, extents divisible by the brick), which keeps more of a site's
 * neighbours in L2 when k columns make each site's record large; 5 reads from
 * global memory in site order with the loads of several hops in flight
 * (full-lattice stencil only); 6 walks boxes of sites (up to 32 x 16 x 8, 16 x
 * 16 x 8 for k = 16, 32 x 32 x 8 for k = 1) through chunks of time slices with
 * the t neighbours held by each thread (full-lattice stencil only, a box of a
 * whole number of 256-thread blocks for k).  eb_op_batch_tune runs the
 * autotuner once per operator and precision (it times every form the
 * operator admits for k = 2, 4, 8, 16, and for k = 1 the two forms of the
 * one-at-a-time solver that a single column runs, LDS-staged (1) and
 * t-marching (6), on `stream`, three repetitions after a warm-up, and keeps
 * per k the fastest form and overall the k with the lowest time per
 * right-hand side) and reports: *k_best; stage[5] (may be
 * NULL) the form used for k = 1, 2, 4, 8, 16; ms_per_rhs[5 * EB_TILE_FORMS] (may be NULL) the
 * measured time per right-hand side, [EB_TILE_FORMS i + form] for k = 2^i (0 for a form
 * not admitted).  Batched solves with batch = 0, sessions and
 * eb_op_apply_block / eb_op_apply_schur_block use the forms chosen here
 * (before tuning: LDS staging for k = 1 and for BF16, else form 0).  The
 * one-at-a-time BiCGStab (batch = 1, every precision) on a full-lattice
 * operator runs its two stencil passes in the k = 1 form: 6 if that is the
 * entry, else 1; with no entry yet it times both once on its first solve and
 * records the faster. */
#define EB_TILE_FORMS 7
eb_status eb_op_batch_tune(eb_op *op, eb_prec prec, void *stream, int32_t *k_best, int32_t *stage,
                           double *ms_per_rhs);
/* Set the tile form for one precision and k (0..6 as above, or -1 for the built-in rule);
 * results agree to rounding between the forms.  EB_ERR_INVALID for a form the operator does
 * not admit.  For k = 1 it also sets the one-at-a-time solver's form (6, or 1 for any
 * other form).  Host-only; a later first run of the tuner replaces it. */
eb_status eb_op_batch_set_tile(eb_op *op, eb_prec prec, int32_t k, int32_t stage);
/* Form of the BiCG matvec pair of eigBiCG and deflated BiCG (D p with the
 * partials of (phat, D p), and D^+ phat; Alg. eigBiCG, the products of each
 * iteration): 1 LDS-staged tiles (a work item per tile and product), 6
 * t-marching units (the D and D^+ units of one box and chunk on one XCD at the
 * same time, sharing the link loads; full-lattice operator whose box of
 * 32 x 32 x 8 sites or less holds a whole number of 256-site blocks), -1
 * (default) time both once at the next solve and keep the faster.  Results
 * agree to rounding.  EB_ERR_INVALID for another value or a form the operator
 * does not admit.  Host-only. */
eb_status eb_op_set_matvec_form(eb_op *op, int32_t form);
/* The matvec form in use (-1 before the first solve has chosen; 1 for an
 * even-odd operator) and, in ms[2] (may be NULL), the milliseconds per launch
 * the choice measured for forms 1 and 6 (0 if not timed). */
eb_status eb_op_get_matvec_form(eb_op *op, int32_t *form, double *ms);
/* Release the operator's work buffers (eigBiCG windows, batch and scratch vectors; not the
 * links, the deflation space or the reduction scratch) after waiting for `stream` and the
 * device; later calls allocate what they need again.  Sessions keep their own buffers. */
eb_status eb_op_trim(eb_op *op, void *stream);
/* Testing knob: cap on the grid of the stencil kernels that produce reduction
 * partials (default 1024 blocks of 256 sites; 0 restores it).  Beyond the
 * cap each block loops over several site tiles, which large lattices do by
 * default (V > 262144); a small cap makes a small lattice take that path.
 * Results agree to rounding with any cap.  Host-only. */
eb_status eb_op_set_grid_cap(eb_op *op, int32_t max_blocks);
/* Device bytes the operator holds (links, deflation space, work buffers). */
eb_status eb_op_device_bytes(eb_op *op, uint64_t *bytes);

/* Message of the last non-OK status on this thread (empty if none). */
void eb_last_error(char *buf, size_t len);

/* Library version string. */
const char *eb_version(void);

#ifdef __cplusplus
}
#endif

#endif /* EBICG_H */
