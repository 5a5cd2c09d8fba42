// C ABI of the library (include/ebicg.h): operator creation, D / D^+
// application, eigBiCG solves that grow the deflation space, deflated
// BiCGStab solves (FP64, or FP32 inner inside FP64 refinement), and the
// Rayleigh-Ritz eigenpairs of the space.
//
// Host-side orchestration only: every vector operation runs in kernels.hip.
// The BiCG scalars stay on the device; the host polls a stop flag every few
// iterations and, for eigBiCG, assembles the window matrix H from the scalar
// history (Alg. eigBiCG: H needs no extra matvecs) in a worker thread, so the
// m x m eigenproblems of Alg. BiCG-eigen overlap the GPU iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/ebicg.h"
#include "hostla.h"
#include "kernels.h"
#include "slot.h"

using namespace ebicg;

namespace {

thread_local std::string g_last_error;

struct EbError {
  eb_status code;
  std::string msg;
};

[[noreturn]] void fail(eb_status code, const std::string &msg) { throw EbError{code, msg}; }

void hipchk(hipError_t e, const char *what) {
  if (e != hipSuccess) fail(EB_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}
#define HIPCHK(expr) hipchk((expr), #expr)

template <typename F>
eb_status guarded(F &&f) {
  try {
    f();
    g_last_error.clear();
    return EB_OK;
  } catch (const EbError &e) {
    g_last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc &) {
    g_last_error = "host allocation failed";
    return EB_ERR_OOM;
  } catch (const std::exception &e) {
    g_last_error = e.what();
    return EB_ERR_INVALID;
  }
}

inline double2 d2(cd z) { return make_double2(z.real(), z.imag()); }
inline cd c2(double2 z) { return cd(z.x, z.y); }

// Device allocation owned by the op.
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  void ensure(size_t b) {
    if (b <= bytes) return;
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    if (hipMalloc(&p, b) != hipSuccess) {
      p = nullptr;
      fail(EB_ERR_OOM, "hipMalloc of " + std::to_string(b) + " bytes failed");
    }
    bytes = b;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <typename T>
  T *as() const {
    return static_cast<T *>(p);
  }
};

struct PinnedBuf {
  void *p = nullptr;
  size_t bytes = 0;
  void ensure(size_t b) {
    if (b <= bytes) return;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
    if (hipHostMalloc(&p, b, hipHostMallocDefault) != hipSuccess) fail(EB_ERR_OOM, "hipHostMalloc failed");
    bytes = b;
  }
  void release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <typename T>
  T *as() const {
    return static_cast<T *>(p);
  }
};

}  // namespace

// ============================================================================
// the operator object
// ============================================================================
struct eb_op {
  Geom g{};
  size_t N = 0;  // length of the solvers' spinors: 12 V, or 12 V / 2 for an even-odd operator
  bool eo = false;  // the solvers run on the even-site Schur complement (eo.hip)
  DevBuf Ueo;       // its links, [parity][4][9][V/2]
  DevBuf Ueo32, Ueo16;  // and FP32 / BF16 copies made on first use
  double kappa = 0;
  int bc_t = -1;
  int device = 0;
  int grid_cap = kDefaultStencilCap;  // grid cap of the reducing stencil kernels (eb_op_set_grid_cap)
  hipStream_t side = nullptr;         // side stream of the device window restarts (default priority)
  DevBuf U64, U32, U16;  // links: FP64, and FP32 / BF16 copies made on first use
  // deflation space: Ul, Ur hold Kcap FP64 SoA spinors each; H = Ul^+ A Ur on the host
  int Kcap = 0, K = 0;
  DevBuf Ul, Ur;
  CMat H;
  // reduction scratch and solver state
  DevBuf partials, state, res, hist;
  int hist_cap = 0;
  PinnedBuf hstate, hres, hhist;
  PinnedBuf hpoll;                          // stop-flag polling (Poller)
  // multi-RHS: chosen columns per batch per precision (0: not tuned yet) and
  // the measured stencil time per right-hand side of each candidate
  int batch_choice[3] = {0, 0, 0};
  // form of the BiCG matvec pair: 1 LDS-staged tiles, kMarchTile t-marching
  // boxes, -1 not chosen yet (timed at the next solve); matvec_ms[form]
  int matvec_form = -1;
  // grid cap of the staged pair, chosen with its form (0: grid_cap)
  int matvec_cap = 0;
  // grid cap of the staged one-column BiCGStab passes per storage (FP64, FP32,
  // BF16), chosen with the k = 1 form (0: grid_cap)
  int stab_cap[3] = {0, 0, 0};
  double matvec_ms[kTileForms] = {};
  double batch_ms[3][kMaxBatch + 1] = {};
  // tile form of the batched stencils per precision and k (1: LDS-staged
  // tile, 0: global neighbour reads, -1: the built-in rule), chosen by the
  // tuner or set by the caller; the tuner's time per right-hand side (ms) of
  // each form
  int batch_stage[3][kMaxBatch + 1];
  double batch_stage_ms[3][kMaxBatch + 1][kTileForms] = {};
  static_assert(kTileForms == EB_TILE_FORMS, "the header counts the tile forms");
  eb_op() {
    for (auto &row : batch_stage)
      for (int &v : row) v = -1;
  }
  hipEvent_t poll_ev[2] = {nullptr, nullptr};
  std::map<std::string, DevBuf> bufs;
  // kernel timing (eb_timing_enable, eb_timing_classes)
  bool timing = false;
  uint32_t timing_mask = ~0u;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  struct TimedLaunch {
    int cls;
    hipEvent_t a, b;
  };
  std::vector<TimedLaunch> pending;
  int64_t t_launch[EB_K_COUNT] = {};
  double t_ms[EB_K_COUNT] = {};
  hipEvent_t next_event() {
    if (ev_used == ev_pool.size()) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e));
      ev_pool.push_back(e);
    }
    return ev_pool[ev_used++];
  }
  void flush_timing() {
    for (auto &t : pending) {
      HIPCHK(hipEventSynchronize(t.b));
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, t.a, t.b));
      t_launch[t.cls] += 1;
      t_ms[t.cls] += ms;
    }
    pending.clear();
    ev_used = 0;
  }
  RedScratch rs() { return RedScratch{partials.as<double>()}; }
  KrylovState *S() { return state.as<KrylovState>(); }
  double2 *vec(const std::string &name, size_t count = 1) {
    DevBuf &b = bufs[name];
    b.ensure(count * N * sizeof(double2));
    return b.as<double2>();
  }
  template <typename T>
  T *raw(const std::string &name, size_t bytes) {
    DevBuf &b = bufs[name];
    b.ensure(bytes);
    return b.as<T>();
  }
  KrylovHistory history(int need) {
    if (need > hist_cap) {
      hist_cap = std::max(need, 2 * hist_cap);
      size_t bytes = size_t(hist_cap) * (4 * sizeof(double2) + sizeof(double));
      hist.release();
      hist.ensure(bytes);
      hhist.release();
      hhist.ensure(bytes);
    }
    return view(hist.p);
  }
  KrylovHistory view(void *base) const {
    char *b = static_cast<char *>(base);
    KrylovHistory h;
    h.alpha = reinterpret_cast<double2 *>(b);
    h.beta = reinterpret_cast<double2 *>(b + size_t(hist_cap) * sizeof(double2));
    h.rho = reinterpret_cast<double2 *>(b + 2 * size_t(hist_cap) * sizeof(double2));
    h.omega = reinterpret_cast<double2 *>(b + 3 * size_t(hist_cap) * sizeof(double2));
    h.rn = reinterpret_cast<double *>(b + 4 * size_t(hist_cap) * sizeof(double2));
    return h;
  }
  void free_all() {
    if (side) (void)hipStreamDestroy(side);
    side = nullptr;
    U64.release();
    Ueo.release();
    Ueo32.release();
    Ueo16.release();
    U32.release();
    U16.release();
    Ul.release();
    Ur.release();
    partials.release();
    state.release();
    res.release();
    hist.release();
    hstate.release();
    hres.release();
    hhist.release();
    hpoll.release();
    for (auto &e : poll_ev) {
      if (e) (void)hipEventDestroy(e);
      e = nullptr;
    }
    for (auto &kv : bufs) kv.second.release();
    bufs.clear();
    pending.clear();
    for (auto e : ev_pool) (void)hipEventDestroy(e);
    ev_pool.clear();
  }
};

namespace {

// Every entry point starts here: the operator's device, and its grid cap for
// the stencil launches this thread makes.
void set_device(eb_op *op) {
  HIPCHK(hipSetDevice(op->device));
  stencil_block_cap() = op->grid_cap;
}

// Launch through `f`, bracketed by timing events when the op records kernel times.
template <typename F>
void timed(eb_op *op, int cls, hipStream_t s, F &&f) {
  if (!op->timing || !((op->timing_mask >> cls) & 1u)) {
    f();
    return;
  }
  if (op->pending.size() > 16384) op->flush_timing();
  hipEvent_t a = op->next_event(), b = op->next_event();
  struct Stamp {  // kernel-stamped events for the launches inside f
    LaunchStamp &ls;
    Stamp(hipEvent_t a, hipEvent_t b) : ls(launch_stamp()) { ls = LaunchStamp{a, b, false}; }
    ~Stamp() { ls = LaunchStamp{}; }
  } stamp(a, b);
  f();
  if (!stamp.ls.started) {  // nothing launched: an empty interval
    HIPCHK(hipEventRecord(a, s));
    HIPCHK(hipEventRecord(b, s));
  }
  op->pending.push_back({cls, a, b});
}
#define TIMED(cls, stream, call) timed(op, cls, stream, [&]() { call; })

void fetch_state(eb_op *op, hipStream_t s, KrylovState &out) {
  HIPCHK(hipMemcpyAsync(op->hstate.p, op->state.p, sizeof(KrylovState), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  out = *op->hstate.as<KrylovState>();
}

// Watches the device stop flag without draining the queue: each step() first
// waits for the copy issued at the previous step (poll interval iterations
// ago), then issues a new one.
struct Poller {
  const KrylovState *dev = nullptr;
  hipStream_t s = nullptr;
  int n = 1;                    // states watched (the columns of a batch)
  KrylovState *host = nullptr;  // two pinned slots of kMaxBatch states, owned by the op
  hipEvent_t *ev = nullptr;     // two events owned by the op
  int issued = 0;
  Poller(eb_op *op, const KrylovState *d, hipStream_t st, int nstates = 1);
  ~Poller() {
    if (issued > 0) (void)hipEventSynchronize(ev[(issued - 1) & 1]);
  }
  // true once every watched state has stopped; then out[0..n) holds them
  bool step(KrylovState *out) {
    if (issued > 0) {
      const int k = (issued - 1) & 1;
      HIPCHK(hipEventSynchronize(ev[k]));
      const KrylovState *h = host + size_t(k) * kMaxBatch;
      bool all = true;
      for (int c = 0; c < n; ++c) all = all && h[c].stopped;
      if (all) {
        for (int c = 0; c < n; ++c) out[c] = h[c];
        return true;
      }
    }
    const int k = issued & 1;
    HIPCHK(hipMemcpyAsync(host + size_t(k) * kMaxBatch, dev, n * sizeof(KrylovState), hipMemcpyDeviceToHost, s));
    HIPCHK(hipEventRecord(ev[k], s));
    ++issued;
    return false;
  }
};
Poller::Poller(eb_op *op, const KrylovState *d, hipStream_t st, int nstates) : dev(d), s(st), n(nstates) {
  if (!op->poll_ev[0]) {
    op->hpoll.ensure(2 * kMaxBatch * sizeof(KrylovState));
    HIPCHK(hipEventCreateWithFlags(&op->poll_ev[0], hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&op->poll_ev[1], hipEventDisableTiming));
  }
  host = op->hpoll.as<KrylovState>();
  ev = op->poll_ev;
}

// The operator of the solvers: the Wilson D, or for an even-odd operator the
// Schur complement Dhat on the even sites (one odd-site scratch spinor).
// residual_launch writes {||r||^2, ||b||^2} to op->res[2 slot], slot < kMaxBatch.
void residual_launch(eb_op *op, double2 *r, const double2 *b, const double2 *x, hipStream_t s, int slot = 0) {
  double *res = op->res.as<double>() + 2 * slot;
  if (op->eo)
    launch_residual_eo(r, b, x, op->vec("eo_tmp"), op->Ueo.as<double2>(), op->g, op->kappa, res, op->rs(), s);
  else
    launch_residual_f64(r, b, x, op->U64.as<double2>(), op->g, op->kappa, res, op->rs(), s);
}
// The geometry the vector passes of the batched BiCGStab see: they use only
// the site count, V/2 for the even-odd form.
Geom vector_geom(const eb_op *op) {
  Geom g = op->g;
  if (op->eo) g.V /= 2;
  return g;
}
void apply64(eb_op *op, double2 *out, const double2 *in, bool dagger, hipStream_t s) {
  if (op->eo)
    launch_schur_eo(out, in, op->vec("eo_tmp"), op->Ueo.as<double2>(), op->g, op->kappa, dagger, s);
  else
    launch_dslash_f64(out, in, op->U64.as<double2>(), op->g, op->kappa, dagger, s);
}

// r = b - A x in FP64; returns (||r||, ||b||).
std::pair<double, double> residual(eb_op *op, double2 *r, const double2 *b, const double2 *x, hipStream_t s) {
  TIMED(EB_K_RESIDUAL, s, residual_launch(op, r, b, x, s));
  HIPCHK(hipMemcpyAsync(op->hres.p, op->res.p, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const double *h = op->hres.as<double>();
  return {std::sqrt(h[0]), std::sqrt(h[1])};
}

// x <- x + U_r d with H d = U_l^+ (b - A x)  (Alg. Incremental eigBiCG, step 2
// first item and step 3 first item).  Returns ||b - A x|| before the update.
double deflate_guess(eb_op *op, const double2 *b, double2 *x, hipStream_t s) {
  double2 *r = op->vec("defl_r");
  auto [rn, bn] = residual(op, r, b, x, s);
  (void)bn;
  if (op->K == 0) return rn;
  const int K = op->K;
  double2 *c = op->raw<double2>("defl_c", size_t(K) * sizeof(double2));
  TIMED(EB_K_PROJ, s, launch_ts_dot(c, op->Ul.as<double2>(), op->N, K, r, op->N, 1, op->N, op->rs(), s));
  std::vector<double2> hc(K);
  HIPCHK(hipMemcpyAsync(hc.data(), c, K * sizeof(double2), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  std::vector<cd> d(K);
  for (int i = 0; i < K; ++i) d[i] = c2(hc[i]);
  if (!lu_solve(op->H, d)) fail(EB_ERR_EIG, "deflation matrix H is singular");
  for (int i = 0; i < K; ++i) hc[i] = d2(d[i]);
  HIPCHK(hipMemcpyAsync(c, hc.data(), K * sizeof(double2), hipMemcpyHostToDevice, s));
  TIMED(EB_K_PROJ, s, launch_ts_update(x, op->N, 1, op->Ur.as<double2>(), op->N, K, c, 1.0, op->N, s));
  HIPCHK(hipStreamSynchronize(s));
  return rn;
}

// ---------------------------------------------------------------------------
// BiCGStab driver (storage S).  Solves A x = b from the current x with the
// given residual r = b - A x already in `r`; stops on convergence
// (||r|| <= tol_abs), on the DefTol threshold, on breakdown or maxiter.
// ---------------------------------------------------------------------------
struct StabResult {
  int iters = 0;
  int reason = 0;
  double rnorm = 0;
};

// Time of the one-column t pass (t = D s with its dots) in tile form
// `stage`: 1 the LDS-staged pass at grid cap `cap` (0: the operator's),
// kMarchTile the t-marching walk; one launch, then the mean of three.
template <typename S>
double one_column_pass_ms(eb_op *op, const S *U, const S *src, S *dst, int stage, int cap, hipStream_t s,
                          hipEvent_t e0, hipEvent_t e1) {
  stencil_block_cap() = cap > 0 ? cap : op->grid_cap;
  KrylovHistory none{};
  auto run = [&]() {  // j = 0: no stop flag of an earlier solve skips it
    if (stage == kMarchTile)
      launch_bstab_t<S>(dst, src, U, op->g, op->kappa, 0, 1, op->S(), op->rs(), s, kMarchTile);
    else
      launch_stab_t<S>(dst, src, U, op->g, op->kappa, 0, op->S(), none, op->rs(), s);
  };
  run();
  HIPCHK(hipEventRecord(e0, s));
  for (int rep = 0; rep < 3; ++rep) run();
  HIPCHK(hipEventRecord(e1, s));
  HIPCHK(hipEventSynchronize(e1));
  float ms = 0;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  stencil_block_cap() = op->grid_cap;
  return ms / 3.0;
}

// The k = 1 entry of the tuning table for storage index pi on a full-lattice
// operator, from the solver's own t pass (D alone misleads: at 32^3 x 64 the
// staged D runs 701 us against 510 us marching, while the staged t pass runs
// 492 us against 571): the staged pass at the operator's grid cap, the staged
// pass with one tile per block (unless a test set the cap; up to the 32 768
// blocks whose records fill a region), and the t-marching walk.  The fastest
// goes into batch_stage[pi][1] with its cap in stab_cap[pi]; the times into
// batch_stage_ms[pi][1] (the staged entry: its faster grid).
template <typename S>
void tune_one_column(eb_op *op, int pi, const S *U, const S *src, S *dst, hipStream_t s) {
  struct Cand {
    int stage, cap;
  };
  std::vector<Cand> cands{{1, 0}};
  if (op->grid_cap == kDefaultStencilCap) cands.push_back({1, int(kRegionDoubles / 4)});
  if (batch_tile_ok(op->g, false, kMarchTile, 1)) cands.push_back({kMarchTile, 0});
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  op->batch_stage_ms[pi][1][1] = op->batch_stage_ms[pi][1][kMarchTile] = 0.0;
  op->batch_stage[pi][1] = 1;
  op->stab_cap[pi] = 0;
  double best = HUGE_VAL;
  for (const Cand &cd : cands) {
    const double t = one_column_pass_ms<S>(op, U, src, dst, cd.stage, cd.cap, s, e0, e1);
    double &slot = op->batch_stage_ms[pi][1][cd.stage];
    if (slot == 0.0 || t < slot) slot = t;
    if (t < best) {
      best = t;
      op->batch_stage[pi][1] = cd.stage;
      op->stab_cap[pi] = cd.cap;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

// Stencil form of the one-column BiCGStab on a full-lattice operator: the
// LDS-staged passes (1) or the t-marching walk (kMarchTile), whichever the
// k = 1 entry of the batch tuning table names, timed on the t pass
// (tune_one_column) when the table has none.  A staged choice with a wider
// grid becomes this entry point's stencil cap, so the records each pass
// writes and the count its consumer sums stay the same.  Even-odd operators
// run Dhat (form 1).
template <typename S>
int single_stab_form(eb_op *op, const S *U, const S *src, S *dst, hipStream_t s) {
  if (op->eo) return 1;
  const int pi = std::is_same<S, double2>::value ? 0 : (std::is_same<S, float2>::value ? 1 : 2);
  if (op->batch_stage[pi][1] < 0) tune_one_column<S>(op, pi, U, src, dst, s);
  const int f = op->batch_stage[pi][1];
  if (f == 1 && op->stab_cap[pi] > 0) stencil_block_cap() = op->stab_cap[pi];
  return f == kMarchTile ? kMarchTile : 1;
}

// Form of the BiCG matvec pair (D p with sigma, D^+ phat) on a full-lattice
// operator: the LDS-staged work items or the t-marching units, as set, or
// else timed once (three launches each after one, on the solve's p, phat and
// product buffers, before its first iteration) and the fastest kept.  The
// staged pair is timed at the operator's grid cap and, unless a test set
// that cap, also with one tile per block, as many as the sigma record region
// holds: at 24^3 x 64 that
// grid ran the pair in 392 against 473-489 us, at 32^3 x 64 it was slower
// (995-1037 against 925-954 us).  A chosen wider grid is made this entry
// point's stencil cap, so the records the matvec writes and the count its
// consumer sums stay the same.  Even-odd operators run Dhat.
int bicg_matvec_form(eb_op *op, double2 *Ap, double2 *Adp, const double2 *p, const double2 *ph, KrylovState *S,
                     hipStream_t s) {
  if (op->eo) return 1;
  if (op->matvec_form < 0) {
    op->matvec_form = 1;
    op->matvec_cap = 0;
    if (batch_tile_ok(op->g, false, kMarchTile, 1)) {
      hipEvent_t e0, e1;
      HIPCHK(hipEventCreate(&e0));
      HIPCHK(hipEventCreate(&e1));
      double best = HUGE_VAL;
      const double2 *U = op->U64.as<double2>();
      KrylovHistory none{};
      // one tile per block up to the blocks whose sigma records (two per tile
      // in the general form, of two doubles each) fill a record region; on
      // lattices of at most kDefaultStencilCap tiles this is the same grid
      const int wide = int(kRegionDoubles / 4);
      struct Cand {
        int form, cap;
      };
      std::vector<Cand> cands{{1, 0}};
      if (op->grid_cap == kDefaultStencilCap) cands.push_back({1, wide});
      cands.push_back({kMarchTile, 0});
      op->matvec_ms[1] = op->matvec_ms[kMarchTile] = 0.0;
      for (const Cand &cd : cands) {
        stencil_block_cap() = cd.cap > 0 ? cd.cap : op->grid_cap;
        auto run = [&]() {  // j = 0: no stop flag of an earlier solve skips it
          if (cd.form == kMarchTile)
            launch_bicg_matvec_march(Ap, Adp, p, ph, U, op->g, op->kappa, 0, S, op->rs(), false, s);
          else
            launch_bicg_matvec(Ap, Adp, p, ph, U, op->g, op->kappa, 0, S, none, op->rs(), false, s);
        };
        run();
        HIPCHK(hipEventRecord(e0, s));
        for (int rep = 0; rep < 3; ++rep) run();
        HIPCHK(hipEventRecord(e1, s));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        double &slot = op->matvec_ms[cd.form];  // the staged pair: its faster grid
        if (slot == 0.0 || ms / 3.0 < slot) slot = ms / 3.0;
        if (ms < best) {
          best = ms;
          op->matvec_form = cd.form;
          op->matvec_cap = cd.cap;
        }
      }
      stencil_block_cap() = op->grid_cap;
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
    }
  }
  if (op->matvec_form == 1 && op->matvec_cap > 0) stencil_block_cap() = op->matvec_cap;
  return op->matvec_form;
}

template <typename S>
StabResult run_bicgstab(eb_op *op, const S *U, S *x, S *r, double tol_abs, double def_thr, int maxiter,
                        const std::string &tag, hipStream_t s) {
  const size_t N = op->N;
  S *rhat = op->raw<S>(tag + "rhat", N * sizeof(S));
  S *p = op->raw<S>(tag + "p", N * sizeof(S));
  S *v = op->raw<S>(tag + "v", N * sizeof(S));
  S *sv = op->raw<S>(tag + "s", N * sizeof(S));
  S *t = op->raw<S>(tag + "t", N * sizeof(S));
  KrylovState *K = op->S();
  KrylovHistory h = op->history(maxiter + 4);
  const int form = single_stab_form<S>(op, U, r, v, s);
  const int nrec = form == kMarchTile ? march_records(op->g, 1) : 0;
  launch_stab_init<S>(rhat, p, r, N, tol_abs, def_thr, maxiter, K, h, op->rs(), s);
  KrylovState hs;
  fetch_state(op, s, hs);
  StabResult out;
  if (hs.stopped) {
    out.reason = hs.reason;
    out.rnorm = hs.rnorm;
    return out;
  }
  // v = A p and t = A s with their dots: the Wilson stencil, or Dhat (U then
  // holds the even-odd links in storage S, and tmp is an odd-site scratch)
  S *tmp = op->eo ? op->raw<S>(tag + "eo_tmp", N * sizeof(S)) : nullptr;
  auto stab_v = [&](int j) {
    if (op->eo)
      launch_stab_v_eo<S>(v, p, rhat, tmp, U, op->g, op->kappa, j, K, op->rs(), s);
    else if (form == kMarchTile)
      launch_bstab_v<S>(v, p, rhat, U, op->g, op->kappa, j, 1, K, op->rs(), s, kMarchTile);
    else
      launch_stab_v<S>(v, p, rhat, U, op->g, op->kappa, j, K, h, op->rs(), s);
  };
  auto stab_t = [&](int j) {
    if (op->eo)
      launch_stab_t_eo<S>(t, sv, tmp, U, op->g, op->kappa, j, K, op->rs(), s);
    else if (form == kMarchTile)
      launch_bstab_t<S>(t, sv, U, op->g, op->kappa, j, 1, K, op->rs(), s, kMarchTile);
    else
      launch_stab_t<S>(t, sv, U, op->g, op->kappa, j, K, h, op->rs(), s);
  };
  const int poll = 8;
  int j = 0;
  bool stopped = false;
  {
    Poller pl(op, K, s);
    while (j < maxiter) {
      ++j;
      TIMED(EB_K_STAB_V, s, stab_v(j));
      TIMED(EB_K_STAB_S, s, launch_stab_s<S>(sv, r, v, N, j, K, h, op->rs(), s, nrec));
      TIMED(EB_K_STAB_T, s, stab_t(j));
      TIMED(EB_K_STAB_XR, s, launch_stab_xr<S>(x, r, p, sv, t, rhat, N, j, K, h, op->rs(), s, nrec));
      TIMED(EB_K_STAB_P, s, launch_stab_p<S>(p, r, v, N, j, K, h, op->rs(), s));
      if (j % poll == 0 && pl.step(&hs)) {
        stopped = true;
        break;
      }
    }
  }
  if (!stopped) fetch_state(op, s, hs);
  out.iters = hs.stopped ? hs.stop_at : j;
  out.reason = hs.stopped ? hs.reason : 4;
  out.rnorm = hs.rnorm;
  return out;
}

// FP64 BiCGStab with the DefTol deflation restarts and the true-residual
// check; x is the (already deflated) start.  Accumulates into st.
void deflated_stab_f64(eb_op *op, const double2 *b, double2 *x, double tol, double deftol, int maxiter,
                       eb_stats &st, hipStream_t s) {
  double2 *r = op->vec("stab_r");
  double thr_factor = deftol;
  while (true) {
    auto [rn, bn] = residual(op, r, b, x, s);
    st.matvec_d += 1;
    if (bn == 0.0) {
      HIPCHK(hipMemsetAsync(x, 0, op->N * sizeof(double2), s));
      st.true_rel_resid = 0;
      return;
    }
    st.true_rel_resid = rn / bn;
    if (rn <= tol * bn) return;
    int left = maxiter - st.iters;
    if (left <= 0) fail(EB_ERR_NOT_CONVERGED, "deflated solve: maxiter reached");
    const double def_thr = (op->K > 0 && deftol > 0) ? thr_factor * bn : 0.0;
    const double2 *U = op->eo ? op->Ueo.as<double2>() : op->U64.as<double2>();
    StabResult R = run_bicgstab<double2>(op, U, x, r, tol * bn, def_thr, left, "f64_", s);
    st.iters += R.iters;
    st.matvec_d += 2 * R.iters;
    st.rec_rel_resid = R.rnorm / bn;
    if (R.reason == 2) fail(EB_ERR_BREAKDOWN, "BiCGStab breakdown");
    if (R.reason == 3) {
      deflate_guess(op, b, x, s);
      st.defl_restarts += 1;
      thr_factor *= deftol;
    }
  }
}

// Deflated two-sided BiCG (method 1), FP64: the BiCG recurrences of Alg.
// eigBiCG without the window (the paper's Sec. 1 discusses BiCG beside
// BiCGStab), with the shadow residual rhat_0 = r_0 of the (already deflated)
// start x.  Two D applications per iteration (D p and D^+ phat); the scalars
// stay on the device as in eigBiCG, with the same breakdown tests.  A solve
// whose FP64 true residual is still above tol after the recursion stopped
// restarts BiCG from x (reading of the listing's convergence test), until tol
// or maxiter.  Accumulates into st.
void deflated_bicg_f64(eb_op *op, const double2 *b, double2 *x, double tol, int maxiter, eb_stats &st,
                       hipStream_t s) {
  const size_t N = op->N;
  double2 *r0 = op->vec("bicg1_r", 2), *rh0 = op->vec("bicg1_rh", 2);
  double2 *r[2] = {r0, r0 + N}, *rh[2] = {rh0, rh0 + N};
  double2 *p = op->vec("bicg_p"), *ph = op->vec("bicg_ph");
  double2 *Ap = op->vec("bicg_Ap"), *Adp = op->vec("bicg_Adp");
  KrylovState *S = op->S();
  while (true) {
    // r_0 = b - A x (FP64) with ||r||^2, ||b||^2 in op->res
    TIMED(EB_K_RESIDUAL, s, residual_launch(op, r[0], b, x, s));
    st.matvec_d += 1;
    double hres[2];
    HIPCHK(hipMemcpyAsync(hres, op->res.p, sizeof(hres), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const double rn = std::sqrt(hres[0]), bn = std::sqrt(hres[1]);
    if (bn == 0.0) {
      HIPCHK(hipMemsetAsync(x, 0, N * sizeof(double2), s));
      st.true_rel_resid = 0;
      return;
    }
    st.true_rel_resid = rn / bn;
    if (rn <= tol * bn) return;
    const int left = maxiter - st.iters;
    if (left <= 0) fail(EB_ERR_NOT_CONVERGED, "deflated BiCG: maxiter reached");
    KrylovHistory dh = op->history(left + 4);
    launch_bicg_init(rh[0], p, ph, r[0], op->res.as<double>(), N, 0, op->g, tol, left, S, dh, op->rs(), s);
    KrylovState hs;
    fetch_state(op, s, hs);
    if (hs.stopped && hs.reason == 2) fail(EB_ERR_BREAKDOWN, "BiCG: (rhat_0, r_0) = 0");
    int j = 0;
    bool stopped = hs.stopped != 0;
    const int mvf = stopped ? 1 : bicg_matvec_form(op, Ap, Adp, p, ph, S, s);
    const int nsig = mvf == kMarchTile ? bicg_matvec_march_records(op->g, false) : 0;
    {
      Poller pl(op, S, s);
      while (!stopped && j < left) {
        ++j;
        const int cur = j & 1, prv = cur ^ 1;
        TIMED(EB_K_BICG_MATVEC, s,
              op->eo ? launch_bicg_matvec_eo(Ap, Adp, p, ph, op->vec("eo_tmp"), op->Ueo.as<double2>(), op->g,
                                             op->kappa, j, S, op->rs(), false, s)
              : mvf == kMarchTile
                  ? launch_bicg_matvec_march(Ap, Adp, p, ph, op->U64.as<double2>(), op->g, op->kappa, j, S,
                                             op->rs(), false, s)
                  : launch_bicg_matvec(Ap, Adp, p, ph, op->U64.as<double2>(), op->g, op->kappa, j, S, dh,
                                       op->rs(), false, s));
        TIMED(EB_K_BICG_UPDATE_R, s,
              launch_bicg_update_r(r[cur], rh[cur], r[prv], rh[prv], Ap, Adp, N, j, S, dh, op->rs(), false, s,
                                   nullptr, nullptr, nsig));
        TIMED(EB_K_BICG_UPDATE_P, s, launch_bicg_update_p(x, p, ph, r[cur], rh[cur], N, j, S, dh, op->rs(), false, s));
        if (j % 8 == 0 && pl.step(&hs)) stopped = true;
      }
    }
    if (!stopped || !hs.stopped) fetch_state(op, s, hs);
    const int done = hs.stopped ? hs.stop_at : j;
    st.iters += done;
    st.matvec_d += done;
    st.matvec_ddag += done;
    st.rec_rel_resid = hs.rnorm / bn;
    // a breakdown before any update cannot be cured by restarting from the same x
    if (hs.stopped && hs.reason == 2 && done == 0) fail(EB_ERR_BREAKDOWN, "BiCG breakdown");
  }
}

// Storage of the inner solve: FP64 (no refinement needed, one outer step),
// FP32, or BF16 with FP32 arithmetic.
template <typename S>
struct Inner;
template <>
struct Inner<double2> {
  static constexpr const char *tag = "f64_";
  static constexpr int index = 0;
  static const double2 *links(eb_op *op, hipStream_t) { return op->U64.as<double2>(); }
  // the links of the operator the solvers run on (even-odd: per parity)
  static const double2 *solver_links(eb_op *op, hipStream_t s) {
    return op->eo ? op->Ueo.as<double2>() : links(op, s);
  }
  static void down(double2 *d, const double2 *x, size_t n, hipStream_t s) { launch_copy_f64(d, x, n, s); }
  static void up(double2 *d, const double2 *x, size_t n, hipStream_t s) { launch_copy_f64(d, x, n, s); }
};
template <>
struct Inner<float2> {
  static constexpr const char *tag = "f32_";
  static constexpr int index = 1;
  static const float2 *links(eb_op *op, hipStream_t s) {
    if (!op->U32.p) {
      op->U32.ensure(size_t(36) * op->g.V * sizeof(float2));
      launch_convert_f64_f32(op->U32.as<float2>(), op->U64.as<double2>(), size_t(36) * op->g.V, s);
    }
    return op->U32.as<float2>();
  }
  static const float2 *solver_links(eb_op *op, hipStream_t s) {
    if (!op->eo) return links(op, s);
    if (!op->Ueo32.p) {
      op->Ueo32.ensure(size_t(36) * op->g.V * sizeof(float2));
      launch_convert_f64_f32(op->Ueo32.as<float2>(), op->Ueo.as<double2>(), size_t(36) * op->g.V, s);
    }
    return op->Ueo32.as<float2>();
  }
  static void down(float2 *d, const double2 *x, size_t n, hipStream_t s) { launch_convert_f64_f32(d, x, n, s); }
  static void up(double2 *d, const float2 *x, size_t n, hipStream_t s) { launch_convert_f32_f64(d, x, n, s); }
};
template <>
struct Inner<bf16c> {
  static constexpr const char *tag = "bf16_";
  static constexpr int index = 2;
  static const bf16c *links(eb_op *op, hipStream_t s) {
    if (!op->U16.p) {
      op->U16.ensure(size_t(36) * op->g.V * sizeof(bf16c));
      launch_convert_f64_bf16(op->U16.as<bf16c>(), op->U64.as<double2>(), size_t(36) * op->g.V, s);
    }
    return op->U16.as<bf16c>();
  }
  static const bf16c *solver_links(eb_op *op, hipStream_t s) {
    if (!op->eo) return links(op, s);
    if (!op->Ueo16.p) {
      op->Ueo16.ensure(size_t(36) * op->g.V * sizeof(bf16c));
      launch_convert_f64_bf16(op->Ueo16.as<bf16c>(), op->Ueo.as<double2>(), size_t(36) * op->g.V, s);
    }
    return op->Ueo16.as<bf16c>();
  }
  static void down(bf16c *d, const double2 *x, size_t n, hipStream_t s) { launch_convert_f64_bf16(d, x, n, s); }
  static void up(double2 *d, const bf16c *x, size_t n, hipStream_t s) { launch_convert_bf16_f64(d, x, n, s); }
};

// Low-precision inner BiCGStab inside FP64 iterative refinement (defect
// correction): every outer step computes r = b - A x in FP64, solves A e = r
// in storage S to a relative reduction inner_tol and adds e to x in FP64.
// Global reductions and scalars stay FP64 in every kernel.  The initial guess
// is deflated once by the caller (Alg. Incremental eigBiCG, step 3); the
// refinement steps are not deflated again: the oblique projector
// I - A U_r H^-1 U_l^+ is not a contraction when the Ritz pairs are poor, and
// applying it to every small correction residual can undo the inner solve.
template <typename S>
void mixed_stab(eb_op *op, const double2 *b, double2 *x, double tol, double inner_tol, int maxiter, eb_stats &st,
                hipStream_t s) {
  const size_t N = op->N;
  const S *U = Inner<S>::solver_links(op, s);
  const std::string tag = Inner<S>::tag;
  double2 *r = op->vec("mix_r");
  double2 *e64 = op->vec("mix_e64");
  S *rl = op->raw<S>(tag + "mix_r", N * sizeof(S));
  S *el = op->raw<S>(tag + "mix_e", N * sizeof(S));
  int outer = 0;
  while (true) {
    auto [rn, bn] = residual(op, r, b, x, s);
    st.matvec_d += 1;
    if (bn == 0.0) {  // b = 0: the solution is x = 0
      HIPCHK(hipMemsetAsync(x, 0, N * sizeof(double2), s));
      st.true_rel_resid = 0;
      return;
    }
    st.true_rel_resid = rn / bn;
    if (rn <= tol * bn) return;
    int left = maxiter - st.iters;
    if (left <= 0 || outer > 200) fail(EB_ERR_NOT_CONVERGED, "mixed-precision solve: maxiter reached");
    Inner<S>::down(rl, r, N, s);
    HIPCHK(hipMemsetAsync(el, 0, N * sizeof(S), s));
    // inner target: reduce this residual by inner_tol, but not below what FP64 needs
    const double inner_abs = std::max(inner_tol * rn, 0.5 * tol * bn);
    StabResult R = run_bicgstab<S>(op, U, el, rl, inner_abs, 0.0, left, tag, s);
    st.iters += R.iters;
    st.matvec_d += 2 * R.iters;
    if (R.reason == 2 && R.iters == 0) fail(EB_ERR_BREAKDOWN, "inner BiCGStab breakdown");
    Inner<S>::up(e64, el, N, s);
    launch_add_f64(x, e64, N, s);
    ++outer;
    st.outer_steps = outer;
  }
}

// ---------------------------------------------------------------------------
// Multi-RHS: kc right-hand sides solved together (batch layout of batch.hip)
// ---------------------------------------------------------------------------
// Deflate the initial guesses of kc FP64 columns at once (Alg. Incremental
// eigBiCG, step 3, first item): C = U_l^+ R on the matrix cores, H D = C on
// the host, X += U_r D on the matrix cores.
void deflate_block(eb_op *op, const double2 *b, double2 *x, int kc, hipStream_t s) {
  if (op->K == 0) return;
  const size_t N = op->N;
  const int K = op->K;
  double2 *r = op->vec("dfb_r", kc);
  for (int c = 0; c < kc; ++c) TIMED(EB_K_RESIDUAL, s, residual_launch(op, r + c * N, b + c * N, x + c * N, s, c));
  double2 *C = op->raw<double2>("dfb_c", size_t(K) * kc * sizeof(double2));
  TIMED(EB_K_PROJ, s, launch_ts_dot(C, op->Ul.as<double2>(), N, K, r, N, kc, N, op->rs(), s));
  std::vector<double2> hc(size_t(K) * kc);
  HIPCHK(hipMemcpyAsync(hc.data(), C, hc.size() * sizeof(double2), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int c = 0; c < kc; ++c) {
    std::vector<cd> d(K);
    for (int i = 0; i < K; ++i) d[i] = c2(hc[i + size_t(c) * K]);
    if (!lu_solve(op->H, d)) fail(EB_ERR_EIG, "deflation matrix H is singular");
    for (int i = 0; i < K; ++i) hc[i + size_t(c) * K] = d2(d[i]);
  }
  HIPCHK(hipMemcpyAsync(C, hc.data(), hc.size() * sizeof(double2), hipMemcpyHostToDevice, s));
  TIMED(EB_K_PROJ, s, launch_ts_update(x, N, kc, op->Ur.as<double2>(), N, K, C, 1.0, N, s));
  HIPCHK(hipStreamSynchronize(s));
}

// Columns per batch for the multi-RHS path: timed once per operator and
// precision.  Each candidate k runs the batched operator of the solvers (the
// stencil, or Dhat) on k columns (three timed repetitions after one warm-up);
// the k with the lowest time per right-hand side wins.  Ties go to the smaller
// k (less memory, earlier exit of converged columns).
template <typename S>
int tune_batch(eb_op *op, hipStream_t s) {
  const S *U = Inner<S>::solver_links(op, s);
  const size_t n = op->N * size_t(kMaxBatch);
  const std::string tag = Inner<S>::tag;
  S *a = op->raw<S>(tag + "b_p", n * sizeof(S));
  S *b = op->raw<S>(tag + "b_v", n * sizeof(S));
  S *tmp = op->eo ? op->raw<S>(tag + "b_eo_tmp", n * sizeof(S)) : nullptr;
  auto apply = [&](int kc, int stage) {
    if (op->eo)
      launch_bschur_eo<S>(b, a, tmp, U, op->g, op->kappa, false, kc, s, stage);
    else
      launch_bdslash<S>(b, a, U, op->g, op->kappa, false, kc, s, stage);
  };
  HIPCHK(hipMemsetAsync(a, 0, n * sizeof(S), s));
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  int best = 1;
  double best_t = HUGE_VAL;
  const int pi = Inner<S>::index;
  for (int kc = 1; kc <= kMaxBatch; kc *= 2) {
    double t_kc = HUGE_VAL;
    if (kc == 1 && !op->eo) {  // one column runs the one-at-a-time solver: its own pass
      tune_one_column<S>(op, pi, U, a, b, s);
      t_kc = op->batch_stage_ms[pi][1][op->batch_stage[pi][1]];
      op->batch_ms[pi][kc] = t_kc;
      best_t = t_kc;
      continue;
    }
    for (int stage = 0; stage < kTileForms; ++stage) {  // every tile form this operator admits
      if (!batch_tile_ok(op->g, op->eo, stage, kc)) continue;
      // one column runs the one-at-a-time solver, whose stencils take the
      // LDS-staged or the t-marching form: time k = 1 in those
      if (kc == 1 && stage != 1 && stage != kMarchTile) continue;
      apply(kc, stage);
      HIPCHK(hipEventRecord(e0, s));
      for (int rep = 0; rep < 3; ++rep) apply(kc, stage);
      HIPCHK(hipEventRecord(e1, s));
      HIPCHK(hipEventSynchronize(e1));
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      const double per_rhs = ms / (3.0 * kc);
      op->batch_stage_ms[pi][kc][stage] = per_rhs;
      if (per_rhs < t_kc) {
        t_kc = per_rhs;
        op->batch_stage[pi][kc] = stage;
      }
    }
    op->batch_ms[pi][kc] = t_kc;
    if (t_kc < 0.97 * best_t) {
      best_t = t_kc;
      best = kc;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return best;
}

int choose_batch(eb_op *op, eb_prec prec, hipStream_t s) {
  const int i = prec == EB_FP64 ? 0 : (prec == EB_FP32 ? 1 : 2);
  if (op->batch_choice[i] == 0)
    op->batch_choice[i] = i == 0 ? tune_batch<double2>(op, s) : (i == 1 ? tune_batch<float2>(op, s) : tune_batch<bf16c>(op, s));
  return op->batch_choice[i];
}

// Batched BiCGStab in storage S on kc interleaved columns: x, r are batches,
// tol_dev the per-column absolute targets (device).  Returns when every
// column has stopped; iters[c] = iterations of column c, reason[c] its stop.
template <typename S>
void run_bicgstab_batch(eb_op *op, const S *U, S *x, S *r, int kc, const double *tol_dev, int maxiter,
                        const std::string &tag, hipStream_t s, int *iters, int *reason) {
  const size_t n = op->N * size_t(kc);
  S *rhat = op->raw<S>(tag + "b_rhat", n * sizeof(S));
  S *p = op->raw<S>(tag + "b_p", n * sizeof(S));
  S *v = op->raw<S>(tag + "b_v", n * sizeof(S));
  S *sv = op->raw<S>(tag + "b_s", n * sizeof(S));
  S *t = op->raw<S>(tag + "b_t", n * sizeof(S));
  S *tmp = op->eo ? op->raw<S>(tag + "b_eo_tmp", n * sizeof(S)) : nullptr;
  const Geom gv = vector_geom(op);
  KrylovState *K = op->S();
  KrylovHistory h = op->history((maxiter + 4) * kc);
  const int stage = op->batch_stage[Inner<S>::index][kc];
  launch_bstab_init<S>(rhat, p, r, op->N, kc, tol_dev, maxiter, K, h, op->rs(), s);
  KrylovState hs[kMaxBatch];
  const int poll = 8;
  int j = 0;
  bool stopped = false;
  {
    Poller pl(op, K, s, kc);
    pl.step(hs);  // a batch whose columns all stop at once needs no iteration
    while (j < maxiter) {
      if (j % poll == 0 && j > 0 && pl.step(hs)) {
        stopped = true;
        break;
      }
      ++j;
      if (op->eo)
        TIMED(EB_K_BSTAB_V, s,
              launch_bstab_v_eo<S>(v, p, rhat, tmp, U, op->g, op->kappa, j, kc, K, op->rs(), s, stage));
      else
        TIMED(EB_K_BSTAB_V, s, launch_bstab_v<S>(v, p, rhat, U, op->g, op->kappa, j, kc, K, op->rs(), s, stage));
      TIMED(EB_K_BSTAB_S, s, launch_bstab_s<S>(sv, r, v, gv, j, kc, K, h, op->rs(), s, stage));
      if (op->eo)
        TIMED(EB_K_BSTAB_T, s,
              launch_bstab_t_eo<S>(t, sv, tmp, U, op->g, op->kappa, j, kc, K, op->rs(), s, stage));
      else
        TIMED(EB_K_BSTAB_T, s, launch_bstab_t<S>(t, sv, U, op->g, op->kappa, j, kc, K, op->rs(), s, stage));
      TIMED(EB_K_BSTAB_XR, s, launch_bstab_xr<S>(x, r, p, sv, t, rhat, gv, j, kc, K, h, op->rs(), s, stage));
      TIMED(EB_K_BSTAB_P, s, launch_bstab_p<S>(p, r, v, gv, j, kc, K, h, op->rs(), s));
    }
  }
  if (!stopped) {
    HIPCHK(hipMemcpyAsync(op->hstate.p, K, kc * sizeof(KrylovState), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int c = 0; c < kc; ++c) hs[c] = op->hstate.as<KrylovState>()[c];
  }
  for (int c = 0; c < kc; ++c) {
    iters[c] = hs[c].stopped ? hs[c].stop_at : j;
    reason[c] = hs[c].stopped ? hs[c].reason : 4;
  }
}

// kc right-hand sides (FP64 SoA columns b, x; x holds the deflated start):
// FP64 iterative refinement around one batched low-precision BiCGStab per
// outer step; column c stops at ||r_c|| <= tol[c] ||b_c||.  Columns that have
// converged keep a target of +inf (they stop at initialisation and their
// correction stays zero).
template <typename S>
void mixed_stab_batch(eb_op *op, const double2 *b, double2 *x, int kc, const double *tol, double inner_tol,
                      int maxiter, eb_stats &st, hipStream_t s) {
  const size_t N = op->N;
  const S *U = Inner<S>::solver_links(op, s);
  const std::string tag = Inner<S>::tag;
  double2 *r = op->vec("mb_r", kc);
  S *rl = op->raw<S>(tag + "mb_r", N * kc * sizeof(S));
  S *el = op->raw<S>(tag + "mb_e", N * kc * sizeof(S));
  double *tol_dev = op->raw<double>("mb_tol", kMaxBatch * sizeof(double));
  double *tol_host = op->hres.as<double>();  // pinned; reused after the residual norms are read
  int outer = 0;
  std::vector<double> rn(kc), bn(kc);
  while (true) {
    for (int c = 0; c < kc; ++c)
      TIMED(EB_K_RESIDUAL, s, residual_launch(op, r + c * N, b + c * N, x + c * N, s, c));
    HIPCHK(hipMemcpyAsync(op->hres.p, op->res.p, 2 * kc * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    st.matvec_d += kc;
    bool all = true;
    double worst = 0;
    for (int c = 0; c < kc; ++c) {
      rn[c] = std::sqrt(op->hres.as<double>()[2 * c]);
      bn[c] = std::sqrt(op->hres.as<double>()[2 * c + 1]);
      if (bn[c] == 0.0 && rn[c] > 0.0) {  // b = 0: the solution is x = 0
        HIPCHK(hipMemsetAsync(x + c * N, 0, N * sizeof(double2), s));
        rn[c] = 0.0;
      }
      const double rel = bn[c] > 0 ? rn[c] / bn[c] : 0.0;
      worst = std::max(worst, rel);
      all = all && rel <= tol[c];
    }
    st.true_rel_resid = worst;
    if (all) return;
    int left = maxiter - st.iters / kc;
    if (left <= 0 || outer > 200) fail(EB_ERR_NOT_CONVERGED, "batched mixed-precision solve: maxiter reached");
    for (int c = 0; c < kc; ++c)
      tol_host[c] =
          (bn[c] == 0 || rn[c] <= tol[c] * bn[c]) ? HUGE_VAL : std::max(inner_tol * rn[c], 0.5 * tol[c] * bn[c]);
    HIPCHK(hipMemcpyAsync(tol_dev, tol_host, kc * sizeof(double), hipMemcpyHostToDevice, s));
    launch_pack_batch<S>(rl, r, N, kc, s);
    HIPCHK(hipMemsetAsync(el, 0, N * kc * sizeof(S), s));
    int it[kMaxBatch], why[kMaxBatch];
    run_bicgstab_batch<S>(op, U, el, rl, kc, tol_dev, left, tag, s, it, why);
    bool progress = false;
    for (int c = 0; c < kc; ++c) {
      st.iters += it[c];
      st.matvec_d += 2 * it[c];
      progress = progress || it[c] > 0;
    }
    if (!progress) fail(EB_ERR_BREAKDOWN, "batched inner BiCGStab made no progress");
    launch_unpack_add_batch<S>(x, el, N, kc, s);
    ++outer;
    st.outer_steps = outer;
  }
}

// ---------------------------------------------------------------------------
// eigBiCG (Alg. eigBiCG with Alg. BiCG-eigen), FP64
// ---------------------------------------------------------------------------
// A window column: a stored BiCG residual (raw r_i in V, raw rhat_i in W) or a
// Ritz vector written by a restart.  Stored residuals carry their scale in H's
// coefficients: v = r_i / ||r_i||, w = (||r_i|| / conj(rho_i)) rhat_i.
struct Col {
  int ritz;  // 1: Ritz column k of the current block, 0: residual
  int idx;   // Ritz index, or the iteration i of r_i
  int slot;  // physical slot (-1: placeholder of a pending restart)
};

// The latest applied restart: its Ritz values and the raw arrow dots.
struct RitzBlock {
  int jr = 0;  // restart iteration
  std::vector<cd> lam;
  std::vector<cd> dV, dW;  // GA^+ V_new[:,k] and W_new[:,k]^+ GB
};

struct HostHist {
  const double2 *alpha, *beta, *rho;
  const double *rn;
};

// H^(n) of the window described by cols (Alg. eigBiCG, H assembly steps;
// arrow entries from the dots of the last restart).
CMat build_H(const std::vector<Col> &cols, const HostHist &h, const RitzBlock &rb) {
  const int n = int(cols.size());
  CMat H(n, n);
  for (int c = 0; c < n; ++c) {
    const Col &C = cols[c];
    if (C.ritz) {
      H(c, c) = rb.lam[C.idx];
      continue;
    }
    const int i = C.idx;
    cd d = 1.0 / c2(h.alpha[i]);
    if (i >= 1) d += c2(h.beta[i - 1]) / c2(h.alpha[i - 1]);
    H(c, c) = d;
    if (c + 1 < n && !cols[c + 1].ritz) {
      const cd a = c2(h.alpha[i]), be = c2(h.beta[i]);
      H(c, c + 1) = -(h.rn[i] / h.rn[i + 1]) * be / a;
      H(c + 1, c) = -(h.rn[i + 1] / h.rn[i]) / a;
    }
    if (c > 0 && cols[c - 1].ritz) {
      // first residual after the Ritz block: the arrow row and column
      const double rn = h.rn[i];
      const cd rho = c2(h.rho[i]);
      for (int k = 0; k < c; ++k) {
        const int rk = cols[k].idx;
        H(c, k) = (rn / rho) * rb.dV[rk];
        H(k, c) = rb.dW[rk] / rn;
      }
    }
  }
  return H;
}

// Two-sided Gram-Schmidt (twice) of columns start.. of Y, Z against the
// earlier ones (which satisfy Z^+ Y = I); pairs with a tiny pivot are dropped.
void biorth_coeff(CMat &Y, CMat &Z, int start) {
  const int n = Y.rows;
  std::vector<std::vector<cd>> ys, zs;
  for (int k = 0; k < start; ++k) {
    ys.emplace_back(Y.col(k), Y.col(k) + n);
    zs.emplace_back(Z.col(k), Z.col(k) + n);
  }
  for (int k = start; k < Y.cols; ++k) {
    std::vector<cd> y(Y.col(k), Y.col(k) + n), z(Z.col(k), Z.col(k) + n);
    for (int pass = 0; pass < 2; ++pass)
      for (size_t q = 0; q < ys.size(); ++q) {
        cd a = 0, b = 0;
        for (int i = 0; i < n; ++i) {
          a += std::conj(zs[q][i]) * y[i];
          b += std::conj(ys[q][i]) * z[i];
        }
        for (int i = 0; i < n; ++i) {
          y[i] -= ys[q][i] * a;
          z[i] -= zs[q][i] * b;
        }
      }
    cd piv = 0;
    double ny = 0, nz = 0;
    for (int i = 0; i < n; ++i) {
      piv += std::conj(z[i]) * y[i];
      ny += std::norm(y[i]);
      nz += std::norm(z[i]);
    }
    ny = std::sqrt(ny);
    nz = std::sqrt(nz);
    if (std::abs(piv) <= 1e-12 * ny * nz) continue;
    for (auto &e : y) e /= ny;
    piv /= ny;
    for (auto &e : z) e /= std::conj(piv);
    ys.push_back(y);
    zs.push_back(z);
  }
  const int kept = int(ys.size());
  CMat Yo(n, kept), Zo(n, kept);
  for (int k = 0; k < kept; ++k)
    for (int i = 0; i < n; ++i) {
      Yo(i, k) = ys[k][i];
      Zo(i, k) = zs[k][i];
    }
  Y = Yo;
  Z = Zo;
}

// Column scales of the stored vectors: V = V_stored diag(eta), W = W_stored diag(zeta).
void col_scales(const std::vector<Col> &cols, const HostHist &h, std::vector<cd> &eta, std::vector<cd> &zeta) {
  eta.resize(cols.size());
  zeta.resize(cols.size());
  for (size_t c = 0; c < cols.size(); ++c) {
    if (cols[c].ritz) {
      eta[c] = zeta[c] = 1.0;
    } else {
      const int i = cols[c].idx;
      eta[c] = 1.0 / h.rn[i];
      zeta[c] = h.rn[i] / std::conj(c2(h.rho[i]));
    }
  }
}

struct RestartJob {
  int jr = 0, nev = 0, which = 0;
  std::vector<Col> cols;
  RitzBlock prev;
  HostHist h{};
  // results
  bool ok = false;
  std::string err;
  int kept = 0;
  std::vector<cd> lam;
  std::vector<double2> CVraw, CWraw;  // m x kept, column-major
  std::atomic<bool> done{false};
  std::thread th;

  void run() {
    try {
      const int m = int(cols.size());
      CMat H = build_H(cols, h, prev);
      std::vector<cd> l1, l2;
      CMat y1, z1, y2, z2;
      if (!eig_small(H, l1, y1, z1, which)) throw std::runtime_error("eig(H^(m)) failed");
      CMat Hm1(m - 1, m - 1);
      for (int jj = 0; jj < m - 1; ++jj)
        for (int i = 0; i < m - 1; ++i) Hm1(i, jj) = H(i, jj);
      if (!eig_small(Hm1, l2, y2, z2, which)) throw std::runtime_error("eig(H^(m-1)) failed");
      // [y^(m)_1..nev, y^(m-1)_1..nev] with a zero appended to the latter
      CMat Y(m, 2 * nev), Z(m, 2 * nev);
      for (int k = 0; k < nev; ++k)
        for (int i = 0; i < m; ++i) {
          Y(i, k) = y1(i, k);
          Z(i, k) = z1(i, k);
          Y(i, nev + k) = (i < m - 1) ? y2(i, k) : cd(0);
          Z(i, nev + k) = (i < m - 1) ? z2(i, k) : cd(0);
        }
      biorth_coeff(Y, Z, nev);
      // T = Zt^+ H Yt, [u, q, Lambda] = eig(T)
      CMat T = matmul(adjoint(Z), matmul(H, Y));
      CMat u, q;
      if (!eig_small(T, lam, u, q, which)) throw std::runtime_error("eig(T) failed");
      CMat CV = matmul(Y, u), CW = matmul(Z, q);
      kept = CV.cols;
      std::vector<cd> eta, zeta;
      col_scales(cols, h, eta, zeta);
      CVraw.resize(size_t(m) * kept);
      CWraw.resize(size_t(m) * kept);
      for (int k = 0; k < kept; ++k) {
        double nrm = 0;
        for (int i = 0; i < m; ++i) nrm += std::norm(CV(i, k));
        nrm = std::sqrt(nrm);
        for (int i = 0; i < m; ++i) {
          CVraw[i + size_t(k) * m] = d2(eta[i] * CV(i, k) / nrm);
          CWraw[i + size_t(k) * m] = d2(zeta[i] * CW(i, k) * nrm);
        }
      }
      ok = true;
    } catch (const std::exception &e) {
      err = e.what();
      ok = false;
    }
    done.store(true, std::memory_order_release);
  }
};

struct EigBiCGOut {
  int iters = 0;
  int restarts = 0;
  int reason = 0;
  double rnorm = 0;
  std::vector<cd> ritz;
  int nvec = 0;  // Ritz pairs written to Ur[:, K..), Ul[:, K..)
};

// Window storage of an eigBiCG solve: FP64 slots that hold the recurrence's
// residuals themselves, or FP32 slots that hold copies of them (the FP64
// recurrence vectors then live in two ping-pong buffers).  Both windows sit in
// one allocation, so a rotation reads right-window slot s and left-window
// slot nslots + s from one base.
template <typename T>
struct Window {
  T *base = nullptr;
  int nslots = 0;
  size_t N = 0;
  T *V(int slot) const { return base + size_t(slot) * N; }
  T *W(int slot) const { return base + size_t(nslots + slot) * N; }
};

// The device restart of one window (Alg. BiCG-eigen on the GPU, side stream):
// which window it was started on and which ring slot holds its results.
struct DevJob {
  int jr = 0;
  int ring = 0;
  std::vector<Col> cols;
};

EigBiCGOut run_eigbicg(eb_op *op, const double2 *b, double2 *x, const eb_eig_params &P, hipStream_t s) {
  const size_t N = op->N;
  const int m = P.m, nev = P.nev;
  const bool w32 = P.window == EB_FP32;  // FP32 window: FP32 copies of r, rhat in the slots
  const bool dev = P.device_eig != 0;    // window eigenproblems on the device
  // iterations a restart may run behind before the solve waits for it (spare
  // window slots); the device restart (one workgroup per eigenproblem) takes
  // longer than the host thread and may lag until just before the next
  // restart is due (m - 2 nev iterations later)
  const int lag = dev ? std::max(8, std::min(24, m - 2 * nev - 1)) : 8;
  const int nslots = m + 1 + lag + 2 * nev;
  const size_t ncoef = size_t(m + 1) * 2 * nev;  // one coefficient block (m x 2nev complex)
  Window<double2> win64;
  Window<float2> win32;
  double2 *R64 = nullptr, *RH64 = nullptr;  // FP32 window: the recurrence's r, rhat (two each)
  if (w32) {
    win32 = Window<float2>{op->raw<float2>("win_VW32", 2 * size_t(nslots) * N * sizeof(float2)), nslots, N};
    R64 = op->vec("win_r64", 2);
    RH64 = op->vec("win_rh64", 2);
  } else {
    win64 = Window<double2>{op->vec("win_VW", 2 * size_t(nslots)), nslots, N};
  }
  // gamma5-Hermitian form (Sec. 4): rhat_j = gamma5 r_j is never formed; the
  // left window's stored residuals are read as gamma5 times the right window's
  const bool g5 = P.rhat == 2;
  double2 *p = op->vec("bicg_p"), *ph = op->vec("bicg_ph");
  double2 *Ap = op->vec("bicg_Ap", 2), *Adp = op->vec("bicg_Adp", 2);
  double2 *GA = op->vec("bicg_GA"), *GB = op->vec("bicg_GB");
  double2 *coef = op->raw<double2>("rot_coef", 4 * ncoef * sizeof(double2));  // 2 ring slots x (V, W)
  double2 *dots = op->raw<double2>("rot_dots", 2 * size_t(2 * nev) * sizeof(double2));
  KrylovHistory dh = op->history(P.maxiter + 4);
  const KrylovHistory hv = op->view(op->hhist.p);
  const HostHist hh{hv.alpha, hv.beta, hv.rho, hv.rn};
  KrylovState *S = op->S();
  // the recurrence's r_i and rhat_i (FP64): in window slot `slot` (FP64
  // window), or in ping-pong buffer i & 1 (FP32 window)
  auto Rrec = [&](int i, int slot) { return w32 ? R64 + size_t(i & 1) * N : win64.V(slot); };
  auto RHrec = [&](int i, int slot) { return w32 ? RH64 + size_t(i & 1) * N : win64.W(slot); };

  EigBiCGOut out;
  // r_0 in V slot 0, rhat_0 in W slot 0
  residual_launch(op, Rrec(0, 0), b, x, s);
  launch_bicg_init(g5 ? nullptr : RHrec(0, 0), p, g5 ? nullptr : ph, Rrec(0, 0), op->res.as<double>(), N, P.rhat,
                   op->g, P.tol, P.maxiter, S, dh, op->rs(), s);
  if (w32) {
    launch_convert_f64_f32(win32.V(0), Rrec(0, 0), N, s);
    if (!g5) launch_convert_f64_f32(win32.W(0), RHrec(0, 0), N, s);
  }
  KrylovState hs;
  fetch_state(op, s, hs);
  if (hs.stopped) {
    out.reason = hs.reason;
    out.rnorm = hs.rnorm;
    if (hs.reason == 2) fail(EB_ERR_BREAKDOWN, "eigBiCG: (rhat_0, r_0) = 0");
    return out;
  }

  std::deque<int> free_slots;
  for (int k = 1; k < nslots; ++k) free_slots.push_back(k);
  std::vector<int> slot_of_r(size_t(P.maxiter) + 2, -1);
  slot_of_r[0] = 0;
  std::vector<Col> cols;
  RitzBlock rb;
  std::unique_ptr<RestartJob> job;
  std::unique_ptr<DevJob> djob;
  // host mirror of the history: after iteration j the device holds alpha, beta
  // for indices < j and rho, rn for indices <= j
  int ab_copied = 0, rr_copied = 0;

  // pinned staging: [0] state at a restart point, [1..] arrow dots, coefficient ring
  PinnedBuf pstate, pdots, pcoef, pdev;
  pstate.ensure(sizeof(KrylovState));
  pdots.ensure(2 * size_t(2 * nev) * sizeof(double2));
  pcoef.ensure(4 * ncoef * sizeof(double2));
  hipEvent_t ev_hist = nullptr, ev_coef[2] = {nullptr, nullptr}, ev_go[2] = {nullptr, nullptr},
             ev_done[2] = {nullptr, nullptr};
  bool coef_used[2] = {false, false};
  int coef_ring = 0;
  HIPCHK(hipEventCreateWithFlags(&ev_hist, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&ev_coef[0], hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&ev_coef[1], hipEventDisableTiming));
  // device restarts: workspace, Ritz values and kept counts per ring slot
  // (slot 2: the final extraction), their pinned mirror, a side stream
  constexpr int kLamStride = 64;
  double2 *wsd = nullptr, *lamd = nullptr;
  int *keptd = nullptr;
  int dring = 0, last_lam = 0;
  struct DevMirror {
    int kept;
    int pad[3];
    double2 lam[kLamStride];
  };
  if (dev) {
    wsd = op->raw<double2>("win_ws", window_restart_ws_entries(m + 1, nev) * sizeof(double2));
    lamd = op->raw<double2>("win_lam", 3 * kLamStride * sizeof(double2));
    keptd = op->raw<int>("win_kept", 3 * sizeof(int));
    pdev.ensure(3 * sizeof(DevMirror));
    if (!op->side) HIPCHK(hipStreamCreateWithFlags(&op->side, hipStreamNonBlocking));
    for (int r = 0; r < 2; ++r) {
      HIPCHK(hipEventCreateWithFlags(&ev_go[r], hipEventDisableTiming));
      HIPCHK(hipEventCreateWithFlags(&ev_done[r], hipEventDisableTiming));
    }
  }
  DevMirror *mir = dev ? pdev.as<DevMirror>() : nullptr;
  struct Cleanup {
    std::function<void()> f;
    ~Cleanup() { f(); }
  } cleanup{[&]() {
    if (job && job->th.joinable()) job->th.join();
    (void)hipStreamSynchronize(s);
    if (dev && op->side) (void)hipStreamSynchronize(op->side);
    (void)hipEventDestroy(ev_hist);
    (void)hipEventDestroy(ev_coef[0]);
    (void)hipEventDestroy(ev_coef[1]);
    for (int r = 0; r < 2; ++r) {
      if (ev_go[r]) (void)hipEventDestroy(ev_go[r]);
      if (ev_done[r]) (void)hipEventDestroy(ev_done[r]);
    }
    pstate.release();
    pdots.release();
    pcoef.release();
    pdev.release();
  }};

  // Upload a (V, W) pair of coefficient blocks through the pinned ring; returns device pointers.
  auto upload_coef = [&](const std::vector<double2> &cv, const std::vector<double2> &cw) {
    const int r = coef_ring;
    coef_ring ^= 1;
    if (coef_used[r]) HIPCHK(hipEventSynchronize(ev_coef[r]));
    double2 *hc = pcoef.as<double2>() + size_t(r) * 2 * ncoef;
    std::copy(cv.begin(), cv.end(), hc);
    std::copy(cw.begin(), cw.end(), hc + ncoef);
    double2 *dc = coef + size_t(r) * 2 * ncoef;
    HIPCHK(hipMemcpyAsync(dc, hc, cv.size() * sizeof(double2), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(dc + ncoef, hc + ncoef, cw.size() * sizeof(double2), hipMemcpyHostToDevice, s));
    HIPCHK(hipEventRecord(ev_coef[r], s));
    coef_used[r] = true;
    return std::make_pair(dc, dc + ncoef);
  };
  auto copy_history = [&](int jdone) {  // the history as it stands after iteration jdone -> host
    const int ab = jdone - ab_copied, rr = jdone + 1 - rr_copied;
    if (ab > 0) {
      HIPCHK(hipMemcpyAsync(hv.alpha + ab_copied, dh.alpha + ab_copied, ab * sizeof(double2), hipMemcpyDeviceToHost,
                            s));
      HIPCHK(hipMemcpyAsync(hv.beta + ab_copied, dh.beta + ab_copied, ab * sizeof(double2), hipMemcpyDeviceToHost,
                            s));
      ab_copied = jdone;
    }
    if (rr > 0) {
      HIPCHK(hipMemcpyAsync(hv.rho + rr_copied, dh.rho + rr_copied, rr * sizeof(double2), hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(hv.rn + rr_copied, dh.rn + rr_copied, rr * sizeof(double), hipMemcpyDeviceToHost, s));
      rr_copied = jdone + 1;
    }
  };
  auto copy_dots = [&]() {
    if (rb.lam.empty()) return;
    HIPCHK(hipMemcpyAsync(pdots.p, dots, 2 * size_t(2 * nev) * sizeof(double2), hipMemcpyDeviceToHost, s));
  };
  auto load_dots = [&]() {  // after an event that followed copy_dots
    if (rb.lam.empty()) return;
    const double2 *pd = pdots.as<double2>();
    const int kept = int(rb.lam.size());
    rb.dV.resize(kept);
    rb.dW.resize(kept);
    for (int k = 0; k < kept; ++k) {
      rb.dV[k] = c2(pd[k]);
      rb.dW[k] = c2(pd[2 * nev + k]);
    }
  };
  auto win_cols = [&](const std::vector<Col> &cs) {
    WinCols wc{};
    wc.n = int(cs.size());
    for (int c = 0; c < wc.n; ++c) {
      wc.idx[c] = cs[c].idx;
      wc.ritz[c] = static_cast<unsigned char>(cs[c].ritz);
    }
    return wc;
  };
  // Inputs of a left-window rotation over the columns cols: in_base = the
  // window's base, a column at window slot s is nslots + s; in the gamma5 form
  // a stored residual is -(s + 1), i.e. gamma5 times right-window slot s.
  auto left_inputs = [&](const std::vector<Col> &cs) {
    SlotList in{};
    in.n = int(cs.size());
    for (int c = 0; c < in.n; ++c)
      in.idx[c] = (g5 && !cs[c].ritz) ? -(cs[c].slot + 1) : nslots + cs[c].slot;
    return in;
  };
  // the window rotations V <- V C_V, W <- W C_W into the slots outl, with the arrow dots
  auto rotate_window = [&](const SlotList &outl, const std::vector<Col> &incols, const double2 *cV, const double2 *cW,
                           int jr) {
    SlotList in{};
    in.n = int(incols.size());
    for (int c = 0; c < in.n; ++c) in.idx[c] = incols[c].slot;
    const SlotList inl = left_inputs(incols);
    if (w32) {
      TIMED(EB_K_ROTATE, s, launch_rotate(win32.base, outl, win32.base, in, cV, N, GA, 0, dots, jr, S, op->rs(), s));
      TIMED(EB_K_ROTATE, s,
            launch_rotate(win32.W(0), outl, win32.base, inl, cW, N, GB, 1, dots + 2 * nev, jr, S, op->rs(), s));
    } else {
      TIMED(EB_K_ROTATE, s, launch_rotate(win64.base, outl, win64.base, in, cV, N, GA, 0, dots, jr, S, op->rs(), s));
      TIMED(EB_K_ROTATE, s,
            launch_rotate(win64.W(0), outl, win64.base, inl, cW, N, GB, 1, dots + 2 * nev, jr, S, op->rs(), s));
    }
  };
  // Apply a finished restart: rotate the old window into `kept` fresh slots
  // (with the arrow dots), free the old slots, replace the placeholders.
  auto finish_restart = [&](int kept, const std::vector<Col> &old, const double2 *cV, const double2 *cW, int jr,
                            const std::vector<cd> &lam) {
    const int mm = int(old.size());
    SlotList outl{};
    outl.n = kept;
    for (int k = 0; k < kept; ++k) {
      if (free_slots.empty()) fail(EB_ERR_INVALID, "window slots exhausted");
      outl.idx[k] = free_slots.front();
      free_slots.pop_front();
    }
    rotate_window(outl, old, cV, cW, jr);
    for (int c = 0; c < mm; ++c) free_slots.push_back(old[c].slot);
    std::vector<Col> nc;
    for (int k = 0; k < kept; ++k) nc.push_back(Col{1, k, outl.idx[k]});
    for (const Col &c : cols)
      if (!(c.ritz && c.slot < 0)) nc.push_back(c);
    cols.swap(nc);
    rb.jr = jr;
    rb.lam = lam;
    rb.dV.clear();
    rb.dW.clear();
    out.restarts += 1;
  };
  auto apply_job = [&]() {
    if (djob) {  // device restart: wait for its results (usually done already)
      const int r = djob->ring;
      HIPCHK(hipEventSynchronize(ev_done[r]));
      const DevMirror &mr = mir[r];
      if (mr.kept == -2) {
        // skipped: the solve stopped before the restart's iteration; the old
        // window stands (the columns after the stop are dropped later)
        std::vector<Col> nc = djob->cols;
        for (const Col &c : cols)
          if (!(c.ritz && c.slot < 0)) nc.push_back(c);
        cols.swap(nc);
        djob.reset();
        return;
      }
      if (mr.kept < 1) fail(EB_ERR_EIG, "window restart on the device: an eigenproblem did not converge");
      std::vector<cd> lam(mr.kept);
      for (int k = 0; k < mr.kept; ++k) lam[k] = c2(mr.lam[k]);
      HIPCHK(hipStreamWaitEvent(s, ev_done[r], 0));
      const double2 *cV = coef + size_t(r) * 2 * ncoef, *cW = cV + ncoef;
      finish_restart(mr.kept, djob->cols, cV, cW, djob->jr, lam);
      last_lam = r;
      djob.reset();
      return;
    }
    if (!job) return;
    if (job->th.joinable()) job->th.join();
    if (!job->ok) fail(EB_ERR_EIG, "window restart: " + job->err);
    const auto cf = upload_coef(job->CVraw, job->CWraw);
    finish_restart(job->kept, job->cols, cf.first, cf.second, job->jr, job->lam);
    job.reset();
  };
  auto job_done = [&]() {
    if (djob) {
      const hipError_t e = hipEventQuery(ev_done[djob->ring]);
      if (e != hipSuccess && e != hipErrorNotReady) hipchk(e, "hipEventQuery");
      return e == hipSuccess;
    }
    return job && job->done.load(std::memory_order_acquire);
  };

  const int poll = 8;
  int j = 0;
  bool stopped = false;
  int stop_at = 0, reason = 0;
  double rnorm = 0;
  // (the timing, if any, runs the pair on p, phat into the second product buffers)
  const int mvf = bicg_matvec_form(op, Ap + N, Adp + N, p, g5 ? p : ph, S, s);
  const int nsig = mvf == kMarchTile ? bicg_matvec_march_records(op->g, g5) : 0;
  {
    Poller pl(op, S, s);
    while (true) {
      ++j;
      if (j > P.maxiter + 1) break;
      const int cur = j & 1, prv = cur ^ 1;
      TIMED(EB_K_BICG_MATVEC, s,
            op->eo ? launch_bicg_matvec_eo(Ap + cur * N, g5 ? nullptr : Adp + cur * N, p, g5 ? nullptr : ph,
                                           op->vec("eo_tmp"), op->Ueo.as<double2>(), op->g, op->kappa, j, S,
                                           op->rs(), g5, s)
            : mvf == kMarchTile
                ? launch_bicg_matvec_march(Ap + cur * N, g5 ? nullptr : Adp + cur * N, p, g5 ? nullptr : ph,
                                           op->U64.as<double2>(), op->g, op->kappa, j, S, op->rs(), g5, s)
                : launch_bicg_matvec(Ap + cur * N, g5 ? nullptr : Adp + cur * N, p, g5 ? nullptr : ph,
                                     op->U64.as<double2>(), op->g, op->kappa, j, S, dh, op->rs(), g5, s));
      if (int(cols.size()) == m) {
        // Restart at iteration j (vs = m).  q = A p and s = A^+ phat were kept
        // from iteration j-1 (vs = m-1) in the other buffer.
        launch_arrow_vectors(GA, GB, g5 ? nullptr : Adp + cur * N, g5 ? nullptr : Adp + prv * N, Ap + cur * N,
                             Ap + prv * N, N, j, S, dh, g5, s);
        if (dev) {
          // Alg. BiCG-eigen on the device, on the side stream: it reads the
          // history through j-1, the last restart's Ritz values and arrow dots,
          // and skips itself if the solve stopped before iteration j
          const int r = dring;
          dring ^= 1;
          HIPCHK(hipEventRecord(ev_go[r], s));
          HIPCHK(hipStreamWaitEvent(op->side, ev_go[r], 0));
          double2 *cV = coef + size_t(r) * 2 * ncoef, *cW = cV + ncoef;
          launch_window_eig(win_cols(cols), nev, 0, P.sort, dh, lamd + size_t(last_lam) * kLamStride, dots, cV, cW,
                            lamd + size_t(r) * kLamStride, keptd + r, wsd, j, S, op->side);
          HIPCHK(hipMemcpyAsync(&mir[r].kept, keptd + r, sizeof(int), hipMemcpyDeviceToHost, op->side));
          HIPCHK(hipMemcpyAsync(mir[r].lam, lamd + size_t(r) * kLamStride, kLamStride * sizeof(double2),
                                hipMemcpyDeviceToHost, op->side));
          HIPCHK(hipEventRecord(ev_done[r], op->side));
          djob.reset(new DevJob);
          djob->jr = j;
          djob->ring = r;
          djob->cols = cols;
        } else {
          // history through j-1 was shipped at the end of iteration j-1; the GPU
          // keeps working on this iteration's matvec meanwhile
          HIPCHK(hipEventSynchronize(ev_hist));
          const KrylovState *ps = pstate.as<KrylovState>();
          if (ps->stopped) {
            stopped = true;
            stop_at = ps->stop_at;
            reason = ps->reason;
            rnorm = ps->rnorm;
            break;
          }
          load_dots();
          job.reset(new RestartJob);
          job->jr = j;
          job->nev = nev;
          job->which = P.sort;
          job->cols = cols;
          job->prev = rb;
          job->h = hh;
          job->th = std::thread([jp = job.get()]() { jp->run(); });
        }
        cols.clear();
        for (int k = 0; k < 2 * nev; ++k) cols.push_back(Col{1, k, -1});
      }
      // vs = vs + 1: the window gains r_{j-1} (already stored raw in its slot)
      cols.push_back(Col{0, j - 1, slot_of_r[j - 1]});
      // a pending restart needs 2 nev free slots for its rotated columns: once
      // the lag has used up the spare slots, wait for it
      if ((job || djob) && free_slots.size() <= size_t(2 * nev)) apply_job();
      if (free_slots.empty()) fail(EB_ERR_INVALID, "window slots exhausted");
      const int snew = free_slots.front();
      free_slots.pop_front();
      slot_of_r[j] = snew;
      const int sold = slot_of_r[j - 1];
      TIMED(EB_K_BICG_UPDATE_R, s,
            launch_bicg_update_r(Rrec(j, snew), g5 ? nullptr : RHrec(j, snew), Rrec(j - 1, sold),
                                 g5 ? nullptr : RHrec(j - 1, sold), Ap + cur * N, g5 ? nullptr : Adp + cur * N, N, j,
                                 S, dh, op->rs(), g5, s, w32 ? win32.V(snew) : nullptr,
                                 (w32 && !g5) ? win32.W(snew) : nullptr, nsig));
      if (job_done()) apply_job();
      TIMED(EB_K_BICG_UPDATE_P, s,
            launch_bicg_update_p(x, p, g5 ? nullptr : ph, Rrec(j, snew), g5 ? nullptr : RHrec(j, snew), N, j, S, dh,
                                 op->rs(), g5, s));
      if (int(cols.size()) == m) {
        // the next iteration restarts: the previous restart must be applied
        // first; then (host restarts) ship the history through j (complete
        // after update_p) and the arrow dots
        apply_job();
        if (int(cols.size()) == m && !dev) {
          copy_history(j);
          copy_dots();
          HIPCHK(hipMemcpyAsync(pstate.p, S, sizeof(KrylovState), hipMemcpyDeviceToHost, s));
          HIPCHK(hipEventRecord(ev_hist, s));
        }
      }
      if (j % poll == 0 && pl.step(&hs)) {
        stopped = true;
        stop_at = hs.stop_at;
        reason = hs.reason;
        rnorm = hs.rnorm;
        break;
      }
    }
  }
  if (!stopped) {
    fetch_state(op, s, hs);
    stop_at = hs.stopped ? hs.stop_at : std::min(j, P.maxiter);
    reason = hs.stopped ? hs.reason : 4;
    rnorm = hs.rnorm;
  }
  if (job || djob) apply_job();
  // roll back the window to iteration stop_at: columns r_i with i >= stop_at
  // were appended by iterations that did not run
  {
    std::vector<Col> nc;
    for (const Col &c : cols)
      if ((c.ritz && c.slot >= 0) || (!c.ritz && c.idx < stop_at)) nc.push_back(c);
    cols.swap(nc);
  }
  out.iters = stop_at;
  out.reason = reason;
  out.rnorm = rnorm;
  if (reason == 2) return out;
  // final eigenpairs from V^(vs), W^(vs), H^(vs) (Alg. eigBiCG, last step)
  const int vs = int(cols.size());
  if (vs == 0) return out;
  const int k = std::min(nev, vs);
  const double2 *cV = nullptr, *cW = nullptr;
  if (dev) {
    const int rf = 2;
    double2 *fV = coef + size_t(dring) * 2 * ncoef, *fW = fV + ncoef;
    launch_window_eig(win_cols(cols), nev, 1, P.sort, dh, lamd + size_t(last_lam) * kLamStride, dots, fV, fW,
                      lamd + size_t(rf) * kLamStride, keptd + rf, wsd, 0, nullptr, s);
    HIPCHK(hipMemcpyAsync(&mir[rf].kept, keptd + rf, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(mir[rf].lam, lamd + size_t(rf) * kLamStride, kLamStride * sizeof(double2),
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (mir[rf].kept != k) fail(EB_ERR_EIG, "final eig(H^(vs)) on the device did not converge");
    for (int c = 0; c < k; ++c) out.ritz.push_back(c2(mir[rf].lam[c]));
    cV = fV;
    cW = fW;
  } else {
    copy_history(stop_at);
    copy_dots();
    HIPCHK(hipStreamSynchronize(s));
    load_dots();
    CMat H = build_H(cols, hh, rb);
    std::vector<cd> lam;
    CMat y, z;
    if (!eig_small(H, lam, y, z, P.sort)) fail(EB_ERR_EIG, "final eig(H^(vs)) failed");
    out.ritz.assign(lam.begin(), lam.begin() + k);
    std::vector<cd> eta, zeta;
    col_scales(cols, hh, eta, zeta);
    std::vector<double2> cv(size_t(vs) * k), cw(size_t(vs) * k);
    for (int c = 0; c < k; ++c)
      for (int i = 0; i < vs; ++i) {
        cv[i + size_t(c) * vs] = d2(eta[i] * y(i, c));
        cw[i + size_t(c) * vs] = d2(zeta[i] * z(i, c));
      }
    const auto cf = upload_coef(cv, cw);
    cV = cf.first;
    cW = cf.second;
  }
  if (op->Kcap - op->K >= k) {
    SlotList in{}, o1{};
    in.n = vs;
    for (int c = 0; c < vs; ++c) in.idx[c] = cols[c].slot;
    o1.n = k;
    for (int c = 0; c < k; ++c) o1.idx[c] = op->K + c;
    if (w32) {
      launch_rotate(op->Ur.as<double2>(), o1, win32.base, in, cV, N, nullptr, 0, nullptr, 0, nullptr, op->rs(), s);
      launch_rotate(op->Ul.as<double2>(), o1, win32.base, left_inputs(cols), cW, N, nullptr, 0, nullptr, 0, nullptr,
                    op->rs(), s);
    } else {
      launch_rotate(op->Ur.as<double2>(), o1, win64.base, in, cV, N, nullptr, 0, nullptr, 0, nullptr, op->rs(), s);
      launch_rotate(op->Ul.as<double2>(), o1, win64.base, left_inputs(cols), cW, N, nullptr, 0, nullptr, 0, nullptr,
                    op->rs(), s);
    }
    HIPCHK(hipStreamSynchronize(s));
    out.nvec = k;
  }
  return out;
}

// Biorthogonalise the nnew pairs in Ur[:, K..K+nnew), Ul[:, K..) against the
// space and among themselves, extend H = Ul^+ A Ur, and grow K (Alg.
// Incremental eigBiCG, step 2, items 3-5).  Returns the number kept.
//
// Against the space: two block passes V' -= Ur (Ul^+ V'), W' -= Ul (Ur^+ W')
// (tall-skinny products that read each column once per pass).  Among
// themselves: a two-sided Gram-Schmidt (twice) carried out in coefficient
// space on the small Gram matrices W'^+ V', V'^+ V', W'^+ W', then applied
// with one out-of-place combination.  In exact arithmetic this gives the same
// vectors as projecting each new pair against the space and the earlier new
// pairs in turn, since the oblique projector onto the complement of the space
// is idempotent and leaves the earlier new pairs unchanged.
int absorb(eb_op *op, int nnew, eb_stats &st, hipStream_t s) {
  const size_t N = op->N;
  const int K = op->K;
  double2 *Ur = op->Ur.as<double2>(), *Ul = op->Ul.as<double2>();
  double2 *Vn = Ur + size_t(K) * N, *Wn = Ul + size_t(K) * N;
  double2 *C = op->raw<double2>("abs_C", size_t(op->Kcap) * nnew * 2 * sizeof(double2));
  if (K > 0) {
    for (int pass = 0; pass < 2; ++pass) {
      TIMED(EB_K_PROJ, s, launch_ts_dot(C, Ul, N, K, Vn, N, nnew, N, op->rs(), s));
      TIMED(EB_K_PROJ, s, launch_ts_dot(C + size_t(K) * nnew, Ur, N, K, Wn, N, nnew, N, op->rs(), s));
      TIMED(EB_K_PROJ, s, launch_ts_update(Vn, N, nnew, Ur, N, K, C, -1.0, N, s));
      TIMED(EB_K_PROJ, s, launch_ts_update(Wn, N, nnew, Ul, N, K, C + size_t(K) * nnew, -1.0, N, s));
    }
  }
  // Gram matrices of the new block: M = W'^+ V', G = V'^+ V', F = W'^+ W'
  const size_t n2 = size_t(nnew) * nnew;
  double2 *gram = op->raw<double2>("abs_gram", 3 * n2 * sizeof(double2));
  TIMED(EB_K_PROJ, s, launch_ts_dot(gram, Wn, N, nnew, Vn, N, nnew, N, op->rs(), s));
  TIMED(EB_K_PROJ, s, launch_ts_dot(gram + n2, Vn, N, nnew, Vn, N, nnew, N, op->rs(), s));
  TIMED(EB_K_PROJ, s, launch_ts_dot(gram + 2 * n2, Wn, N, nnew, Wn, N, nnew, N, op->rs(), s));
  std::vector<double2> hg(3 * n2);
  HIPCHK(hipMemcpyAsync(hg.data(), gram, hg.size() * sizeof(double2), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  CMat M(nnew, nnew), G(nnew, nnew), F(nnew, nnew);
  for (int b2 = 0; b2 < nnew; ++b2)
    for (int a2 = 0; a2 < nnew; ++a2) {
      M(a2, b2) = c2(hg[a2 + size_t(b2) * nnew]);
      G(a2, b2) = c2(hg[n2 + a2 + size_t(b2) * nnew]);
      F(a2, b2) = c2(hg[2 * n2 + a2 + size_t(b2) * nnew]);
    }
  // inner products of combinations: w^+ v = cw^+ M cv, v^+ v = cv^+ G cv, w^+ w = cw^+ F cw
  auto quad = [&](const CMat &A, const std::vector<cd> &x, const std::vector<cd> &y) {
    cd acc = 0;
    for (int i2 = 0; i2 < nnew; ++i2) {
      cd row = 0;
      for (int j2 = 0; j2 < nnew; ++j2) row += A(i2, j2) * y[j2];
      acc += std::conj(x[i2]) * row;
    }
    return acc;
  };
  std::vector<std::vector<cd>> cvs, cws;
  for (int k = 0; k < nnew; ++k) {
    std::vector<cd> cv(nnew, 0.0), cw(nnew, 0.0);
    cv[k] = cw[k] = 1.0;
    for (int pass = 0; pass < 2; ++pass)
      for (size_t q = 0; q < cvs.size(); ++q) {
        const cd a1 = quad(M, cws[q], cv);                 // w_q^+ v
        const cd b1 = std::conj(quad(M, cw, cvs[q]));      // v_q^+ w = conj(w^+ v_q)
        for (int i2 = 0; i2 < nnew; ++i2) {
          cv[i2] -= cvs[q][i2] * a1;
          cw[i2] -= cws[q][i2] * b1;
        }
      }
    const cd piv = quad(M, cw, cv);
    const double nv = std::sqrt(std::max(0.0, quad(G, cv, cv).real()));
    const double nw = std::sqrt(std::max(0.0, quad(F, cw, cw).real()));
    if (!(std::abs(piv) > 1e-12 * nv * nw)) continue;
    for (auto &e : cv) e /= nv;
    const cd pn = piv / nv;
    for (auto &e : cw) e /= std::conj(pn);
    cvs.push_back(cv);
    cws.push_back(cw);
  }
  const int kept = int(cvs.size());
  if (kept == 0) return 0;
  std::vector<double2> cv(size_t(nnew) * kept), cw(size_t(nnew) * kept);
  for (int k = 0; k < kept; ++k)
    for (int i2 = 0; i2 < nnew; ++i2) {
      cv[i2 + size_t(k) * nnew] = d2(cvs[k][i2]);
      cw[i2 + size_t(k) * nnew] = d2(cws[k][i2]);
    }
  double2 *dc = op->raw<double2>("abs_coef", 2 * size_t(nnew) * kept * sizeof(double2));
  HIPCHK(hipMemcpyAsync(dc, cv.data(), cv.size() * sizeof(double2), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(dc + cv.size(), cw.data(), cw.size() * sizeof(double2), hipMemcpyHostToDevice, s));
  double2 *tv = op->vec("abs_tv", kept), *tw = op->vec("abs_tw", kept);
  SlotList in{}, o{};
  in.n = nnew;
  for (int i2 = 0; i2 < nnew; ++i2) in.idx[i2] = K + i2;
  o.n = kept;
  for (int k = 0; k < kept; ++k) o.idx[k] = k;
  TIMED(EB_K_ROTATE, s, launch_rotate(tv, o, Ur, in, dc, N, nullptr, 0, nullptr, 0, nullptr, op->rs(), s));
  TIMED(EB_K_ROTATE, s, launch_rotate(tw, o, Ul, in, dc + cv.size(), N, nullptr, 0, nullptr, 0, nullptr, op->rs(), s));
  HIPCHK(hipMemcpyAsync(Vn, tv, size_t(kept) * N * sizeof(double2), hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(Wn, tw, size_t(kept) * N * sizeof(double2), hipMemcpyDeviceToDevice, s));
  // A V', A^+ W'
  double2 *AV = op->vec("abs_AV", kept), *AdW = op->vec("abs_AdW", kept);
  for (int k = 0; k < kept; ++k) {
    TIMED(EB_K_DSLASH, s, apply64(op, AV + size_t(k) * N, Vn + size_t(k) * N, false, s));
    TIMED(EB_K_DSLASH, s, apply64(op, AdW + size_t(k) * N, Wn + size_t(k) * N, true, s));
  }
  st.matvec_d += kept;
  st.matvec_ddag += kept;
  const int Kn = K + kept;
  double2 *blk = op->raw<double2>("abs_blk", size_t(Kn) * kept * sizeof(double2));
  double2 *blk2 = op->raw<double2>("abs_blk2", size_t(std::max(K, 1)) * kept * sizeof(double2));
  // Ul_all^+ (A V'): rows < K give the new column block, rows >= K give W'^+ A V'
  TIMED(EB_K_PROJ, s, launch_ts_dot(blk, Ul, N, Kn, AV, N, kept, N, op->rs(), s));
  // Ur^+ (A^+ W'): its conjugate transpose is W'^+ A Ur
  if (K > 0) TIMED(EB_K_PROJ, s, launch_ts_dot(blk2, Ur, N, K, AdW, N, kept, N, op->rs(), s));
  std::vector<double2> h1(size_t(Kn) * kept), h2(size_t(K) * kept);
  HIPCHK(hipMemcpyAsync(h1.data(), blk, h1.size() * sizeof(double2), hipMemcpyDeviceToHost, s));
  if (K > 0) HIPCHK(hipMemcpyAsync(h2.data(), blk2, h2.size() * sizeof(double2), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  CMat Hn(Kn, Kn);
  for (int jj = 0; jj < K; ++jj)
    for (int i = 0; i < K; ++i) Hn(i, jj) = op->H(i, jj);
  for (int c = 0; c < kept; ++c) {
    for (int i = 0; i < Kn; ++i) Hn(i, K + c) = c2(h1[i + size_t(c) * Kn]);
    for (int i = 0; i < K; ++i) Hn(K + c, i) = std::conj(c2(h2[i + size_t(c) * K]));
  }
  op->H = Hn;
  op->K = Kn;
  return kept;
}

eb_stats zero_stats() {
  eb_stats st;
  std::memset(&st, 0, sizeof(st));
  return st;
}

void ensure_space(eb_op *op) {
  if (op->Kcap > 0 && !op->Ur.p) {
    op->Ur.ensure(size_t(op->Kcap) * op->N * sizeof(double2));
    op->Ul.ensure(size_t(op->Kcap) * op->N * sizeof(double2));
  }
}

}  // namespace

// ============================================================================
// Allocation-free operator application (eb_op_apply_noalloc)
// ============================================================================
// For callers that cannot allocate device memory (code under stream capture,
// tight serving loops): the two SoA staging spinors of D live in this
// file-scope array instead of the operator's work buffers.  Each device holds
// its own copy until the process ends; every call on a device shares it, so
// calls that overlap on one device race.
constexpr size_t kNoAllocScratchBytes = size_t(48) << 20;  // two FP64 spinors of 16^3 x 32
static __device__ __align__(256) double2 scratch[kNoAllocScratchBytes / sizeof(double2)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double2 *g_scratch_ptr[kMaxDevices] = {};
// Device address of `scratch` on device dev, which must be current; looked
// up once per device.  The host-side name `scratch` is only a stand-in for
// the symbol and never reaches a kernel or a copy.
double2 *scratch_address(int dev) {
  if (dev < 0 || dev >= kMaxDevices) fail(EB_ERR_INVALID, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) fail(EB_ERR_HIP, "hipGetSymbolAddress returned a null address");
    g_scratch_ptr[dev] = static_cast<double2 *>(p);
  }
  return g_scratch_ptr[dev];
}
}  // namespace

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

static eb_status create_impl(const double *gauge, double kappa, const int32_t dims[4], int32_t bc_t,
                             int32_t defl_capacity, eb_op **out, bool eo) {
  return guarded([&]() {
    if (!out || !gauge || !dims) fail(EB_ERR_INVALID, "null argument");
    *out = nullptr;
    for (int i = 0; i < 4; ++i)
      if (dims[i] < 2) fail(EB_ERR_INVALID, "every lattice extent must be >= 2");
    if (!std::isfinite(kappa)) fail(EB_ERR_INVALID, "kappa must be finite");
    if (bc_t != 1 && bc_t != -1) fail(EB_ERR_INVALID, "bc_t must be +1 or -1");
    if (defl_capacity < 0 || defl_capacity > kMaxCols) fail(EB_ERR_INVALID, "defl_capacity out of range [0, 128]");
    if (eo && (dims[0] % 2 || dims[1] % 2 || dims[2] % 2 || dims[3] % 2))
      fail(EB_ERR_INVALID, "the even-odd form needs even lattice extents");
    const long long V = 1LL * dims[0] * dims[1] * dims[2] * dims[3];
    if (V > kMaxVolume) fail(EB_ERR_INVALID, "lattice too large (V > " + std::to_string(kMaxVolume) + ")");
    std::unique_ptr<eb_op> op(new eb_op);
    HIPCHK(hipGetDevice(&op->device));
    op->g = Geom{dims[0], dims[1], dims[2], dims[3], int(V)};
    op->eo = eo;
    op->N = size_t(V) * 12 / (eo ? 2 : 1);
    op->kappa = kappa;
    op->bc_t = bc_t;
    op->Kcap = defl_capacity;
    op->partials.ensure(kMaxPartials * sizeof(double));
    op->state.ensure(kMaxBatch * sizeof(KrylovState));
    op->res.ensure(2 * kMaxBatch * sizeof(double));
    op->hstate.ensure(kMaxBatch * sizeof(KrylovState));
    op->hres.ensure(2 * kMaxBatch * sizeof(double));
    op->U64.ensure(size_t(36) * V * sizeof(double2));
    DevBuf tmp;
    tmp.ensure(size_t(36) * V * sizeof(double2));
    HIPCHK(hipMemcpy(tmp.p, gauge, size_t(36) * V * sizeof(double2), hipMemcpyHostToDevice));
    launch_pack_gauge_f64(op->U64.as<double2>(), tmp.as<double2>(), op->g, bc_t, nullptr);
    if (eo) {
      op->Ueo.ensure(size_t(36) * V * sizeof(double2));
      launch_pack_gauge_eo(op->Ueo.as<double2>(), tmp.as<double2>(), op->g, bc_t, nullptr);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipDeviceSynchronize());
    tmp.release();
    *out = op.release();
  });
}

eb_status eb_op_create(const double *gauge, double kappa, const int32_t dims[4], int32_t bc_t, int32_t defl_capacity,
                       eb_op **out) {
  return create_impl(gauge, kappa, dims, bc_t, defl_capacity, out, false);
}
eb_status eb_op_create_eo(const double *gauge, double kappa, const int32_t dims[4], int32_t bc_t,
                          int32_t defl_capacity, eb_op **out) {
  return create_impl(gauge, kappa, dims, bc_t, defl_capacity, out, true);
}

eb_status eb_op_destroy(eb_op *op) {
  return guarded([&]() {
    if (!op) return;
    (void)hipSetDevice(op->device);
    (void)hipDeviceSynchronize();
    op->free_all();
    delete op;
  });
}

static eb_status apply_impl(eb_op *op, void *out, const void *in, eb_prec prec, void *stream, bool dagger) {
  return guarded([&]() {
    if (!op || !out || !in) fail(EB_ERR_INVALID, "null argument");
    if (out == in) fail(EB_ERR_INVALID, "in and out must not overlap");
    set_device(op);
    hipStream_t s = static_cast<hipStream_t>(stream);
    // the full lattice (an even-odd operator's solver spinors hold half of it)
    const size_t N = size_t(op->g.V) * 12;
    if (prec == EB_FP64) {
      double2 *a = op->vec("apply_a", op->eo ? 2 : 1), *b = op->vec("apply_b", op->eo ? 2 : 1);
      launch_to_soa_f64(a, static_cast<const double2 *>(in), op->g, s);
      TIMED(EB_K_DSLASH, s, launch_dslash_f64(b, a, op->U64.as<double2>(), op->g, op->kappa, dagger, s));
      launch_from_soa_f64(static_cast<double2 *>(out), b, op->g, s);
    } else if (prec == EB_FP32) {
      const float2 *U = Inner<float2>::links(op, s);
      float2 *a = op->raw<float2>("apply_a32", N * sizeof(float2));
      float2 *b = op->raw<float2>("apply_b32", N * sizeof(float2));
      launch_to_soa_f32(a, static_cast<const float2 *>(in), op->g, s);
      TIMED(EB_K_DSLASH, s, launch_dslash_f32(b, a, U, op->g, op->kappa, dagger, s));
      launch_from_soa_f32(static_cast<float2 *>(out), b, op->g, s);
    } else if (prec == EB_BF16) {
      const bf16c *U = Inner<bf16c>::links(op, s);
      bf16c *a = op->raw<bf16c>("apply_a16", N * sizeof(bf16c));
      bf16c *b = op->raw<bf16c>("apply_b16", N * sizeof(bf16c));
      launch_to_soa_bf16(a, static_cast<const bf16c *>(in), op->g, s);
      TIMED(EB_K_DSLASH, s, launch_dslash_bf16(b, a, U, op->g, op->kappa, dagger, s));
      launch_from_soa_bf16(static_cast<bf16c *>(out), b, op->g, s);
    } else {
      fail(EB_ERR_INVALID, "unknown precision");
    }
    HIPCHK(hipGetLastError());
  });
}

eb_status eb_op_apply_schur(eb_op *op, void *out, const void *in, int32_t dagger, void *stream) {
  return guarded([&]() {
    if (!op || !out || !in) fail(EB_ERR_INVALID, "null argument");
    if (out == in) fail(EB_ERR_INVALID, "in and out must not overlap");
    if (!op->eo) fail(EB_ERR_INVALID, "eb_op_apply_schur needs an even-odd operator (eb_op_create_eo)");
    set_device(op);
    hipStream_t s = static_cast<hipStream_t>(stream);
    double2 *a = op->vec("schur_a"), *b = op->vec("schur_b");
    launch_to_eo(a, op->vec("schur_odd"), static_cast<const double2 *>(in), op->g, s);
    TIMED(EB_K_DSLASH, s, apply64(op, b, a, dagger != 0, s));
    launch_from_eo(static_cast<double2 *>(out), b, nullptr, op->g, s);
    HIPCHK(hipGetLastError());
  });
}

eb_status eb_op_apply(eb_op *op, void *out, const void *in, eb_prec prec, void *stream) {
  return apply_impl(op, out, in, prec, stream, false);
}
eb_status eb_op_apply_dagger(eb_op *op, void *out, const void *in, eb_prec prec, void *stream) {
  return apply_impl(op, out, in, prec, stream, true);
}

eb_status eb_op_apply_noalloc(eb_op *op, void *out, const void *in, int32_t dagger, void *stream) {
  return guarded([&]() {
    if (!op || !out || !in) fail(EB_ERR_INVALID, "null argument");
    if (out == in) fail(EB_ERR_INVALID, "in and out must not overlap");
    const size_t N = size_t(op->g.V) * 12;  // the full lattice, also for an even-odd operator
    if (2 * N * sizeof(double2) > kNoAllocScratchBytes)
      fail(EB_ERR_INVALID, "lattice too large for the allocation-free path (V <= " +
                               std::to_string(kNoAllocScratchBytes / (24 * sizeof(double2))) + ")");
    set_device(op);
    double2 *a = scratch_address(op->device), *b = a + N;
    hipStream_t s = static_cast<hipStream_t>(stream);
    launch_to_soa_f64(a, static_cast<const double2 *>(in), op->g, s);
    launch_dslash_f64(b, a, op->U64.as<double2>(), op->g, op->kappa, dagger != 0, s);
    launch_from_soa_f64(static_cast<double2 *>(out), b, op->g, s);
    HIPCHK(hipGetLastError());
  });
}

// A canonical right-hand side and start vector -> the solvers' vectors b, x.
// Wilson D: SoA copies; returns 1.  Even-odd: b = b_e + kappa H_eo b_o and
// x = x_e, with b_o kept in bo (N entries) for the reconstruction; returns
// ||b|| / ||b_hat||, the factor that turns a tolerance relative to the full
// right-hand side into one relative to the even system's (the residual of the
// full system with x_o reconstructed equals the even system's).
double load_system(eb_op *op, const double2 *b_can, const double2 *x_can, double2 *b, double2 *x, double2 *bo,
                   hipStream_t s) {
  if (!op->eo) {
    launch_to_soa_f64(b, b_can, op->g, s);
    launch_to_soa_f64(x, x_can, op->g, s);
    return 1.0;
  }
  const size_t N = op->N;
  double2 *be = op->vec("eo_be"), *xo = op->vec("eo_xo");
  launch_to_eo(be, bo, b_can, op->g, s);
  launch_to_eo(x, xo, x_can, op->g, s);
  launch_prep_eo(b, be, bo, op->g, op->Ueo.as<double2>(), op->kappa, 0, s);
  double2 *nr = op->raw<double2>("eo_norms", 3 * sizeof(double2));
  launch_ts_dot(nr, be, N, 1, be, N, 1, N, op->rs(), s);
  launch_ts_dot(nr + 1, bo, N, 1, bo, N, 1, N, op->rs(), s);
  launch_ts_dot(nr + 2, b, N, 1, b, N, 1, N, op->rs(), s);
  double2 h[3];
  HIPCHK(hipMemcpyAsync(h, nr, sizeof(h), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const double bfull = std::sqrt(h[0].x + h[1].x), bhat = std::sqrt(h[2].x);
  return bhat > 0 ? bfull / bhat : 1.0;
}

// The solvers' x -> canonical x_can (even-odd: x_o = b_o + kappa H_oe x_e,
// with b_o as kept by the matching load_system).
void store_solution(eb_op *op, const double2 *x, const double2 *bo, double2 *x_can, hipStream_t s) {
  if (!op->eo) {
    launch_from_soa_f64(x_can, x, op->g, s);
    return;
  }
  double2 *xo = op->vec("eo_xo");
  launch_prep_eo(xo, bo, x, op->g, op->Ueo.as<double2>(), op->kappa, 1, s);
  launch_from_eo(x_can, x, xo, op->g, s);
}

// ||b - D x|| / ||b|| of canonical vectors on the full lattice (FP64).
double full_rel_residual(eb_op *op, const double2 *b_can, const double2 *x_can, hipStream_t s) {
  const size_t halves = op->eo ? 2 : 1;
  double2 *b = op->vec("full_b", halves), *x = op->vec("full_x", halves), *r = op->vec("full_r", halves);
  launch_to_soa_f64(b, b_can, op->g, s);
  launch_to_soa_f64(x, x_can, op->g, s);
  launch_residual_f64(r, b, x, op->U64.as<double2>(), op->g, op->kappa, op->res.as<double>(), op->rs(), s);
  double h[2];
  HIPCHK(hipMemcpyAsync(h, op->res.p, sizeof(h), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return h[1] > 0 ? std::sqrt(h[0] / h[1]) : 0.0;
}

eb_status eb_eigbicg_solve(eb_op *op, const void *b_can, void *x_can, const eb_eig_params *P, double *ritz,
                           eb_stats *stats, void *stream) {
  eb_stats st = zero_stats();
  auto t0 = std::chrono::steady_clock::now();
  eb_status rc = guarded([&]() {
    if (!op || !b_can || !x_can || !P) fail(EB_ERR_INVALID, "null argument");
    if (P->nev < 1 || P->m <= 2 * P->nev) fail(EB_ERR_INVALID, "need nev >= 1 and m > 2 nev");
    if (P->m + 1 > kMaxCols || 2 * P->nev > 64) fail(EB_ERR_INVALID, "window too large (m <= 127, nev <= 32)");
    if (!(P->tol > 0) || P->maxiter < 1) fail(EB_ERR_INVALID, "tol > 0 and maxiter >= 1 required");
    if (P->rhat < 0 || P->rhat > 2) fail(EB_ERR_INVALID, "rhat must be 0, 1 or 2");
    if (P->window != EB_FP64 && P->window != EB_FP32) fail(EB_ERR_INVALID, "window must be EB_FP64 or EB_FP32");
    if (P->device_eig != 0 && P->device_eig != 1) fail(EB_ERR_INVALID, "device_eig must be 0 or 1");
    if (P->sort < EB_SORT_SMALLEST_MAG || P->sort > EB_SORT_LARGEST_MAG) fail(EB_ERR_INVALID, "unknown sort criterion");
    set_device(op);
    hipStream_t s = static_cast<hipStream_t>(stream);
    ensure_space(op);
    double2 *b = op->vec("solve_b"), *x = op->vec("solve_x");
    const double2 *bcan = static_cast<const double2 *>(b_can);
    double2 *xcan = static_cast<double2 *>(x_can);
    // tolerance on the solvers' system (the even system of an even-odd operator)
    double2 *bo = op->eo ? op->vec("eo_bo") : nullptr;
    const double scale = load_system(op, bcan, xcan, b, x, bo, s);
    eb_eig_params Ps = *P;
    Ps.tol = P->tol * scale;
    const double tol = Ps.tol;
    if (op->K > 0) deflate_guess(op, b, x, s);
    EigBiCGOut R = run_eigbicg(op, b, x, Ps, s);
    st.iters = R.iters;
    st.matvec_d = R.iters + 1;
    st.matvec_ddag = P->rhat == 2 ? 0 : R.iters;
    st.window_restarts = R.restarts;
    if (R.reason == 2) fail(EB_ERR_BREAKDOWN, "eigBiCG breakdown");
    if (ritz)
      for (size_t i = 0; i < R.ritz.size(); ++i) {
        ritz[2 * i] = R.ritz[i].real();
        ritz[2 * i + 1] = R.ritz[i].imag();
      }
    // true residual in FP64; continue with BiCGStab if the recursion drifted
    double2 *r = op->vec("solve_r");
    auto [rn, bn] = residual(op, r, b, x, s);
    st.rec_rel_resid = bn > 0 ? R.rnorm / (bn * scale) : 0;
    st.true_rel_resid = bn > 0 ? rn / bn : 0;
    if (bn > 0 && rn > tol * bn) {
      const int K0 = op->K;
      op->K = 0;  // the pairs of this solve are not absorbed yet; continue undeflated
      try {
        deflated_stab_f64(op, b, x, tol, 0.0, P->maxiter + st.iters, st, s);
      } catch (...) {
        op->K = K0;
        throw;
      }
      op->K = K0;
    }
    if (R.reason == 4 && st.true_rel_resid > tol) {
      store_solution(op, x, bo, xcan, s);
      HIPCHK(hipStreamSynchronize(s));
      fail(EB_ERR_NOT_CONVERGED, "eigBiCG: maxiter reached");
    }
    if (R.nvec > 0) st.nev_added = absorb(op, R.nvec, st, s);
    store_solution(op, x, bo, xcan, s);
    if (op->eo) st.true_rel_resid = full_rel_residual(op, bcan, xcan, s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
  });
  st.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (stats) *stats = st;
  return rc;
}

eb_status eb_deflated_bicg_solve(eb_op *op, const void *b_can, void *x_can, const eb_solve_params *P,
                                 eb_stats *stats, void *stream) {
  eb_stats st = zero_stats();
  auto t0 = std::chrono::steady_clock::now();
  eb_status rc = guarded([&]() {
    if (!op || !b_can || !x_can || !P) fail(EB_ERR_INVALID, "null argument");
    if (!(P->tol > 0) || P->maxiter < 1 || P->nrhs < 1) fail(EB_ERR_INVALID, "tol > 0, maxiter >= 1, nrhs >= 1");
    if (P->deftol < 0 || P->deftol >= 1) fail(EB_ERR_INVALID, "deftol must be in [0, 1)");
    if (!(P->inner_tol < 1)) fail(EB_ERR_INVALID, "inner_tol must be < 1 (<= 0 selects the default)");
    if (P->method != 0 && P->method != 1) fail(EB_ERR_INVALID, "method must be 0 (BiCGStab) or 1 (BiCG)");
    if (P->method == 1 && (P->inner != EB_FP64 || P->deftol != 0))
      fail(EB_ERR_INVALID, "method 1 (BiCG) runs in FP64 without DefTol restarts (inner = EB_FP64, deftol = 0)");
    if (P->inner != EB_FP64 && P->inner != EB_FP32 && P->inner != EB_BF16)
      fail(EB_ERR_INVALID, "inner precision must be EB_FP64, EB_FP32 or EB_BF16");
    if (P->batch != 0 && !batch_size_ok(P->batch)) fail(EB_ERR_INVALID, "batch must be 0, 1, 2, 4, 8 or 16");
    set_device(op);
    hipStream_t s = static_cast<hipStream_t>(stream);
    ensure_space(op);
    const double inner_tol = P->inner_tol > 0 ? P->inner_tol : (P->inner == EB_BF16 ? 1e-2 : 1e-6);
    double worst = 0;
    auto merge = [&](const eb_stats &sc) {
      st.iters += sc.iters;
      st.matvec_d += sc.matvec_d;
      st.matvec_ddag += sc.matvec_ddag;
      st.defl_restarts += sc.defl_restarts;
      st.outer_steps += sc.outer_steps;
      st.rec_rel_resid = std::max(st.rec_rel_resid, sc.rec_rel_resid);
      worst = std::max(worst, sc.true_rel_resid);
      st.true_rel_resid = worst;
    };
    const int kmax = (P->deftol > 0 || P->nrhs == 1 || P->method == 1)
                         ? 1
                         : (P->batch ? P->batch : choose_batch(op, P->inner, s));
    const size_t Ncan = size_t(op->g.V) * 12;  // canonical spinor length
    // Columns go in groups of up to kMaxBatch: a group is loaded and deflated
    // at once (one pass over U_l and U_r for all its columns), then solved in
    // batches of the chosen k (the largest power of two that fits; a single
    // leftover column runs the one-at-a-time solver, already deflated).
    const int gmax = kmax > 1 ? kMaxBatch : 1;
    int c0 = 0;
    while (c0 < P->nrhs) {
      const int gsz = std::min(gmax, P->nrhs - c0);
      const double2 *bc = static_cast<const double2 *>(b_can) + size_t(c0) * Ncan;
      double2 *xc = static_cast<double2 *>(x_can) + size_t(c0) * Ncan;
      double2 *b = op->vec("solve_b", gsz), *x = op->vec("solve_x", gsz);
      double2 *bo = op->eo ? op->vec("eo_bo", gsz) : nullptr;
      // per column: the tolerance on the solvers' system (even-odd: scaled by ||b|| / ||b_hat||)
      double scale[kMaxBatch], tolc[kMaxBatch];
      for (int c = 0; c < gsz; ++c) {
        scale[c] = load_system(op, bc + c * Ncan, xc + c * Ncan, b + c * op->N, x + c * op->N,
                               bo ? bo + c * op->N : nullptr, s);
        tolc[c] = P->tol * scale[c];
      }
      eb_stats sc = zero_stats();  // the group's: the sum (and the worst residuals) of its batches'
      eb_stats sb = zero_stats();  // the batch in flight
      auto add_batch = [&]() {
        sc.iters += sb.iters;
        sc.matvec_d += sb.matvec_d;
        sc.matvec_ddag += sb.matvec_ddag;
        sc.defl_restarts += sb.defl_restarts;
        sc.outer_steps += sb.outer_steps;
        sc.rec_rel_resid = std::max(sc.rec_rel_resid, sb.rec_rel_resid);
        sc.true_rel_resid = std::max(sc.true_rel_resid, sb.true_rel_resid);
        sb = zero_stats();
      };
      auto store = [&]() {
        for (int c = 0; c < gsz; ++c)
          store_solution(op, x + c * op->N, bo ? bo + c * op->N : nullptr, xc + c * Ncan, s);
      };
      try {
        if (gsz == 1) {
          if (op->K > 0) deflate_guess(op, b, x, s);
        } else {
          deflate_block(op, b, x, gsz, s);
        }
        int off = 0;
        while (off < gsz) {
          int kc = 1;
          while (kc * 2 <= kmax && off + kc * 2 <= gsz) kc *= 2;
          double2 *bb = b + size_t(off) * op->N, *xx = x + size_t(off) * op->N;
          if (kc == 1) {
            if (P->method == 1)
              deflated_bicg_f64(op, bb, xx, tolc[off], P->maxiter, sb, s);
            else if (P->inner == EB_FP64)
              deflated_stab_f64(op, bb, xx, tolc[off], P->deftol, P->maxiter, sb, s);
            else if (P->inner == EB_FP32)
              mixed_stab<float2>(op, bb, xx, tolc[off], inner_tol, P->maxiter, sb, s);
            else
              mixed_stab<bf16c>(op, bb, xx, tolc[off], inner_tol, P->maxiter, sb, s);
          } else if (P->inner == EB_FP64) {
            mixed_stab_batch<double2>(op, bb, xx, kc, tolc + off, 0.5 * P->tol, P->maxiter, sb, s);
          } else if (P->inner == EB_FP32) {
            mixed_stab_batch<float2>(op, bb, xx, kc, tolc + off, inner_tol, P->maxiter, sb, s);
          } else {
            mixed_stab_batch<bf16c>(op, bb, xx, kc, tolc + off, inner_tol, P->maxiter, sb, s);
          }
          add_batch();
          off += kc;
        }
      } catch (...) {
        // x holds the last iterate and the stats are filled
        add_batch();
        store();
        (void)hipStreamSynchronize(s);
        merge(sc);
        throw;
      }
      store();
      if (op->eo) {  // the full system's residuals; the recursive one relative to ||b||
        double worst_full = 0;
        for (int c = 0; c < gsz; ++c)
          worst_full = std::max(worst_full, full_rel_residual(op, bc + c * Ncan, xc + c * Ncan, s));
        sc.true_rel_resid = worst_full;
        if (gsz == 1) sc.rec_rel_resid /= scale[0];
      }
      merge(sc);
      c0 += gsz;
    }
    st.true_rel_resid = worst;
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
  });
  st.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (stats) *stats = st;
  return rc;
}

eb_status eb_op_apply_block(eb_op *op, void *out, const void *in, int32_t k, int32_t dagger, eb_prec prec,
                            void *stream) {
  return guarded([&]() {
    if (!op || !out || !in) fail(EB_ERR_INVALID, "null argument");
    if (out == in) fail(EB_ERR_INVALID, "in and out must not overlap");
    if (!batch_size_ok(k)) fail(EB_ERR_INVALID, "k must be 1, 2, 4, 8 or 16");
    set_device(op);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t n = size_t(op->g.V) * 12 * size_t(k);  // the full D, also for an even-odd operator
    auto run = [&](auto *tag, const auto *U) {
      using S = std::remove_pointer_t<decltype(tag)>;
      S *a = op->raw<S>(std::string(Inner<S>::tag) + "blk_a", n * sizeof(S));
      S *b = op->raw<S>(std::string(Inner<S>::tag) + "blk_b", n * sizeof(S));
      launch_to_batch<S>(a, static_cast<const S *>(in), op->g, k, s);
      TIMED(EB_K_BDSLASH, s,
            launch_bdslash<S>(b, a, U, op->g, op->kappa, dagger != 0, k, s, op->batch_stage[Inner<S>::index][k]));
      launch_from_batch<S>(static_cast<S *>(out), b, op->g, k, s);
    };
    if (prec == EB_FP64)
      run(static_cast<double2 *>(nullptr), Inner<double2>::links(op, s));
    else if (prec == EB_FP32)
      run(static_cast<float2 *>(nullptr), Inner<float2>::links(op, s));
    else if (prec == EB_BF16)
      run(static_cast<bf16c *>(nullptr), Inner<bf16c>::links(op, s));
    else
      fail(EB_ERR_INVALID, "unknown precision");
    HIPCHK(hipGetLastError());
  });
}

eb_status eb_op_apply_schur_block(eb_op *op, void *out, const void *in, int32_t k, int32_t dagger, eb_prec prec,
                                  void *stream) {
  return guarded([&]() {
    if (!op || !out || !in) fail(EB_ERR_INVALID, "null argument");
    if (out == in) fail(EB_ERR_INVALID, "in and out must not overlap");
    if (!batch_size_ok(k)) fail(EB_ERR_INVALID, "k must be 1, 2, 4, 8 or 16");
    if (!op->eo) fail(EB_ERR_INVALID, "eb_op_apply_schur_block needs an even-odd operator (eb_op_create_eo)");
    if (prec != EB_FP64 && prec != EB_FP32 && prec != EB_BF16) fail(EB_ERR_INVALID, "unknown precision");
    set_device(op);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t N = op->N, Ncan = size_t(op->g.V) * 12;
    double2 *e = op->vec("sblk_e", k), *odd = op->vec("schur_odd");
    const double2 *inp = static_cast<const double2 *>(in);
    double2 *outp = static_cast<double2 *>(out);
    for (int c = 0; c < k; ++c) launch_to_eo(e + c * N, odd, inp + c * Ncan, op->g, s);
    auto run = [&](auto *tag) {
      using S = std::remove_pointer_t<decltype(tag)>;
      const std::string tg = Inner<S>::tag;
      const S *U = Inner<S>::solver_links(op, s);
      S *a = op->raw<S>(tg + "sblk_a", N * k * sizeof(S));
      S *b = op->raw<S>(tg + "sblk_b", N * k * sizeof(S));
      S *t = op->raw<S>(tg + "sblk_t", N * k * sizeof(S));
      launch_pack_batch<S>(a, e, N, k, s);
      TIMED(EB_K_BDSLASH, s,
            launch_bschur_eo<S>(b, a, t, U, op->g, op->kappa, dagger != 0, k, s, op->batch_stage[Inner<S>::index][k]));
      HIPCHK(hipMemsetAsync(e, 0, N * k * sizeof(double2), s));
      launch_unpack_add_batch<S>(e, b, N, k, s);
    };
    if (prec == EB_FP64)
      run(static_cast<double2 *>(nullptr));
    else if (prec == EB_FP32)
      run(static_cast<float2 *>(nullptr));
    else
      run(static_cast<bf16c *>(nullptr));
    for (int c = 0; c < k; ++c) launch_from_eo(outp + c * Ncan, e + c * N, nullptr, op->g, s);
    HIPCHK(hipGetLastError());
  });
}

eb_status eb_get_eigenpairs(eb_op *op, int32_t *k, double *evals, void *right, void *left, void *stream) {
  return guarded([&]() {
    if (!op || !k) fail(EB_ERR_INVALID, "null argument");
    set_device(op);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int K = op->K;
    const int kk = std::min<int>(*k, K);
    *k = kk;
    if (kk == 0) return;
    std::vector<cd> lam;
    CMat y, z;
    if (!eig_small(op->H, lam, y, z)) fail(EB_ERR_EIG, "eig(H) failed");
    if (evals)
      for (int i = 0; i < kk; ++i) {
        evals[2 * i] = lam[i].real();
        evals[2 * i + 1] = lam[i].imag();
      }
    if (!right && !left) return;
    const size_t N = op->N;
    double2 *R = op->vec("eig_R", kk), *L = op->vec("eig_L", kk);
    double2 *C = op->raw<double2>("eig_C", size_t(K) * kk * sizeof(double2));
    std::vector<double2> hc(size_t(K) * kk);
    // right = Ur y, left = Ul z; then ||right|| = 1, left^+ right = 1
    for (int side = 0; side < 2; ++side) {
      for (int c = 0; c < kk; ++c)
        for (int i = 0; i < K; ++i) hc[i + size_t(c) * K] = d2(side == 0 ? y(i, c) : z(i, c));
      HIPCHK(hipMemcpyAsync(C, hc.data(), hc.size() * sizeof(double2), hipMemcpyHostToDevice, s));
      double2 *dst = side == 0 ? R : L;
      HIPCHK(hipMemsetAsync(dst, 0, size_t(kk) * N * sizeof(double2), s));
      launch_ts_update(dst, N, kk, side == 0 ? op->Ur.as<double2>() : op->Ul.as<double2>(), N, K, C, 1.0, N, s);
      HIPCHK(hipStreamSynchronize(s));
    }
    double2 *d = op->raw<double2>("eig_d", 2 * sizeof(double2));
    std::vector<double2> hd(2);
    for (int c = 0; c < kk; ++c) {
      double2 *rc = R + size_t(c) * N, *lc = L + size_t(c) * N;
      launch_ts_dot(d, rc, N, 1, rc, N, 1, N, op->rs(), s);
      launch_ts_dot(d + 1, lc, N, 1, rc, N, 1, N, op->rs(), s);
      HIPCHK(hipMemcpyAsync(hd.data(), d, 2 * sizeof(double2), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      const double nr = std::sqrt(hd[0].x);
      const cd q = c2(hd[1]) / nr;
      launch_scale_f64(rc, make_double2(1.0 / nr, 0), N, s);
      launch_scale_f64(lc, d2(1.0 / std::conj(q)), N, s);
      // canonical full-lattice output (even-odd: zero on the odd sites)
      const size_t Ncan = size_t(op->g.V) * 12;
      double2 *ro = right ? static_cast<double2 *>(right) + size_t(c) * Ncan : nullptr;
      double2 *lo = left ? static_cast<double2 *>(left) + size_t(c) * Ncan : nullptr;
      if (op->eo) {
        if (ro) launch_from_eo(ro, rc, nullptr, op->g, s);
        if (lo) launch_from_eo(lo, lc, nullptr, op->g, s);
      } else {
        if (ro) launch_from_soa_f64(ro, rc, op->g, s);
        if (lo) launch_from_soa_f64(lo, lc, op->g, s);
      }
    }
    HIPCHK(hipStreamSynchronize(s));
  });
}

eb_status eb_defl_info(eb_op *op, int32_t *K, double *H) {
  return guarded([&]() {
    if (!op || !K) fail(EB_ERR_INVALID, "null argument");
    *K = op->K;
    if (H)
      for (int i = 0; i < op->K; ++i)
        for (int j = 0; j < op->K; ++j) {
          H[2 * (i * op->K + j)] = op->H(i, j).real();
          H[2 * (i * op->K + j) + 1] = op->H(i, j).imag();
        }
  });
}

eb_status eb_defl_reset(eb_op *op) {
  return guarded([&]() {
    if (!op) fail(EB_ERR_INVALID, "null argument");
    op->K = 0;
    op->H = CMat();
  });
}

eb_status eb_small_eig(int32_t n, const double *Cin, double *lambda, double *y, double *z) {
  return guarded([&]() {
    if (n < 0 || (n > 0 && (!Cin || !lambda))) fail(EB_ERR_INVALID, "bad arguments");
    CMat C(n, n);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) C(i, j) = cd(Cin[2 * (i * n + j)], Cin[2 * (i * n + j) + 1]);
    std::vector<cd> lam;
    CMat Y, Z;
    if (!eig_small(C, lam, Y, Z)) fail(EB_ERR_EIG, "QR iteration did not converge");
    for (int i = 0; i < n; ++i) {
      lambda[2 * i] = lam[i].real();
      lambda[2 * i + 1] = lam[i].imag();
    }
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        if (y) {
          y[2 * (i * n + j)] = Y(i, j).real();
          y[2 * (i * n + j) + 1] = Y(i, j).imag();
        }
        if (z) {
          z[2 * (i * n + j)] = Z(i, j).real();
          z[2 * (i * n + j) + 1] = Z(i, j).imag();
        }
      }
  });
}

eb_status eb_small_eig_device(int32_t n, const double *Cin, double *lambda, double *y, double *z) {
  return guarded([&]() {
    if (n < 1 || n > kMaxCols || !Cin || !lambda) fail(EB_ERR_INVALID, "need 1 <= n <= 128 and non-null C, lambda");
    const size_t nn = size_t(n) * n;
    std::vector<double2> hc(nn), hy(nn), hz(nn), hl(n);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) hc[i + size_t(j) * n] = make_double2(Cin[2 * (i * n + j)], Cin[2 * (i * n + j) + 1]);
    DevBuf d;
    d.ensure((3 * nn + n + window_eig_ws_entries(n)) * sizeof(double2) + 256);
    double2 *dc = d.as<double2>(), *dy = dc + nn, *dz = dy + nn, *dl = dz + nn, *ws = dl + n;
    int *dst = reinterpret_cast<int *>(ws + window_eig_ws_entries(n));
    hipStream_t s = nullptr;
    HIPCHK(hipMemcpyAsync(dc, hc.data(), nn * sizeof(double2), hipMemcpyHostToDevice, s));
    launch_small_eig(dc, n, dl, dy, dz, ws, dst, s);
    HIPCHK(hipGetLastError());
    int status = 0;
    HIPCHK(hipMemcpyAsync(hy.data(), dy, nn * sizeof(double2), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(hz.data(), dz, nn * sizeof(double2), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(hl.data(), dl, n * sizeof(double2), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&status, dst, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    d.release();
    if (status != 1) fail(EB_ERR_EIG, "device QR iteration did not converge");
    for (int i = 0; i < n; ++i) {
      lambda[2 * i] = hl[i].x;
      lambda[2 * i + 1] = hl[i].y;
      for (int j = 0; j < n; ++j) {
        if (y) {
          y[2 * (i * n + j)] = hy[i + size_t(j) * n].x;
          y[2 * (i * n + j) + 1] = hy[i + size_t(j) * n].y;
        }
        if (z) {
          z[2 * (i * n + j)] = hz[i + size_t(j) * n].x;
          z[2 * (i * n + j) + 1] = hz[i + size_t(j) * n].y;
        }
      }
    }
  });
}

eb_status eb_timing_enable(eb_op *op, int32_t enable) {
  return guarded([&]() {
    if (!op) fail(EB_ERR_INVALID, "null argument");
    set_device(op);
    op->flush_timing();
    for (int k = 0; k < EB_K_COUNT; ++k) {
      op->t_launch[k] = 0;
      op->t_ms[k] = 0;
    }
    op->timing = enable != 0;
  });
}

eb_status eb_timing_classes(eb_op *op, uint32_t mask) {
  return guarded([&]() {
    if (!op) fail(EB_ERR_INVALID, "null argument");
    op->timing_mask = mask;
  });
}

eb_status eb_timing_read(eb_op *op, int32_t kclass, int64_t *launches, double *total_ms) {
  return guarded([&]() {
    if (!op || !launches || !total_ms || kclass < 0 || kclass >= EB_K_COUNT) fail(EB_ERR_INVALID, "bad argument");
    set_device(op);
    op->flush_timing();
    *launches = op->t_launch[kclass];
    *total_ms = op->t_ms[kclass];
  });
}

void eb_last_error(char *buf, size_t len) {
  if (!buf || len == 0) return;
  std::snprintf(buf, len, "%s", g_last_error.c_str());
}

const char *eb_version(void) { return "ebicg 0.1 (gfx950)"; }

}  // extern "C"

// ============================================================================
// Serving sessions: continuous batching of deflated solves on one operator
// ============================================================================
// A session keeps kc slots in one batch of the multi-RHS BiCGStab.  Requests
// are admitted into free slots between chunks of iterations: the start is
// deflated with the operator's space as it is at admission (Alg. Incremental
// eigBiCG, step 3, first item), then each slot runs its own FP64 refinement
// around the inner BiCGStab in the session's precision.  A slot whose inner
// solve stopped is harvested at the next chunk boundary (x += e in FP64, true
// residual in FP64) and either finishes or restarts from the new residual, so
// slots free up and refill while the other columns keep iterating.  The
// session owns its reduction scratch, Krylov states and scalar history, so
// other solves on the operator (eigBiCG growing the space) can run between
// its chunks on the same stream.
struct SessionSlot {
  enum Phase { FREE = 0, PENDING, RUNNING } phase = FREE;
  int64_t tag = 0;
  const double2 *b_can = nullptr;
  double2 *x_can = nullptr;
  double scale = 1.0;  // tolerance factor of the solvers' system (even-odd: ||b|| / ||b_hat||)
  int iters = 0;       // inner iterations over all refinement steps
  int step_iters = 0;  // inner iterations of the current refinement step
  int outer = 0;
  int matvec = 0;
  std::chrono::steady_clock::time_point t0;
};
struct SessionDone {
  int64_t tag;
  eb_status status;
  eb_stats st;
};

struct eb_session {
  eb_op *op = nullptr;
  hipStream_t s = nullptr;
  int kc = 1;
  eb_prec prec = EB_FP64;
  double tol = 0, inner_tol = 0;
  int maxiter = 0, chunk = 8;
  size_t selem = 0;  // bytes of one inner-storage complex entry
  DevBuf partials, state, hist, res;
  PinnedBuf hstate, hres;
  DevBuf b, x, r, bo, tmp64;                     // FP64 columns of the solvers' system, kc each
  DevBuf rl, e, rhat, p, v, sv, t, tmp;          // the batch in the inner storage
  std::vector<SessionSlot> slot;
  std::deque<SessionDone> done;
  hipEvent_t ev = nullptr;
  bool inflight = false;
  int inflight_j = 0;
  int64_t chunks = 0;
  bool use_graph = true;            // replay one captured chunk (hipGraph) instead of launching it
  hipGraphExec_t graph = nullptr;
  RedScratch rs() { return RedScratch{partials.as<double>()}; }
  KrylovState *K() { return state.as<KrylovState>(); }
  KrylovHistory view() {
    const size_t cap = size_t(chunk + 2) * kc;
    char *base = static_cast<char *>(hist.p);
    KrylovHistory h;
    h.alpha = reinterpret_cast<double2 *>(base);
    h.beta = reinterpret_cast<double2 *>(base + cap * sizeof(double2));
    h.rho = reinterpret_cast<double2 *>(base + 2 * cap * sizeof(double2));
    h.omega = reinterpret_cast<double2 *>(base + 3 * cap * sizeof(double2));
    h.rn = reinterpret_cast<double *>(base + 4 * cap * sizeof(double2));
    return h;
  }
  size_t device_bytes() const {
    size_t n = 0;
    for (const DevBuf *d : {&partials, &state, &hist, &res, &b, &x, &r, &bo, &tmp64, &rl, &e, &rhat, &p, &v, &sv, &t,
                            &tmp})
      n += d->bytes;
    return n;
  }
  void release() {
    for (DevBuf *d : {&partials, &state, &hist, &res, &b, &x, &r, &bo, &tmp64, &rl, &e, &rhat, &p, &v, &sv, &t,
                      &tmp})
      d->release();
    hstate.release();
    hres.release();
    if (ev) (void)hipEventDestroy(ev);
    ev = nullptr;
    if (graph) (void)hipGraphExecDestroy(graph);
    graph = nullptr;
  }
};

namespace {

// The session's inner-storage operations for storage S.
template <typename S>
struct SessionOps {
  static S *at(DevBuf &d) { return d.as<S>(); }
  static void prepare(eb_session *ss) { (void)Inner<S>::solver_links(ss->op, ss->s); }
  // one chunk of `n` batched BiCGStab iterations (j = 1..n) on every slot
  static void chunk(eb_session *ss, int n) {
    eb_op *op = ss->op;
    const S *U = Inner<S>::solver_links(op, ss->s);
    const Geom gv = vector_geom(op);
    KrylovState *K = ss->K();
    KrylovHistory h = ss->view();
    const RedScratch rs = ss->rs();
    const int kc = ss->kc;
    const int stage = op->batch_stage[Inner<S>::index][kc];
    hipStream_t s = ss->s;
    S *x = at(ss->e), *r = at(ss->rl), *rhat = at(ss->rhat), *p = at(ss->p), *v = at(ss->v), *sv = at(ss->sv),
      *t = at(ss->t), *tmp = op->eo ? at(ss->tmp) : nullptr;
    for (int j = 1; j <= n; ++j) {
      if (op->eo)
        TIMED(EB_K_BSTAB_V, s, launch_bstab_v_eo<S>(v, p, rhat, tmp, U, op->g, op->kappa, j, kc, K, rs, s, stage));
      else
        TIMED(EB_K_BSTAB_V, s, launch_bstab_v<S>(v, p, rhat, U, op->g, op->kappa, j, kc, K, rs, s, stage));
      TIMED(EB_K_BSTAB_S, s, launch_bstab_s<S>(sv, r, v, gv, j, kc, K, h, rs, s, stage));
      if (op->eo)
        TIMED(EB_K_BSTAB_T, s, launch_bstab_t_eo<S>(t, sv, tmp, U, op->g, op->kappa, j, kc, K, rs, s, stage));
      else
        TIMED(EB_K_BSTAB_T, s, launch_bstab_t<S>(t, sv, U, op->g, op->kappa, j, kc, K, rs, s, stage));
      TIMED(EB_K_BSTAB_XR, s, launch_bstab_xr<S>(x, r, p, sv, t, rhat, gv, j, kc, K, h, rs, s, stage));
      TIMED(EB_K_BSTAB_P, s, launch_bstab_p<S>(p, r, v, gv, j, kc, K, h, rs, s));
    }
  }
  // slot c starts an inner solve from the FP64 residual in r[:, c]
  static void start(eb_session *ss, int c, double tol_abs, int maxiter) {
    const size_t N = ss->op->N;
    launch_slot_load<S>(at(ss->rl), at(ss->e), ss->r.as<double2>() + c * N, N, ss->kc, c, ss->s);
    launch_slot_init<S>(at(ss->rhat), at(ss->p), at(ss->rl), N, ss->kc, c, tol_abs, maxiter, ss->K(), ss->view(),
                        ss->rs(), ss->s);
  }
  static void add(eb_session *ss, int c) {
    const size_t N = ss->op->N;
    launch_slot_add<S>(ss->x.as<double2>() + c * N, at(ss->e), N, ss->kc, c, ss->s);
  }
};

template <typename F>
void session_dispatch(eb_prec prec, F &&f) {
  if (prec == EB_FP64)
    f(SessionOps<double2>{});
  else if (prec == EB_FP32)
    f(SessionOps<float2>{});
  else
    f(SessionOps<bf16c>{});
}

// r[:, c] = b[:, c] - A x[:, c] in FP64 for the listed slots; returns
// (||r||, ||b||) per listed slot (one synchronisation for all of them).
std::vector<std::pair<double, double>> session_residuals(eb_session *ss, const std::vector<int> &cols) {
  eb_op *op = ss->op;
  const size_t N = op->N;
  double *res = ss->res.as<double>();
  for (int c : cols) {
    double2 *r = ss->r.as<double2>() + c * N;
    const double2 *b = ss->b.as<double2>() + c * N, *x = ss->x.as<double2>() + c * N;
    if (op->eo)
      TIMED(EB_K_RESIDUAL, ss->s,
            launch_residual_eo(r, b, x, ss->tmp64.as<double2>(), op->Ueo.as<double2>(), op->g, op->kappa,
                               res + 2 * c, ss->rs(), ss->s));
    else
      TIMED(EB_K_RESIDUAL, ss->s,
            launch_residual_f64(r, b, x, op->U64.as<double2>(), op->g, op->kappa, res + 2 * c, ss->rs(), ss->s));
  }
  HIPCHK(hipMemcpyAsync(ss->hres.p, res, 2 * ss->kc * sizeof(double), hipMemcpyDeviceToHost, ss->s));
  HIPCHK(hipStreamSynchronize(ss->s));
  std::vector<std::pair<double, double>> out;
  const double *h = ss->hres.as<double>();
  for (int c : cols) out.push_back({std::sqrt(h[2 * c]), std::sqrt(h[2 * c + 1])});
  return out;
}

// Slot c is done: write its solution back (even-odd: reconstruct the odd
// sites), report the full system's residual, free the slot.
void session_finish(eb_session *ss, int c, eb_status status, double rel) {
  eb_op *op = ss->op;
  SessionSlot &q = ss->slot[c];
  const size_t N = op->N;
  store_solution(op, ss->x.as<double2>() + c * N, op->eo ? ss->bo.as<double2>() + c * N : nullptr, q.x_can, ss->s);
  eb_stats st = zero_stats();
  st.iters = q.iters;
  st.matvec_d = q.matvec;
  st.outer_steps = q.outer;
  st.true_rel_resid = op->eo ? full_rel_residual(op, q.b_can, q.x_can, ss->s) : rel;
  HIPCHK(hipStreamSynchronize(ss->s));
  st.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - q.t0).count();
  ss->done.push_back({q.tag, status, st});
  q = SessionSlot{};
}

// After the FP64 residuals of the listed slots: finish those at their target
// (or out of budget), start a refinement step on the others.
void session_advance(eb_session *ss, const std::vector<int> &cols, const std::vector<int> &why) {
  if (cols.empty()) return;
  auto rb = session_residuals(ss, cols);
  for (size_t i = 0; i < cols.size(); ++i) {
    const int c = cols[i];
    SessionSlot &q = ss->slot[c];
    q.matvec += 1;
    const double rn = rb[i].first, bn = rb[i].second;
    const double tolc = ss->tol * q.scale;
    if (bn == 0.0) {  // b = 0: the solution is x = 0
      HIPCHK(hipMemsetAsync(ss->x.as<double2>() + c * ss->op->N, 0, ss->op->N * sizeof(double2), ss->s));
      session_finish(ss, c, EB_OK, 0.0);
      continue;
    }
    const double rel = rn / bn;
    if (rel <= tolc) {
      session_finish(ss, c, EB_OK, rel / q.scale);
      continue;
    }
    if (q.iters >= ss->maxiter) {
      session_finish(ss, c, EB_ERR_NOT_CONVERGED, rel / q.scale);
      continue;
    }
    if (why[i] == 2 && q.step_iters == 0) {  // the inner solve broke down before its first update
      session_finish(ss, c, EB_ERR_BREAKDOWN, rel / q.scale);
      continue;
    }
    if (q.outer > 0 && q.step_iters == 0) {
      // a refinement step that stopped at initialisation leaves x unchanged:
      // the next one would do the same, so the request cannot progress
      session_finish(ss, c, EB_ERR_NOT_CONVERGED, rel / q.scale);
      continue;
    }
    const double target = std::max(ss->inner_tol * rn, 0.5 * tolc * bn);
    session_dispatch(ss->prec, [&](auto ops) { decltype(ops)::start(ss, c, target, ss->maxiter - q.iters); });
    q.step_iters = 0;
    q.outer += 1;
  }
}

// Wait for the chunk in flight and harvest the slots whose inner solve stopped.
void session_harvest(eb_session *ss) {
  if (!ss->inflight) return;
  HIPCHK(hipEventSynchronize(ss->ev));
  ss->inflight = false;
  const int jl = ss->inflight_j;
  launch_batch_rebase(ss->K(), ss->view(), ss->kc, jl, ss->s);
  const KrylovState *hs = ss->hstate.as<KrylovState>();
  std::vector<int> cols, why;
  for (int c = 0; c < ss->kc; ++c) {
    SessionSlot &q = ss->slot[c];
    if (q.phase != SessionSlot::RUNNING) continue;
    const int it = hs[c].stopped ? std::max(hs[c].stop_at, 0) : jl;
    q.iters += it;
    q.step_iters += it;
    q.matvec += 2 * it;
    if (hs[c].stopped) {
      session_dispatch(ss->prec, [&](auto ops) { decltype(ops)::add(ss, c); });
      cols.push_back(c);
      why.push_back(hs[c].reason);
    }
  }
  session_advance(ss, cols, why);
}

// Start the admitted requests: load b and x0, deflate x0 with the operator's
// current space, then the first refinement step (or finish at once).
void session_admit_pending(eb_session *ss) {
  eb_op *op = ss->op;
  const size_t N = op->N;
  std::vector<int> cols, why;
  for (int c = 0; c < ss->kc; ++c) {
    SessionSlot &q = ss->slot[c];
    if (q.phase != SessionSlot::PENDING) continue;
    double2 *b = ss->b.as<double2>() + c * N, *x = ss->x.as<double2>() + c * N;
    q.scale = load_system(op, q.b_can, q.x_can, b, x, op->eo ? ss->bo.as<double2>() + c * N : nullptr, ss->s);
    if (op->K > 0) deflate_guess(op, b, x, ss->s);
    q.phase = SessionSlot::RUNNING;
    cols.push_back(c);
    why.push_back(0);
  }
  session_advance(ss, cols, why);
}

// Launch the next chunk if any slot is running; the states are copied to the
// pinned mirror behind it.
void session_launch(eb_session *ss) {
  bool any = false;
  for (const auto &q : ss->slot) any = any || q.phase == SessionSlot::RUNNING;
  if (!any) return;
  auto launch = [&]() { session_dispatch(ss->prec, [&](auto ops) { decltype(ops)::chunk(ss, ss->chunk); }); };
  if (ss->use_graph && ss->s != nullptr && !ss->op->timing) {  // the null stream cannot be captured
    // every chunk launches the same kernels with the same arguments (j = 1..chunk,
    // the session's buffers and states), so one capture serves all of them
    if (!ss->graph) {
      hipGraph_t g = nullptr;
      HIPCHK(hipStreamBeginCapture(ss->s, hipStreamCaptureModeThreadLocal));
      try {
        launch();
      } catch (...) {
        (void)hipStreamEndCapture(ss->s, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
      }
      HIPCHK(hipStreamEndCapture(ss->s, &g));
      const hipError_t e = hipGraphInstantiate(&ss->graph, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      HIPCHK(e);
    }
    HIPCHK(hipGraphLaunch(ss->graph, ss->s));
  } else {
    launch();
  }
  HIPCHK(hipMemcpyAsync(ss->hstate.p, ss->state.p, ss->kc * sizeof(KrylovState), hipMemcpyDeviceToHost, ss->s));
  HIPCHK(hipEventRecord(ss->ev, ss->s));
  ss->inflight = true;
  ss->inflight_j = ss->chunk;
  ++ss->chunks;
}

size_t op_device_bytes(const eb_op *op) {
  size_t n = 0;
  for (const DevBuf *d : {&op->U64, &op->U32, &op->U16, &op->Ueo, &op->Ueo32, &op->Ueo16, &op->Ul, &op->Ur,
                          &op->partials, &op->state, &op->res, &op->hist})
    n += d->bytes;
  for (const auto &kv : op->bufs) n += kv.second.bytes;
  return n;
}

}  // namespace

extern "C" {

eb_status eb_session_create(eb_op *op, const eb_session_params *P, void *stream, eb_session **out) {
  return guarded([&]() {
    if (!op || !P || !out) fail(EB_ERR_INVALID, "null argument");
    *out = nullptr;
    if (!batch_size_ok(P->slots)) fail(EB_ERR_INVALID, "slots must be 1, 2, 4, 8 or 16");
    if (P->inner != EB_FP64 && P->inner != EB_FP32 && P->inner != EB_BF16)
      fail(EB_ERR_INVALID, "inner precision must be EB_FP64, EB_FP32 or EB_BF16");
    if (!(P->tol > 0) || P->maxiter < 1) fail(EB_ERR_INVALID, "tol > 0 and maxiter >= 1 required");
    if (P->chunk < 1 || P->chunk > 1024) fail(EB_ERR_INVALID, "chunk must be in [1, 1024]");
    if (!(P->inner_tol < 1)) fail(EB_ERR_INVALID, "inner_tol must be < 1 (<= 0 selects the default)");
    set_device(op);
    std::unique_ptr<eb_session> ss(new eb_session);
    ss->op = op;
    ss->s = static_cast<hipStream_t>(stream);
    ss->kc = P->slots;
    ss->prec = P->inner;
    ss->tol = P->tol;
    ss->inner_tol = P->inner_tol > 0 ? P->inner_tol : (P->inner == EB_BF16 ? 1e-2 : (P->inner == EB_FP32 ? 1e-6 : 0.0));
    ss->maxiter = P->maxiter;
    ss->chunk = P->chunk;
    ss->use_graph = P->graph != 0;
    ss->selem = P->inner == EB_FP64 ? sizeof(double2) : (P->inner == EB_FP32 ? sizeof(float2) : sizeof(bf16c));
    ss->slot.resize(ss->kc);
    const size_t N = op->N, kc = ss->kc;
    ss->partials.ensure(8 * kRegionDoubles * sizeof(double));  // one record region per producer kernel
    ss->state.ensure(kMaxBatch * sizeof(KrylovState));
    ss->hist.ensure(size_t(ss->chunk + 2) * kc * (4 * sizeof(double2) + sizeof(double)));
    ss->res.ensure(2 * kMaxBatch * sizeof(double));
    ss->hstate.ensure(kMaxBatch * sizeof(KrylovState));
    ss->hres.ensure(2 * kMaxBatch * sizeof(double));
    for (DevBuf *d : {&ss->b, &ss->x, &ss->r}) d->ensure(kc * N * sizeof(double2));
    if (op->eo) {
      ss->bo.ensure(kc * N * sizeof(double2));
      ss->tmp64.ensure(N * sizeof(double2));
    }
    for (DevBuf *d : {&ss->rl, &ss->e, &ss->rhat, &ss->p, &ss->v, &ss->sv, &ss->t}) d->ensure(kc * N * ss->selem);
    if (op->eo) ss->tmp.ensure(kc * N * ss->selem);
    // every slot starts stopped (inactive)
    std::vector<KrylovState> idle(kMaxBatch);
    for (auto &k : idle) {
      std::memset(&k, 0, sizeof(k));
      k.stopped = 1;
      k.stop_at = -1;
    }
    std::memcpy(ss->hstate.p, idle.data(), kMaxBatch * sizeof(KrylovState));
    HIPCHK(hipMemcpyAsync(ss->state.p, ss->hstate.p, kMaxBatch * sizeof(KrylovState), hipMemcpyHostToDevice, ss->s));
    session_dispatch(ss->prec, [&](auto ops) { decltype(ops)::prepare(ss.get()); });  // inner-precision links
    (void)choose_batch(op, ss->prec, ss->s);  // the batch autotuner's tile forms (once per operator and precision)
    HIPCHK(hipEventCreateWithFlags(&ss->ev, hipEventDisableTiming));
    HIPCHK(hipStreamSynchronize(ss->s));
    *out = ss.release();
  });
}

eb_status eb_session_destroy(eb_session *ss) {
  if (!ss) return EB_OK;
  eb_status rc = guarded([&]() {
    set_device(ss->op);
    if (ss->inflight) HIPCHK(hipEventSynchronize(ss->ev));
    HIPCHK(hipStreamSynchronize(ss->s));
  });
  ss->release();
  delete ss;
  return rc;
}

eb_status eb_session_admit(eb_session *ss, const void *b, void *x, int64_t tag, int32_t *slot) {
  return guarded([&]() {
    if (!ss || !b || !x) fail(EB_ERR_INVALID, "null argument");
    for (int c = 0; c < ss->kc; ++c) {
      SessionSlot &q = ss->slot[c];
      if (q.phase != SessionSlot::FREE) continue;
      q = SessionSlot{};
      q.phase = SessionSlot::PENDING;
      q.tag = tag;
      q.b_can = static_cast<const double2 *>(b);
      q.x_can = static_cast<double2 *>(x);
      q.t0 = std::chrono::steady_clock::now();
      if (slot) *slot = c;
      return;
    }
    fail(EB_ERR_CAPACITY, "no free slot");
  });
}

eb_status eb_session_step(eb_session *ss) {
  return guarded([&]() {
    if (!ss) fail(EB_ERR_INVALID, "null argument");
    eb_op *op = ss->op;
    set_device(op);
    session_harvest(ss);
    session_admit_pending(ss);
    session_launch(ss);
    HIPCHK(hipGetLastError());
  });
}

eb_status eb_session_ready(eb_session *ss, int32_t *ready) {
  return guarded([&]() {
    if (!ss || !ready) fail(EB_ERR_INVALID, "null argument");
    set_device(ss->op);
    *ready = 1;
    if (!ss->inflight) return;
    const hipError_t e = hipEventQuery(ss->ev);
    if (e == hipErrorNotReady) {
      *ready = 0;
      return;
    }
    HIPCHK(e);
  });
}

eb_status eb_session_poll(eb_session *ss, int32_t max, int64_t *tags, int32_t *status, eb_stats *stats,
                          int32_t *n) {
  return guarded([&]() {
    if (!ss || !n || max < 0 || (max > 0 && (!tags || !status))) fail(EB_ERR_INVALID, "bad argument");
    int k = 0;
    while (k < max && !ss->done.empty()) {
      const SessionDone &d = ss->done.front();
      tags[k] = d.tag;
      status[k] = d.status;
      if (stats) stats[k] = d.st;
      ss->done.pop_front();
      ++k;
    }
    *n = k;
  });
}

eb_status eb_session_info(eb_session *ss, int32_t *free_slots, int32_t *busy, int32_t *done, uint64_t *device_bytes) {
  return guarded([&]() {
    if (!ss) fail(EB_ERR_INVALID, "null argument");
    int nf = 0, nb = 0;
    for (const auto &q : ss->slot) (q.phase == SessionSlot::FREE ? nf : nb) += 1;
    if (free_slots) *free_slots = nf;
    if (busy) *busy = nb;
    if (done) *done = int32_t(ss->done.size());
    if (device_bytes) *device_bytes = ss->device_bytes();
  });
}

eb_status eb_op_batch_tune(eb_op *op, eb_prec prec, void *stream, int32_t *k_best, int32_t *stage,
                           double *ms_per_rhs) {
  return guarded([&]() {
    if (!op || !k_best) fail(EB_ERR_INVALID, "null argument");
    if (prec != EB_FP64 && prec != EB_FP32 && prec != EB_BF16) fail(EB_ERR_INVALID, "unknown precision");
    set_device(op);
    hipStream_t s = static_cast<hipStream_t>(stream);
    *k_best = choose_batch(op, prec, s);
    const int pi = prec == EB_FP64 ? 0 : (prec == EB_FP32 ? 1 : 2);
    for (int i = 0, kc = 1; kc <= kMaxBatch; ++i, kc *= 2) {
      if (stage) stage[i] = op->batch_stage[pi][kc];
      if (ms_per_rhs)
        for (int f = 0; f < kTileForms; ++f) ms_per_rhs[kTileForms * i + f] = op->batch_stage_ms[pi][kc][f];
    }
  });
}

eb_status eb_op_batch_set_tile(eb_op *op, eb_prec prec, int32_t k, int32_t stage) {
  return guarded([&]() {
    if (!op) fail(EB_ERR_INVALID, "null argument");
    if (prec != EB_FP64 && prec != EB_FP32 && prec != EB_BF16) fail(EB_ERR_INVALID, "unknown precision");
    if (!batch_size_ok(k)) fail(EB_ERR_INVALID, "k must be 1, 2, 4, 8 or 16");
    if (!batch_tile_ok(op->g, op->eo, stage, k))
      fail(EB_ERR_INVALID,
           "tile form must be -1, 0 or 1, or 2..6 on a full-lattice operator whose extents the form's brick or box fits");
    op->batch_stage[prec == EB_FP64 ? 0 : (prec == EB_FP32 ? 1 : 2)][k] = stage;
    if (k == 1) op->stab_cap[prec == EB_FP64 ? 0 : (prec == EB_FP32 ? 1 : 2)] = 0;  // a forced form: the grid cap
  });
}

eb_status eb_op_set_matvec_form(eb_op *op, int32_t form) {
  return guarded([&]() {
    if (!op) fail(EB_ERR_INVALID, "null argument");
    if (form != -1 && form != 1 && form != kMarchTile) fail(EB_ERR_INVALID, "matvec form must be -1, 1 or 6");
    if (form == kMarchTile && !batch_tile_ok(op->g, op->eo, kMarchTile, 1))
      fail(EB_ERR_INVALID, "the t-marching matvec needs a full-lattice operator whose box fits");
    op->matvec_form = form;
    op->matvec_cap = 0;  // a forced staged pair runs at the operator's grid cap
  });
}

eb_status eb_op_get_matvec_form(eb_op *op, int32_t *form, double *ms) {
  return guarded([&]() {
    if (!op || !form) fail(EB_ERR_INVALID, "null argument");
    *form = op->eo ? 1 : op->matvec_form;
    if (ms) {
      ms[0] = op->matvec_ms[1];
      ms[1] = op->matvec_ms[kMarchTile];
    }
  });
}

eb_status eb_op_trim(eb_op *op, void *stream) {
  return guarded([&]() {
    if (!op) fail(EB_ERR_INVALID, "null argument");
    set_device(op);
    HIPCHK(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
    HIPCHK(hipDeviceSynchronize());
    for (auto &kv : op->bufs) kv.second.release();
    op->bufs.clear();
    op->hist.release();
    op->hist_cap = 0;
  });
}

eb_status eb_op_set_grid_cap(eb_op *op, int32_t max_blocks) {
  return guarded([&]() {
    if (!op) fail(EB_ERR_INVALID, "null argument");
    if (max_blocks < 0) fail(EB_ERR_INVALID, "max_blocks must be >= 0");
    op->grid_cap = max_blocks == 0 ? kDefaultStencilCap : max_blocks;
  });
}

eb_status eb_op_device_bytes(eb_op *op, uint64_t *bytes) {
  return guarded([&]() {
    if (!op || !bytes) fail(EB_ERR_INVALID, "null argument");
    *bytes = op_device_bytes(op);
  });
}

}  // extern "C"

