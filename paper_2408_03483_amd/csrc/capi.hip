// C ABI entry points (include/tt_fv.h): argument checks, context/arena management and the
// translation of internal exceptions into return codes.
#include "common.h"
#include "rules.h"

#include <cmath>
#include <cstring>
#include <map>
#include <memory>

namespace ttfv {

Solver *solver_create(const tt_fv_params *p, const tt_matrix q0[3], void *stream,
                      size_t arena_bytes);
void solver_step(Solver *s, double dt, int nsteps);
void solver_get_state(Solver *s, tt_matrix q[3]);
void solver_stats(Solver *s, tt_fv_stats *o);
void solver_destroy(Solver *s);
void solver_time_kernel(Solver *s, const char *name, int every);
void solver_set_pivots(Solver *s, int mode, PivotModel *pm);
void solver_set_acceptance(Solver *s, double abs_tol, double rel_slack);
void solver_set_terms(Solver *s, const tt_fv_term *terms, int count);
void solver_max_speed(Solver *s, double out[2]);
double solver_cfl_dt(Solver *s, double cfl);
void solver_replay_pivots(Solver *s, long long step, int site, const int *J, int nJ,
                          const int *I, int nI);
int solver_get_pivots(Solver *s, int site, int *J, int capJ, int *nJ, int *I, int capI,
                      int *nI);
struct Grid;
Grid *grid_create(const tt_fv_params *p, void *stream);
void grid_step(Grid *s, double *U, double dt, int nsteps);
void grid_destroy(Grid *s);
void grid_set_terms(Grid *s, const tt_fv_term *terms, int count);
struct Ensemble;
Ensemble *ensemble_create(int workers, size_t arena_bytes);
void ensemble_destroy(Ensemble *e);
void ensemble_step(Ensemble *e, Solver *const *members, int count, const double *dts,
                   int nsteps, int concurrency);

namespace {
thread_local std::string g_last_error;
}

void set_last_error(const std::string &m) { g_last_error = m; }

Arena::~Arena() {
  if (base_ && owned_) (void)hipFree(base_);
}

constexpr size_t kArenaHeader = 256;   // status words (Arena::status)

void Arena::init(size_t bytes) {
  TT_REQUIRE(base_ == nullptr, "arena already initialised");
  TT_REQUIRE(bytes > kArenaHeader, "arena too small");
  HIP_CHECK(hipMalloc(&base_, bytes));
  owned_ = true;
  HIP_CHECK(hipMemset(base_, 0, kArenaHeader));
  cap_ = bytes;
  top_ = hw_ = kArenaHeader;
}

void Arena::adopt(void *base, size_t bytes) {
  TT_REQUIRE(base_ == nullptr, "arena already initialised");
  TT_REQUIRE(base && bytes > kArenaHeader && ((uintptr_t)base & 255) == 0,
             "arena: bad caller memory");
  base_ = static_cast<char *>(base);
  owned_ = false;
  cap_ = bytes;
  top_ = hw_ = kArenaHeader;
}

void *Arena::alloc(size_t bytes) {
  const size_t a = (top_ + 255) & ~(size_t)255;
  if (a + bytes > cap_)
    throw Error(TT_ENOMEM, "arena exhausted: need " + std::to_string(a + bytes) + " of " +
                               std::to_string(cap_) + " bytes");
  top_ = a + bytes;
  hw_ = std::max(hw_, top_);
  return base_ + a;
}

void Ctx::sync() {
  if (capturing) return;   // nothing runs before the graph is launched
  if (no_alloc) {          // creates no event
    HIP_CHECK(hipStreamSynchronize(stream));
    return;
  }
  // an event with default flags is waited for by polling, which wakes the host sooner than a
  // stream synchronisation that may yield the thread
  if (!sync_ev) HIP_CHECK(hipEventCreateWithFlags(&sync_ev, hipEventDisableTiming));
  HIP_CHECK(hipEventRecord(sync_ev, stream));
  HIP_CHECK(hipEventSynchronize(sync_ev));
  // every sampled launch on this stream has ended: resolve its event pair (a pair HIP cannot
  // time is dropped from the sample) and recycle the events
  std::vector<KernelTimer::Rec> done;
  done.swap(timer.pending);
  for (const auto &r : done) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.start, r.stop) == hipSuccess) {
      timer.ms += ms;
      timer.flops += r.flops;
      timer.bytes += r.bytes;
      timer.launches++;
    }
    timer.spare.push_back({r.start, r.stop});
  }
}

int Ctx::jacobi_capped() {
  int v = 0;
  HIP_CHECK(hipMemcpyAsync(&v, arena.status(), sizeof(int), hipMemcpyDeviceToHost, stream));
  sync();
  return v;
}

int jacobi_warning(Ctx &c) {
  const int n = c.jacobi_capped();
  const int w = n > c.jacobi_seen ? TT_WJACOBI : 0;
  c.jacobi_seen = n;
  c.cnt.warnings |= w;
  return w;
}

constexpr int kTileCounters = 16384;

int *Ctx::tile_counters() {
  if (!tile_cnt) {
    if (no_alloc) throw Error(TT_EINVAL, "no_alloc context without tile counters");
    HIP_CHECK(hipMalloc(&tile_cnt, kTileCounters * sizeof(int)));
    HIP_CHECK(hipMemsetAsync(tile_cnt, 0, kTileCounters * sizeof(int), stream));
  }
  return tile_cnt;
}

void Ctx::prepare(int term_events) {
  if (no_alloc) return;
  (void)tile_counters();
  (void)pinned_staging();
  if (!sync_ev) HIP_CHECK(hipEventCreateWithFlags(&sync_ev, hipEventDisableTiming));
  while ((int)term_ev.size() < term_events) {
    hipEvent_t e;
    HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    term_ev.push_back(e);
  }
  HIP_CHECK(hipStreamSynchronize(stream));
}

double *Ctx::pinned_staging() {
  if (no_alloc) return nullptr;
  if (!pinned) HIP_CHECK(hipHostMalloc((void **)&pinned, kPinnedDoubles * sizeof(double)));
  return pinned;
}

Ctx::~Ctx() {
  if (tile_cnt || pinned) (void)hipStreamSynchronize(stream);
  if (sync_ev) (void)hipEventDestroy(sync_ev);
  for (hipEvent_t e : term_ev) (void)hipEventDestroy(e);
  if (tile_cnt && !no_alloc) (void)hipFree(tile_cnt);
  if (pinned) (void)hipHostFree(pinned);
  for (auto &e : timer.spare) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  for (auto &e : timer.pending) {
    (void)hipEventDestroy(e.start);
    (void)hipEventDestroy(e.stop);
  }
}

TimedLaunch::TimedLaunch(Ctx &ctx, const char *name, double flops, double bytes)
    : c(ctx), on(false) {
  const std::string &fam = c.timer.name;
  if (fam.empty() || std::strncmp(name, fam.c_str(), fam.size()) != 0) return;
  if ((c.timer.seen++ % c.timer.every) != 0) return;   // a sample keeps the cost small
  if (c.timer.spare.empty()) {
    hipEvent_t a = nullptr, b = nullptr;
    HIP_CHECK(hipEventCreate(&a));
    if (hipEventCreate(&b) != hipSuccess) {
      (void)hipEventDestroy(a);
      throw Error(TT_EHIP, "hipEventCreate failed");
    }
    c.timer.spare.push_back({a, b});
  }
  const auto ev = c.timer.spare.back();
  c.timer.spare.pop_back();
  c.timer.pending.push_back({ev.first, ev.second, flops, bytes});
  c.ev_start = ev.first;
  c.ev_stop = ev.second;
  on = true;
}

TimedLaunch::~TimedLaunch() {
  if (!on) return;
  c.ev_start = nullptr;
  c.ev_stop = nullptr;
}

DTT view(const tt_matrix *m) {
  DTT t;
  t.n1 = m->n1;
  t.n2 = m->n2;
  t.r = m->rank;
  t.A = m->g1;
  t.B = m->g2;
  return t;
}

void check_matrix(const tt_matrix *m, const char *what, bool need_rank) {
  if (!m) throw Error(TT_EINVAL, std::string(what) + ": null tt_matrix");
  if (m->n1 < 1 || m->n2 < 1) throw Error(TT_EINVAL, std::string(what) + ": bad mode sizes");
  if (!m->g1 || !m->g2) throw Error(TT_EINVAL, std::string(what) + ": null core pointer");
  if (need_rank && (m->rank < 1 || m->rank > m->cap))
    throw Error(TT_EINVAL, std::string(what) + ": rank out of [1, cap]");
}

}  // namespace ttfv

// ---------------------------------------------------------------------------------------
// Scratch of tt_round_noalloc: one fixed device array, held on every GPU the library runs on
// until the process ends.  Layout: split-K arrival counters (kScratchCounterBytes), then an
// arena (its first 256 bytes are status words).  Host code never uses the array's name as an
// address: each GPU's copy is reached through the pointer hipGetSymbolAddress returns with
// that GPU current, fetched once per device.
namespace ttfv {
namespace {

constexpr size_t kScratchCounterBytes = (size_t)kTileCounters * sizeof(int);
static_assert(kScratchCounterBytes % 256 == 0, "arena part must stay 256-byte aligned");

__device__ __align__(256) unsigned char scratch[TT_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::map<int, unsigned char *> g_scratch_addr;   // device -> its copy of `scratch`

unsigned char *scratch_address(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(dev);
  if (it != g_scratch_addr.end()) return it->second;
  unsigned char *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || ptr == nullptr)
    throw Error(TT_EHIP, std::string("tt_round_noalloc: hipGetSymbolAddress(scratch): ") +
                             hipGetErrorString(e));
  g_scratch_addr[dev] = ptr;
  return ptr;
}

}  // namespace
}  // namespace ttfv

struct tt_ctx {
  ttfv::Ctx c;
};

struct tt_fv {
  ttfv::Solver *s;
};

struct tt_ens {
  ttfv::Ensemble *e;
};

struct tt_pm {
  std::unique_ptr<ttfv::PivotModel> m;
};

using namespace ttfv;

template <typename F>
static int guarded(F &&f) {
  try {
    return f();
  } catch (const Error &e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::exception &e) {
    set_last_error(e.what());
    return TT_EINVAL;
  }
}

// the fiber description of a cross's entry function fn (TT_FN_*) over its inputs; ghost
// extensions of WENO inputs are allocated on the context's arena (the caller's scope)
static FiberSpec make_fiber_spec(Ctx &c, int fn, const tt_matrix *inputs, int n_inputs,
                                 const double *fparams, int n1, int n2) {
  static WenoTables wt = derive_weno_tables();
  FiberSpec fs;
  fs.fn = fn;
  fs.wt = &wt;
  switch (fn) {
    case TT_FN_IDENTITY:
    case TT_FN_RECIP:
      TT_REQUIRE(n_inputs == 1, "identity/recip: one input");
      check_matrix(&inputs[0], "input", true);
      TT_REQUIRE(inputs[0].n1 == n1 && inputs[0].n2 == n2, "identity: input shape");
      fs.n_in = 1;
      fs.in[0] = {inputs[0].g1, inputs[0].g2, n1, n2, inputs[0].rank};
      break;
    case TT_FN_LLF_LAMBDA:
      TT_REQUIRE(n_inputs == 4 && fparams, "lambda: four inputs and g");
      for (int t = 0; t < 4; ++t) {
        check_matrix(&inputs[t], "input", true);
        TT_REQUIRE(inputs[t].n1 == n1 && inputs[t].n2 == n2, "lambda: input shape");
        fs.in[t] = {inputs[t].g1, inputs[t].g2, n1, n2, inputs[t].rank};
      }
      fs.n_in = 4;
      fs.g = fparams[0];
      break;
    case TT_FN_LLF_FLUX:
      TT_REQUIRE(n_inputs == 6 && fparams, "llf flux: six inputs and g");
      TT_REQUIRE(n2 % 3 == 0, "llf flux: n2 must be 3 x the inputs' columns");
      for (int t = 0; t < 6; ++t) {
        check_matrix(&inputs[t], "input", true);
        TT_REQUIRE(inputs[t].n1 == n1 && inputs[t].n2 * 3 == n2, "llf flux: input shape");
        fs.in[t] = {inputs[t].g1, inputs[t].g2, n1, n2 / 3, inputs[t].rank};
      }
      fs.n_in = 6;
      fs.g = fparams[0];
      fs.ncol = n2 / 3;
      break;
    case TT_FN_WENO_FACE_M:
    case TT_FN_WENO_FACE_P: {
      TT_REQUIRE(n_inputs == 1 && fparams, "weno face: one input and params");
      const tt_matrix &v = inputs[0];
      check_matrix(&v, "input", true);
      const bool per = fparams[0] != 0.0;
      TT_REQUIRE(v.n2 == n2 && n1 == (per ? v.n1 : v.n1 + 1) && v.n1 >= 3,
                 "weno face: shapes (n_f x n from an n x n input)");
      double *Ae = c.arena.dalloc((size_t)(v.n1 + 6) * v.rank);
      ghost_extend(c, v.g1, v.n1, v.rank, per ? Ghost::Periodic : Ghost::Wall, fparams[1], Ae);
      fs.n_in = 1;
      fs.in[0] = {Ae, v.g2, v.n1 + 6, v.n2, v.rank};
      fs.eps_w = fparams[2];
      break;
  }
  case TT_FN_WENO_QUAD: {
    TT_REQUIRE(n_inputs == 1 && fparams, "weno quad: one input and params");
    const tt_matrix &v = inputs[0];
    check_matrix(&v, "input", true);
    TT_REQUIRE(v.n1 == n1 && n2 == 3 * v.n2 && v.n2 >= 3, "weno quad: shapes (n_f x 3n)");
    double *Be = c.arena.dalloc((size_t)(v.n2 + 6) * v.rank);
    ghost_extend(c, v.g2, v.n2, v.rank, fparams[0] != 0.0 ? Ghost::Periodic : Ghost::Wall,
                 fparams[1], Be);
    fs.n_in = 1;
    fs.in[0] = {v.g1, Be, v.n1, v.n2 + 6, v.rank};
    fs.eps_w = fparams[2];
    fs.nq = 3;
    break;
  }
  default:
    throw Error(TT_EINVAL, "tt_cross: unknown fn id");
  }
  return fs;
}

extern "C" {

const char *tt_last_error(void) { return g_last_error.c_str(); }

int tt_ctx_create(tt_ctx **out, size_t arena_bytes, void *hip_stream) {
  return guarded([&]() {
    TT_REQUIRE(out, "tt_ctx_create: null out");
    TT_REQUIRE(arena_bytes >= ((size_t)1 << 20), "tt_ctx_create: arena below 1 MiB");
    tt_ctx *c = new tt_ctx();
    try {
      c->c.stream = (hipStream_t)hip_stream;
      c->c.arena.init(arena_bytes);
      c->c.prepare();
    } catch (...) {
      delete c;
      throw;
    }
    *out = c;
    return 0;
  });
}

void tt_ctx_destroy(tt_ctx *ctx) { delete ctx; }

int tt_ctx_set_sketch(tt_ctx *ctx, int width, int power_iters) {
  return guarded([&]() {
    TT_REQUIRE(ctx, "null ctx");
    TT_REQUIRE(width >= 0 && width <= QR_MAXM, "sketch width out of [0, 96]");
    TT_REQUIRE(power_iters >= 0 && power_iters <= 8, "power_iters out of [0, 8]");
    ctx->c.sketch_width = width;
    ctx->c.power_iters = power_iters;
    return 0;
  });
}

int tt_ctx_set_limits(tt_ctx *ctx, int jacobi_max_sweeps, int sketch_max_iters) {
  return guarded([&]() {
    TT_REQUIRE(ctx, "null ctx");
    TT_REQUIRE(jacobi_max_sweeps >= 1 && jacobi_max_sweeps <= 100,
               "jacobi_max_sweeps out of [1, 100]");
    TT_REQUIRE(sketch_max_iters >= 0 && sketch_max_iters <= 16,
               "sketch_max_iters out of [0, 16]");
    ctx->c.jacobi_max_sweeps = jacobi_max_sweeps;
    ctx->c.sketch_max_iters = sketch_max_iters;
    return 0;
  });
}

int tt_ctx_set_precision(tt_ctx *ctx, int precision) {
  return guarded([&]() {
    TT_REQUIRE(ctx, "null ctx");
    TT_REQUIRE(precision == TT_PREC_F64 || precision == TT_PREC_F32, "unknown precision");
    ctx->c.fp32 = precision == TT_PREC_F32;
    return 0;
  });
}

int tt_ctx_set_qr(tt_ctx *ctx, int method, int max_passes) {
  return guarded([&]() {
    TT_REQUIRE(ctx, "null ctx");
    TT_REQUIRE(method == TT_QR_AUTO || method == TT_QR_CHOLESKY || method == TT_QR_HOUSEHOLDER,
               "unknown QR method");
    TT_REQUIRE(max_passes >= 2 && max_passes <= 8, "max_passes out of [2, 8]");
    ctx->c.qr = method;
    ctx->c.cqr_passes = max_passes;
    return 0;
  });
}

int tt_ctx_set_enrichment(tt_ctx *ctx, int mode) {
  return guarded([&]() {
    TT_REQUIRE(ctx, "null ctx");
    TT_REQUIRE(mode == TT_ENRICH_KICKS || mode == TT_ENRICH_RESIDUAL,
               "tt_ctx_set_enrichment: unknown mode");
    ctx->c.enrich = mode;
    return 0;
  });
}

int tt_ctx_set_fixed(tt_ctx *ctx, int on) {
  return guarded([&]() {
    TT_REQUIRE(ctx, "null ctx");
    TT_REQUIRE(on == 0 || on == 1, "tt_ctx_set_fixed: on must be 0 or 1");
    ctx->c.fixed = on == 1;
    ctx->c.householder = on == 1;
    return 0;
  });
}

int tt_rule_trunc_rank(const double *s, int m, double eps, int r_max, double floor_rel,
                       int *capped) {
  return guarded([&]() {
    TT_REQUIRE(s && m >= 1 && m <= 128 && r_max >= 1, "tt_rule_trunc_rank: bad arguments");
    double tail[129];
    bool cap = false;
    const int k = rule_trunc_rank(s, m, eps, r_max, floor_rel, tail, &cap);
    if (capped) *capped = cap ? 1 : 0;
    return k;
  });
}

int tt_rule_kicks(const int *have, int nhave, int n, int count, uint64_t key, int *out) {
  return guarded([&]() {
    TT_REQUIRE((have || nhave == 0) && (out || count == 0) && nhave >= 0 && nhave <= 4096 &&
                   count >= 0 && count <= 4096 && n >= 1,
               "tt_rule_kicks: bad arguments");
    std::vector<int> J(have, have + nhave);
    J.resize((size_t)nhave + count);
    const int added = count ? rule_kicks(J.data(), nhave, n, count, key) : 0;
    for (int i = 0; i < added; ++i) out[i] = J[(size_t)nhave + i];
    return added;
  });
}

int tt_round(tt_ctx *ctx, const tt_matrix *x, double eps, int r_max, tt_matrix *y,
             double *sigma_out) {
  return guarded([&]() {
    TT_REQUIRE(ctx, "null ctx");
    check_matrix(x, "tt_round x", true);
    check_matrix(y, "tt_round y", false);
    TT_REQUIRE(eps >= 0.0 && r_max >= 1, "tt_round: eps < 0 or r_max < 1");
    TT_REQUIRE(y->cap >= r_max, "tt_round: y->cap < r_max");
    TT_REQUIRE(x->n1 == y->n1 && x->n2 == y->n2, "tt_round: shape mismatch");
    DTT xv = view(x), yv = view(y);
    if (ctx->c.fixed) {
      // the rank chosen on the device; the buffers' columns after it up to the static rank
      // are zero
      Scope sc(ctx->c.arena);
      int *kd = ctx->c.arena.ialloc(1);
      round_fixed(ctx->c, xv, eps, r_max, yv, kd);
      int k = 0;
      HIP_CHECK(hipMemcpyAsync(&k, kd, sizeof(int), hipMemcpyDeviceToHost, ctx->c.stream));
      const int w = fixed_status(ctx->c);
      y->rank = std::max(k, 1);
      return w | jacobi_warning(ctx->c);
    }
    std::vector<double> s;
    const int w = round_tt(ctx->c, xv, eps, r_max, yv, &s);
    y->rank = yv.r;
    if (sigma_out)
      for (size_t i = 0; i < s.size(); ++i) sigma_out[i] = s[i];
    return w | jacobi_warning(ctx->c);
  });
}

int tt_round_nd(tt_ctx *ctx, const tt_tensor *x, double eps, int r_max, tt_tensor *y,
                double *sigma_out) {
  return guarded([&]() {
    TT_REQUIRE(ctx && x && y, "tt_round_nd: null argument");
    TT_REQUIRE(x->d >= 2 && x->d == y->d && x->n && x->r && x->cores && y->n && y->r && y->cores,
               "tt_round_nd: bad tensors");
    TT_REQUIRE(eps >= 0.0 && r_max >= 1, "tt_round_nd: eps < 0 or r_max < 1");
    for (int k = 0; k < x->d; ++k) {
      TT_REQUIRE(x->n[k] == y->n[k], "tt_round_nd: modes differ");
      TT_REQUIRE(x->cores[k] && y->cores[k], "tt_round_nd: null core");
    }
    std::vector<double> s;
    const int w = round_nd(ctx->c, x->d, x->n, x->r, x->cores, eps, r_max, y->cores, y->r, &s);
    if (sigma_out)
      for (size_t i = 0; i < s.size(); ++i) sigma_out[i] = s[i];
    return w | jacobi_warning(ctx->c);
  });
}

int tt_compress(tt_ctx *ctx, const double *F, int n1, int n2, int ld, double eps, int r_max,
                tt_matrix *y, double *sigma_out) {
  return guarded([&]() {
    TT_REQUIRE(ctx && F, "tt_compress: null argument");
    check_matrix(y, "tt_compress y", false);
    TT_REQUIRE(n1 >= 1 && n2 >= 1 && ld >= n1, "tt_compress: bad shape or leading dimension");
    TT_REQUIRE(eps >= 0.0 && r_max >= 1, "tt_compress: eps < 0 or r_max < 1");
    TT_REQUIRE(y->n1 == n1 && y->n2 == n2 && y->cap >= r_max, "tt_compress: y shape or cap");
    DTT yv = view(y);
    std::vector<double> s;
    const int w = compress_dense(ctx->c, F, n1, n2, ld, eps, r_max, yv, &s);
    y->rank = yv.r;
    if (sigma_out)
      for (size_t i = 0; i < s.size(); ++i) sigma_out[i] = s[i];
    return w | jacobi_warning(ctx->c);
  });
}

int tt_round_noalloc(const tt_matrix *x, double eps, int r_max, tt_matrix *y,
                     double *sigma_out, void *hip_stream) {
  return guarded([&]() {
    check_matrix(x, "tt_round_noalloc x", true);
    check_matrix(y, "tt_round_noalloc y", false);
    TT_REQUIRE(eps >= 0.0 && r_max >= 1, "tt_round_noalloc: eps < 0 or r_max < 1");
    TT_REQUIRE(y->cap >= r_max, "tt_round_noalloc: y->cap < r_max");
    TT_REQUIRE(x->n1 == y->n1 && x->n2 == y->n2, "tt_round_noalloc: shape mismatch");
    const size_t need = round_arena_bound(x->n1, x->n2, x->rank, r_max) + kScratchCounterBytes;
    if (need > TT_NOALLOC_SCRATCH_BYTES)
      throw Error(TT_ENOMEM, "tt_round_noalloc: a " + std::to_string(x->n1) + " x " +
                                 std::to_string(x->n2) + " TT of rank " +
                                 std::to_string(x->rank) + " may need " + std::to_string(need) +
                                 " bytes of scratch; the fixed maximum is " +
                                 std::to_string((size_t)TT_NOALLOC_SCRATCH_BYTES));
    int dev = 0;
    HIP_CHECK(hipGetDevice(&dev));
    unsigned char *base = scratch_address(dev);
    Ctx c;
    c.no_alloc = true;
    c.stream = (hipStream_t)hip_stream;
    c.tile_cnt = reinterpret_cast<int *>(base);
    c.arena.adopt(base + kScratchCounterBytes, TT_NOALLOC_SCRATCH_BYTES - kScratchCounterBytes);
    // the split-K arrival counters and the arena's status words start at zero (a fill
    // kernel, not a memset node, so the call may also be captured)
    const int nz = (int)((kScratchCounterBytes + 256) / sizeof(double));
    fill_value(c, reinterpret_cast<double *>(base), nz, nz, 1, 0.0);
    DTT xv = view(x), yv = view(y);
    std::vector<double> s;
    const int w = round_tt(c, xv, eps, r_max, yv, &s);
    y->rank = yv.r;
    if (sigma_out)
      for (size_t i = 0; i < s.size(); ++i) sigma_out[i] = s[i];
    return w | jacobi_warning(c);
  });
}

int tt_hadamard_round(tt_ctx *ctx, const tt_matrix *x, const tt_matrix *z, double eps, int r_max,
                      tt_matrix *y) {
  return guarded([&]() {
    TT_REQUIRE(ctx, "null ctx");
    check_matrix(x, "tt_hadamard_round x", true);
    check_matrix(z, "tt_hadamard_round z", true);
    check_matrix(y, "tt_hadamard_round y", false);
    TT_REQUIRE(x->n1 == z->n1 && x->n2 == z->n2 && x->n1 == y->n1 && x->n2 == y->n2,
               "tt_hadamard_round: shape mismatch");
    TT_REQUIRE(y->cap >= r_max && r_max >= 1 && eps >= 0.0, "tt_hadamard_round: bad cap/eps");
    Ctx &c = ctx->c;
    Scope sc(c.arena);
    const int R = x->rank * z->rank;
    DTT p{x->n1, x->n2, R, c.arena.dalloc((size_t)x->n1 * R), c.arena.dalloc((size_t)x->n2 * R)};
    khatri_rao(c, p.A, x->n1, x->g1, x->rank, z->g1, z->rank);
    khatri_rao(c, p.B, x->n2, x->g2, x->rank, z->g2, z->rank);
    DTT yv = view(y);
    const int w = round_tt(c, p, eps, r_max, yv, nullptr);
    y->rank = yv.r;
    return w | jacobi_warning(ctx->c);
  });
}

int tt_reciprocal(tt_ctx *ctx, const tt_matrix *x, double eps, int max_terms, int r_max,
                  tt_matrix *y, double *err_out, int *terms_out) {
  return guarded([&]() {
    TT_REQUIRE(ctx, "null ctx");
    check_matrix(x, "tt_reciprocal x", true);
    check_matrix(y, "tt_reciprocal y", false);
    TT_REQUIRE(x->n1 == y->n1 && x->n2 == y->n2, "tt_reciprocal: shape mismatch");
    TT_REQUIRE(max_terms >= 1 && r_max >= 1 && eps >= 0.0 && y->cap >= r_max,
               "tt_reciprocal: bad max_terms / r_max / eps / cap");
    DTT xv = view(x), yv = view(y);
    const int w = reciprocal_tt(ctx->c, xv, eps, max_terms, r_max, yv, err_out, terms_out);
    y->rank = yv.r;
    return w | jacobi_warning(ctx->c);
  });
}

int tt_maxvol(tt_ctx *ctx, const double *q, int n, int r, int ldq, double tau, int maxit,
              int *rows_out) {
  return guarded([&]() {
    TT_REQUIRE(ctx && q && rows_out, "tt_maxvol: null argument");
    TT_REQUIRE(r >= 1 && r <= 96 && n >= r && ldq >= n, "tt_maxvol: bad shape");
    TT_REQUIRE(tau >= 1.0 && maxit >= 0, "tt_maxvol: tau < 1 or maxit < 0");
    std::vector<int> I = maxvol_host(ctx->c, q, n, r, ldq, tau, maxit);
    for (int i = 0; i < r; ++i) rows_out[i] = I[i];
    return 0;
  });
}

int tt_cross(tt_ctx *ctx, int fn, const tt_matrix *inputs, int n_inputs, const double *fparams,
             int n1, int n2, const int *J0, int nJ0, double eps, int r_max, int sweeps, int kick,
             uint64_t key, tt_matrix *y, int *J_out, int *nJ_out) {
  return guarded([&]() {
    TT_REQUIRE(ctx && inputs && J0 && y, "tt_cross: null argument");
    check_matrix(y, "tt_cross y", false);
    TT_REQUIRE(y->n1 == n1 && y->n2 == n2 && y->cap >= r_max, "tt_cross: bad output");
    TT_REQUIRE(r_max >= 1 && r_max <= 64 && eps >= 0.0 && sweeps >= 1 && kick >= 0,
               "tt_cross: bad r_max / eps / sweeps / kick");
    TT_REQUIRE(nJ0 >= 1, "tt_cross: empty J0");
    std::vector<int> J(J0, J0 + nJ0);
    for (int j : J) TT_REQUIRE(j >= 0 && j < n2, "tt_cross: J0 index out of range");
    Ctx &c = ctx->c;
    Scope sc(c.arena);
    FiberSpec fs = make_fiber_spec(c, fn, inputs, n_inputs, fparams, n1, n2);
    DTT yv = view(y);
    std::vector<int> Jo;
    if (c.fixed) {
      // device column set of r_max entries; the kicks' key split into (site, step) words
      TT_REQUIRE(nJ0 <= r_max, "tt_cross: fixed shapes need nJ0 <= r_max");
      int *Jd = c.arena.ialloc(r_max + 1), *kd = c.arena.ialloc(1);
      long long *sd = static_cast<long long *>(c.arena.alloc(sizeof(long long)));
      std::vector<int> h(r_max + 1, 0);
      std::copy(J.begin(), J.end(), h.begin());
      h[r_max] = nJ0;
      const long long step = (long long)(key & 0xFFFFFFFFull);
      HIP_CHECK(hipMemcpyAsync(Jd, h.data(), h.size() * sizeof(int), hipMemcpyHostToDevice,
                               c.stream));
      HIP_CHECK(hipMemcpyAsync(sd, &step, sizeof(step), hipMemcpyHostToDevice, c.stream));
      cross_fixed(c, fs, n1, n2, Jd, Jd + r_max, r_max, eps, r_max, sweeps, kick, key >> 32, sd,
                  yv, kd);
      int k = 0;
      HIP_CHECK(hipMemcpyAsync(h.data(), Jd, h.size() * sizeof(int), hipMemcpyDeviceToHost,
                               c.stream));
      HIP_CHECK(hipMemcpyAsync(&k, kd, sizeof(int), hipMemcpyDeviceToHost, c.stream));
      const int w = fixed_status(c);
      y->rank = std::max(k, 1);
      if (J_out)
        for (int i = 0; i < h[r_max]; ++i) J_out[i] = h[i];
      if (nJ_out) *nJ_out = h[r_max];
      return w | jacobi_warning(ctx->c);
    }
    const int w = cross_tt(c, fs, n1, n2, J, eps, r_max, sweeps, kick, key, yv, &Jo);
    y->rank = yv.r;
    if (J_out)
      for (size_t i = 0; i < Jo.size(); ++i) J_out[i] = Jo[i];
    if (nJ_out) *nJ_out = (int)Jo.size();
    return w | jacobi_warning(ctx->c);
  });
}

int tt_recon_core(tt_ctx *ctx, const double *core, int n, int rank, int scheme, int periodic,
                  double sign, double *face_m, double *face_p, double *quad) {
  return guarded([&]() {
    TT_REQUIRE(ctx && core, "tt_recon_core: null argument");
    TT_REQUIRE(n >= 3 && rank >= 1, "tt_recon_core: n >= 3 and rank >= 1");
    TT_REQUIRE(scheme == 3 || scheme == 5, "tt_recon_core: scheme must be 3 or 5");
    StencilSet st = derive_stencils(scheme);
    const int nf = periodic ? n : n + 1;
    if (face_m && face_p)
      recon_face(ctx->c, core, n, rank, periodic ? Ghost::Periodic : Ghost::Wall, sign, st,
                 face_m, face_p, nf);
    if (quad)
      recon_quad(ctx->c, core, n, rank, periodic ? Ghost::Periodic : Ghost::Wall, sign, st,
                 quad);
    ctx->c.sync();
    return 0;
  });
}

struct tt_grid {
  ttfv::Grid *g;
};

int tt_grid_init(tt_grid **out, const tt_fv_params *p, void *hip_stream) {
  return guarded([&]() {
    TT_REQUIRE(out, "tt_grid_init: null out");
    *out = new tt_grid{grid_create(p, hip_stream)};
    return 0;
  });
}

int tt_grid_step(tt_grid *s, double *U, double dt, int nsteps) {
  return guarded([&]() {
    TT_REQUIRE(s, "null grid solver");
    grid_step(s->g, U, dt, nsteps);
    return 0;
  });
}

int tt_grid_set_terms(tt_grid *s, const tt_fv_term *terms, int count) {
  return guarded([&]() {
    TT_REQUIRE(s, "null grid solver");
    grid_set_terms(s->g, terms, count);
    return 0;
  });
}

void tt_grid_destroy(tt_grid *s) {
  if (!s) return;
  grid_destroy(s->g);
  delete s;
}

int tt_fv_init(tt_fv **out, const tt_fv_params *p, const tt_matrix q0[3], void *hip_stream,
               size_t arena_bytes) {
  return guarded([&]() {
    TT_REQUIRE(out, "tt_fv_init: null out");
    for (int v = 0; v < 3; ++v) check_matrix(&q0[v], "tt_fv_init q0", true);
    Solver *s = solver_create(p, q0, hip_stream, arena_bytes);
    *out = new tt_fv{s};
    return 0;
  });
}

int tt_fv_step(tt_fv *s, double dt, int nsteps) {
  return guarded([&]() {
    TT_REQUIRE(s, "null solver");
    solver_step(s->s, dt, nsteps);
    tt_fv_stats st{};
    solver_stats(s->s, &st);
    return st.warnings & (TT_WRANKCAP | TT_WNOCONV);
  });
}

int tt_fv_max_speed(tt_fv *s, double speed[2]) {
  return guarded([&]() {
    TT_REQUIRE(s && speed, "null argument");
    solver_max_speed(s->s, speed);
    return 0;
  });
}

int tt_fv_cfl_dt(tt_fv *s, double cfl, double *dt) {
  return guarded([&]() {
    TT_REQUIRE(s && dt, "null argument");
    TT_REQUIRE(cfl > 0.0 && std::isfinite(cfl), "tt_fv_cfl_dt: cfl must be positive");
    *dt = solver_cfl_dt(s->s, cfl);
    return 0;
  });
}

int tt_fv_set_terms(tt_fv *s, const tt_fv_term *terms, int count) {
  return guarded([&]() {
    TT_REQUIRE(s, "null solver");
    solver_set_terms(s->s, terms, count);
    return 0;
  });
}

int tt_fv_get_state(tt_fv *s, tt_matrix q[3]) {
  return guarded([&]() {
    TT_REQUIRE(s && q, "null argument");
    solver_get_state(s->s, q);
    return 0;
  });
}

int tt_fv_time_kernel(tt_fv *s, const char *name, int every) {
  return guarded([&]() {
    TT_REQUIRE(s, "null solver");
    TT_REQUIRE(every >= 1, "tt_fv_time_kernel: every < 1");
    solver_time_kernel(s->s, name ? name : "", every);
    return 0;
  });
}

int tt_fv_get_stats(tt_fv *s, tt_fv_stats *out) {
  return guarded([&]() {
    TT_REQUIRE(s && out, "null argument");
    solver_stats(s->s, out);
    return 0;
  });
}

int tt_ens_create(tt_ens **out, int workers, size_t arena_bytes_per_worker) {
  return guarded([&]() {
    TT_REQUIRE(out, "tt_ens_create: null out");
    Ensemble *e = ensemble_create(workers, arena_bytes_per_worker);
    *out = new tt_ens{e};
    return 0;
  });
}

int tt_ens_step(tt_ens *e, tt_fv *const *members, int count, const double *dts, int nsteps,
                int concurrency) {
  return guarded([&]() {
    TT_REQUIRE(e && members && count >= 1, "tt_ens_step: null argument");
    TT_REQUIRE(nsteps >= 0, "tt_ens_step: nsteps < 0");
    std::vector<Solver *> m(count);
    for (int i = 0; i < count; ++i) {
      TT_REQUIRE(members[i], "tt_ens_step: null member");
      m[i] = members[i]->s;
    }
    ensemble_step(e->e, m.data(), count, dts, nsteps, concurrency);
    int w = 0;
    for (int i = 0; i < count; ++i) {
      tt_fv_stats st{};
      solver_stats(m[i], &st);
      w |= st.warnings & (TT_WRANKCAP | TT_WNOCONV);
    }
    return w;
  });
}

void tt_ens_destroy(tt_ens *e) {
  if (!e) return;
  ensemble_destroy(e->e);
  delete e;
}

void tt_fv_destroy(tt_fv *s) {
  if (!s) return;
  solver_destroy(s->s);
  delete s;
}

}  // extern "C"

// ---- learned pivot proposer -------------------------------------------------------------

int tt_pm_create(tt_pm **out, size_t max_rows, unsigned long long seed) {
  return guarded([&]() {
    TT_REQUIRE(out, "null argument");
    auto *h = new tt_pm();
    try {
      h->m = std::make_unique<PivotModel>(max_rows, (uint64_t)seed);
    } catch (...) {
      delete h;
      throw;
    }
    *out = h;
    return 0;
  });
}

void tt_pm_destroy(tt_pm *pm) { delete pm; }

int tt_pm_set_weights(tt_pm *pm, const float *host, size_t n) {
  return guarded([&]() {
    TT_REQUIRE(pm && host && n == PM_NPARAM, "tt_pm_set_weights: null or n != TT_PM_NPARAM");
    pm->m->set_weights(host);
    return 0;
  });
}

int tt_pm_get_weights(tt_pm *pm, float *host, size_t n) {
  return guarded([&]() {
    TT_REQUIRE(pm && host && n == PM_NPARAM, "tt_pm_get_weights: null or n != TT_PM_NPARAM");
    pm->m->get_weights(host);
    return 0;
  });
}

int tt_pm_forward(tt_pm *pm, const float *X_dev, int N, float *s_dev) {
  return guarded([&]() {
    TT_REQUIRE(pm && X_dev && s_dev && N >= 1, "tt_pm_forward: bad argument");
    PivotModel &m = *pm->m;
    std::lock_guard<std::mutex> lk(m.mu);
    Scope sc(m.c.arena);
    bf16_t *Xb = static_cast<bf16_t *>(m.c.arena.alloc((size_t)N * PM_F * sizeof(bf16_t)));
    to_bf16(m.c, X_dev, (size_t)N * PM_F, Xb);
    m.forward(m.c, Xb, N, s_dev, nullptr, nullptr);
    m.c.sync();
    return 0;
  });
}

int tt_pm_grad(tt_pm *pm, const float *X_dev, const float *y_dev, int N, double pos_weight,
               float *grad_host, size_t n, double *loss_out) {
  return guarded([&]() {
    TT_REQUIRE(pm && X_dev && y_dev && grad_host && N >= 1 && n == PM_NPARAM,
               "tt_pm_grad: bad argument");
    PivotModel &m = *pm->m;
    std::lock_guard<std::mutex> lk(m.mu);
    Scope sc(m.c.arena);
    bf16_t *Xb = static_cast<bf16_t *>(m.c.arena.alloc((size_t)N * PM_F * sizeof(bf16_t)));
    to_bf16(m.c, X_dev, (size_t)N * PM_F, Xb);
    const double l = m.grad(m.c, Xb, y_dev, N, pos_weight);
    HIP_CHECK(hipMemcpyAsync(grad_host, m.g, PM_NPARAM * sizeof(float), hipMemcpyDeviceToHost,
                             m.c.stream));
    m.c.sync();
    if (loss_out) *loss_out = l;
    return 0;
  });
}

int tt_pm_adam(tt_pm *pm, const float *grad_host, size_t n, double lr) {
  return guarded([&]() {
    TT_REQUIRE(pm && grad_host && n == PM_NPARAM && lr > 0.0, "tt_pm_adam: bad argument");
    PivotModel &m = *pm->m;
    std::lock_guard<std::mutex> lk(m.mu);
    HIP_CHECK(hipMemcpyAsync(m.g, grad_host, PM_NPARAM * sizeof(float), hipMemcpyHostToDevice,
                             m.c.stream));
    m.adam(m.c, lr);
    m.refresh_bf16();
    m.c.sync();
    return 0;
  });
}

int tt_pm_train(tt_pm *pm, int epochs, int batch, double lr, double *loss_out) {
  return guarded([&]() {
    TT_REQUIRE(pm && lr > 0.0, "tt_pm_train: bad argument");
    const double l = pm->m->train(epochs, batch, lr);
    if (loss_out) *loss_out = l;
    return 0;
  });
}

int tt_pm_dataset(tt_pm *pm, size_t *rows, size_t *positives) {
  return guarded([&]() {
    TT_REQUIRE(pm, "null model");
    std::lock_guard<std::mutex> lk(pm->m->mu);
    if (rows) *rows = pm->m->rows;
    if (positives) *positives = pm->m->positives;
    return 0;
  });
}

int tt_pm_features(tt_ctx *ctx, const double *B0, int n2, int r, int ldb, const int *J_dev,
                   int nJ, float *X_dev) {
  return guarded([&]() {
    TT_REQUIRE(ctx && B0 && X_dev && n2 >= 1 && r >= 1 && ldb >= n2 && nJ >= 0 && nJ <= 128 &&
                   (nJ == 0 || J_dev),
               "tt_pm_features: bad argument");
    pivot_features(ctx->c, B0, n2, r, ldb, J_dev, nJ, X_dev, nullptr);
    ctx->c.sync();
    return 0;
  });
}

int tt_pm_topk(tt_ctx *ctx, const float *s_dev, int n, int k, int *idx_dev) {
  return guarded([&]() {
    TT_REQUIRE(ctx && s_dev && idx_dev && n >= 1 && k >= 1 && k <= n, "tt_pm_topk: bad argument");
    topk_indices(ctx->c, s_dev, n, k, idx_dev);
    ctx->c.sync();
    return 0;
  });
}

int tt_fv_set_pivots(tt_fv *s, int mode, tt_pm *pm) {
  return guarded([&]() {
    TT_REQUIRE(s, "null solver");
    TT_REQUIRE(mode == TT_PIV_MAXVOL || mode == TT_PIV_LOG || mode == TT_PIV_LEARNED ||
                   mode == TT_PIV_REPLAY || mode == TT_PIV_KICKS,
               "tt_fv_set_pivots: unknown mode");
    TT_REQUIRE(mode == TT_PIV_MAXVOL || mode == TT_PIV_REPLAY || mode == TT_PIV_KICKS || pm,
               "tt_fv_set_pivots: mode needs a model");
    solver_set_pivots(s->s, mode, pm ? pm->m.get() : nullptr);
    return 0;
  });
}

int tt_fv_set_pivot_acceptance(tt_fv *s, double abs_tol, double rel_slack) {
  return guarded([&]() {
    TT_REQUIRE(s, "null solver");
    TT_REQUIRE(abs_tol >= 0.0 && std::isfinite(abs_tol) && std::isfinite(rel_slack),
               "tt_fv_set_pivot_acceptance: bad tolerance");
    solver_set_acceptance(s->s, abs_tol, rel_slack);
    return 0;
  });
}

int tt_fv_replay_pivots(tt_fv *s, long long step, int site, const int *J, int nJ, const int *I,
                        int nI) {
  return guarded([&]() {
    TT_REQUIRE(s, "null solver");
    solver_replay_pivots(s->s, step, site, J, nJ, I, nI);
    return 0;
  });
}

int tt_fv_get_pivots(tt_fv *s, int site, int *J, int capJ, int *nJ, int *I, int capI, int *nI) {
  return guarded([&]() {
    TT_REQUIRE(s && J && nJ && I && nI, "tt_fv_get_pivots: null argument");
    return solver_get_pivots(s->s, site, J, capJ, nJ, I, capI, nI);
  });
}

int tt_cross_skeleton(tt_ctx *ctx, int fn, const tt_matrix *inputs, int n_inputs,
                      const double *fparams, int n1, int n2, const int *J, int nJ, const int *I,
                      int nI, double eps, int r_max, tt_matrix *y) {
  return guarded([&]() {
    TT_REQUIRE(ctx && inputs && J && y && (I || nI == 0), "tt_cross_skeleton: null argument");
    check_matrix(y, "tt_cross_skeleton y", false);
    TT_REQUIRE(y->n1 == n1 && y->n2 == n2 && y->cap >= r_max, "tt_cross_skeleton: bad output");
    TT_REQUIRE(r_max >= 1 && eps >= 0.0, "tt_cross_skeleton: bad r_max / eps");
    TT_REQUIRE(nJ >= 1 && nI >= 0 && nI <= nJ, "tt_cross_skeleton: bad pivot counts");
    Scope sc(ctx->c.arena);
    FiberSpec fs = make_fiber_spec(ctx->c, fn, inputs, n_inputs, fparams, n1, n2);
    DTT out = view(y);
    const int w = skeleton_tt(ctx->c, fs, n1, n2, std::vector<int>(J, J + nJ),
                              std::vector<int>(I, I + nI), eps, r_max, out);
    y->rank = out.r;
    return w | jacobi_warning(ctx->c);
  });
}

int tt_gemm_autotune(int on, int *classes_out) {
  return guarded([&]() {
    gemm_autotune(on != 0);
    if (classes_out) *classes_out = gemm_tuned_classes();
    return 0;
  });
}
