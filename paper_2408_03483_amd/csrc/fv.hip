// The TT finite-volume step (Section 4) on the GPU.
//
// One right-hand side L(Q) (Sections 4.1-4.3), for the x direction; the y direction is
// the same sequence on the transposed TTs with the momenta swapped, so the normal
// momentum is always the second variable:
//   reconstruction  Upwind: face stencils on the first core, Gauss-point stencils on the
//                   second core, minus/plus states share the second core (Section 4.3.1).
//                   WENO5: Algorithm 2 (two crosses over the five x-shifted copies) and
//                   Algorithm 3 (two crosses over five y-shifts, all Gauss points at once on
//                   the merged column index j*nq + m) (Section 4.3.2).
//   flux            linear: LLF assembled directly, never rounded (Section 4.2).
//                   nonlinear, per side: 1/h by Algorithm 1 or by a cross of 1/x (the
//                   alternative Section 4.2 names), u = round(hu o 1/h),
//                   w = round(hv o 1/h), P1 = round(hu o u), P2 = round(h o h),
//                   F2 = round(P1 + g/2 P2), F3 = round(hu o w); lambda by one cross of
//                   max(|hu-/h-| + sqrt(g h-), |hu+/h+| + sqrt(g h+));
//                   D_c = round(lambda o (q_c+ - q_c-)), Fhat_c = round((F- + F+)/2 - D_c/2).
//                   Or (TT_FLUX_LF_CROSS) the whole LLF flux vector of a direction by one
//                   cross over (face, component x quadrature column): the LF-cross that
//                   Section 4.2 contrasts with the products.
//   finish          Gauss-Legendre sum on the second core, (T - 1) on the first (Section 4.1).
// SSP-RK3 (Section 4.4): Q1 = F(Qn), Q2 = round(3/4 Qn + 1/4 F(Q1)),
// Qn+1 = round(1/3 Qn + 2/3 F(Q2)), F(q) = round(q + dt L(q)).
// Tolerances: eps for every rounding, or Section 4.4's rule (TT_EPS_PAPER), set at the start
// of each step: eq. eps-tt-formula for the roundings inside L, the reciprocal and the
// crosses (eps_in), eq. modified-eps-tt-formula per variable for its time-stepping roundings
// (eps_q).
//
// Boundaries per axis: periodic, walls, or exact (Section 5's exact-solution boundaries): on an
// exact axis the state's cores are extended by zeros and each separable ghost term
// amp cos(omega t + phase) X Y becomes further rank columns of the reconstructed TTs (its
// factor along the exact axis an explicit column of n + 6 rows, zero inside the domain, its
// other factor extended by the other axis's rule), since the reconstruction is linear.
// Separable forcing terms add rank-1 TTs to L.  Terms are evaluated at the SSP-RK3 stage
// times t, t + dt, t + dt/2.
//
// Every TT of the step lives in the solver's arena.  By default ranks are known on the host after
// each rounding (one stream synchronisation per rounding), so every launch has its exact shape.
// In graph mode (tt_fv_params.graph) every decision is taken on the device (fixed.hip), every TT
// keeps the static rank of its buffer with zero columns after the device's rank, and the step is
// captured in a HIP graph after one eager step and replayed.
#include "common.h"
#include "pool.h"

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <thread>

namespace ttfv {

namespace {
const double SIGN_NORMAL[3] = {1.0, -1.0, 1.0};
const double SIGN_TANGENT[3] = {1.0, 1.0, -1.0};
}  // namespace

struct Solver {
  tt_fv_params p{};
  Ctx c;                       // caller's stream; owns the state and phase outputs
  std::unique_ptr<Pool> pool;  // own worker streams for independent chains (may be empty)
  Pool *exec = nullptr;        // pool the phases run on: the own pool or an ensemble's
  StencilSet st;
  WenoTables wt{};
  int n = 0, nq = 0;
  // per axis (0 = x, 1 = y): ghost rule of the state's cores, periodic or not, face count
  Ghost rule_ax[2] = {Ghost::Periodic, Ghost::Periodic};
  bool periodic_ax[2] = {true, true};
  int nf_ax[2] = {0, 0};
  double t = 0.0;              // time at the start of the next step
  // separable terms on the device: ghost terms keep their exact-axis column (n + 6 rows,
  // zero inside the domain) in e and their other factor extended by the other axis's rule
  // (n + 6 rows) in o; forcing terms keep X and Y (n rows each) in e and o
  struct DevTerm {
    int var, where;
    double amp, omega, phase;
    double *e, *o;
  };
  std::vector<DevTerm> terms;
  double *term_mem = nullptr;
  // exact boundaries with WENO5: the 6 tangent ghost rows (0, 1, 2, n+3, n+4, n+5) and the
  // unit columns at those rows, (n + 6) x 6
  int *ghost_rows6 = nullptr;
  double *unit6 = nullptr;
  DTT Q[3];
  std::map<int, std::vector<int>> piv;
  std::mutex mu;               // guards piv and the Taylor statistics
  long long step_index = 0;
  int last_terms = 0;
  double last_err = 0.0;
  int *rep_idx = nullptr;      // row j*nq + m -> j
  // tolerances of the current step: roundings inside L, reciprocal and crosses; and each
  // variable's forward-Euler and SSP-RK3 combination roundings
  double eps_in = 0.0;
  double eps_q[3] = {0.0, 0.0, 0.0};
  // learned pivot proposer (TT_PIV_*): model, per-site validation error of the last plain
  // cross, and counters
  // helper contexts of the Taylor reciprocal's partial sums, one per (direction, side); used
  // when the solver steps on its own pool
  std::unique_ptr<Ctx> aux[4];
  PivotModel *pm = nullptr;
  int piv_mode = TT_PIV_MAXVOL;
  // acceptance of a one-sweep cross from proposed columns (TT_PIV_LEARNED, TT_PIV_KICKS):
  // validation error <= acc_abs, or with acc_rel >= 0 also <= (1 + acc_rel) times the error of
  // the site's last plain cross
  double acc_abs = 1e-6, acc_rel = -1.0;
  std::map<int, double> ref_err;
  // pivot replay (TT_PIV_REPLAY): (step, site) -> (J, I) given by the caller; and the last
  // sweep's (J, I) of every site's latest cross, for the caller to read back
  std::map<std::pair<long long, int>, std::pair<std::vector<int>, std::vector<int>>> replay;
  std::map<int, std::pair<std::vector<int>, std::vector<int>>> last_piv;
  long long sweeps_run = 0, learned = 0, fallbacks = 0;
  double max_learned_err = 0.0;
  // graph mode (tt_fv_params.graph): fixed shapes on the solver's stream, the step captured in a
  // HIP graph after one eager step and replayed.  Device state: the step counter the crosses'
  // kicks are keyed by, and per cross site its column set (site_cap entries, then the count).
  long long *dev_step = nullptr;
  int *site_J = nullptr;
  int site_cap = 0;
  static constexpr int kSites = 6 << 6;
  std::vector<char> site_have;
  bool warm = false;              // eager fixed-shape steps have set the static ranks (and,
                                  // with the GEMM autotuner on, tuned the static shapes)
  int eager_steps = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  double graph_dt = 0.0;
  size_t graph_mark = 0;
  Counters graph_cnt;             // host counters of one captured step
  long long graph_sweeps = 0;
  long long graph_launches = 0;
  hipStream_t own_stream = nullptr;   // graph mode: the solver's stream (capturable)
  hipStream_t user_stream = nullptr;  // the stream given at init
  hipEvent_t user_ev = nullptr;

  // graph mode: the solver's own (non-blocking) stream does not wait for the caller's, which
  // may be the null stream; calls that read or write caller memory first order it after the
  // caller's stream
  void after_user() {
    if (!own_stream) return;
    HIP_CHECK(hipEventRecord(user_ev, user_stream));
    HIP_CHECK(hipStreamWaitEvent(own_stream, user_ev, 0));
  }
  // graph mode: branch contexts (own stream and arena each) the independent tasks of a phase
  // fork onto from the solver's stream and join back, by events, so that a captured step
  // keeps the phases' concurrency as parallel branches of its graph
  std::vector<std::unique_ptr<Ctx>> branch;
  hipEvent_t fork_ev = nullptr;
  std::vector<hipEvent_t> join_ev;

  ~Solver() {
    if (gexec || graph) (void)hipStreamSynchronize(c.stream);
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    for (auto &b : branch) {
      hipStream_t st = b->stream;
      (void)hipStreamSynchronize(st);
      b.reset();
      (void)hipStreamDestroy(st);
    }
    if (fork_ev) (void)hipEventDestroy(fork_ev);
    if (user_ev) (void)hipEventDestroy(user_ev);
    for (hipEvent_t e : join_ev) (void)hipEventDestroy(e);
    if (own_stream) {
      (void)hipStreamSynchronize(own_stream);
      c.stream = user_stream;   // the context's own clean-up must not see the destroyed stream
      (void)hipStreamDestroy(own_stream);
    }
    if (term_mem) {
      (void)hipStreamSynchronize(c.stream);
      (void)hipFree(term_mem);
    }
    for (auto &a : aux) {
      if (!a) continue;
      hipStream_t st = a->stream;
      (void)hipStreamSynchronize(st);
      a.reset();
      (void)hipStreamDestroy(st);
    }
  }

  static DTT alloc(Ctx &w, int n1, int n2, int cap) {
    DTT t;
    t.n1 = n1;
    t.n2 = n2;
    t.r = 0;
    t.A = w.arena.dalloc((size_t)n1 * std::max(cap, 1));
    t.B = w.arena.dalloc((size_t)n2 * std::max(cap, 1));
    return t;
  }

  // every task sets its worker's arithmetic to this solver's (an ensemble shares workers)
  void run_tasks(std::vector<Pool::Task> tasks) {
    const bool f32 = p.precision == TT_PREC_F32;
    const int qr = p.qr;
    const double drop = p.cross_drop;
    const int enrich = p.cross_enrich;
    for (auto &t : tasks)
      t = [f32, qr, drop, enrich, f = std::move(t)](Ctx &w) {
        w.fp32 = f32;
        w.qr = qr;
        w.cross_drop = drop;
        w.enrich = enrich;
        f(w);
      };
    if (p.graph) {
      const int K = std::min((int)branch.size(), (int)tasks.size());
      if (K <= 1) {               // one stream: the tasks in order, temporaries per task
        for (auto &t : tasks) {
          Scope sc(c.arena);
          t(c);
        }
        return;
      }
      // fork: the branches wait for the solver's stream; task i runs on branch i mod K, in
      // that branch's arena; join: the solver's stream waits for every branch used
      HIP_CHECK(hipEventRecord(fork_ev, c.stream));
      for (int b = 0; b < K; ++b) HIP_CHECK(hipStreamWaitEvent(branch[b]->stream, fork_ev, 0));
      for (size_t i = 0; i < tasks.size(); ++i) {
        Ctx &w = *branch[i % K];
        Scope sc(w.arena);
        tasks[i](w);
      }
      for (int b = 0; b < K; ++b) {
        HIP_CHECK(hipEventRecord(join_ev[b], branch[b]->stream));
        HIP_CHECK(hipStreamWaitEvent(c.stream, join_ev[b], 0));
      }
      return;
    }
    exec->run(std::move(tasks));
  }

  DTT rnd(Ctx &w, const DTT &x) {
    DTT y = alloc(w, x.n1, x.n2, p.r_max);
    round_tt(w, x, eps_in, p.r_max, y, nullptr);
    return y;
  }

  static DTT transposed(const DTT &x) {
    DTT t;
    t.n1 = x.n2;
    t.n2 = x.n1;
    t.r = x.r;
    t.A = x.B;
    t.B = x.A;
    return t;
  }

  // sum of coefficient * TT; terms whose second cores are the same buffer add their first cores
  static DTT add(Ctx &w, const std::vector<std::pair<double, DTT>> &terms) {
    struct G {
      std::vector<std::pair<double, const DTT *>> parts;
      const double *B;
      int r;
    };
    std::vector<G> groups;
    for (auto &t : terms) {
      bool found = false;
      for (auto &g : groups)
        if (g.B == t.second.B && g.r == t.second.r) {
          g.parts.push_back({t.first, &t.second});
          found = true;
          break;
        }
      if (!found) groups.push_back({{{t.first, &t.second}}, t.second.B, t.second.r});
    }
    int R = 0;
    for (auto &g : groups) R += g.r;
    const int n1 = terms[0].second.n1, n2 = terms[0].second.n2;
    DTT out = alloc(w, n1, n2, R);
    out.r = R;
    int off = 0;
    for (auto &g : groups) {
      double *dA = out.A + (size_t)n1 * off;
      copy_scale(w, dA, n1, g.parts[0].second->A, n1, n1, g.r, g.parts[0].first);
      for (size_t k = 1; k < g.parts.size(); ++k)
        axpby(w, dA, n1, dA, n1, 1.0, g.parts[k].second->A, n1, g.parts[k].first, n1, g.r);
      copy_scale(w, out.B + (size_t)n2 * off, n2, g.B, n2, n2, g.r, 1.0);
      off += g.r;
    }
    return out;
  }

  static DTT had(Ctx &w, const DTT &x, const DTT &y) {
    const int R = x.r * y.r;
    DTT out = alloc(w, x.n1, x.n2, R);
    out.r = R;
    khatri_rao(w, out.A, x.n1, x.A, x.r, y.A, y.r);
    khatri_rao(w, out.B, x.n2, x.B, x.r, y.B, y.r);
    return out;
  }

  static double norm2(Ctx &w, const DTT &x) {
    Scope sc(w.arena);
    double *ga = w.arena.dalloc((size_t)x.r * x.r), *gb = w.arena.dalloc((size_t)x.r * x.r);
    gemm(w, true, x.r, x.r, x.n1, 1.0, x.A, x.n1, x.A, x.n1, 0.0, ga, x.r);
    gemm(w, true, x.r, x.r, x.n2, 1.0, x.B, x.n2, x.B, x.n2, 0.0, gb, x.r);
    std::vector<double> ha((size_t)x.r * x.r), hb((size_t)x.r * x.r);
    HIP_CHECK(hipMemcpyAsync(ha.data(), ga, ha.size() * 8, hipMemcpyDeviceToHost, w.stream));
    HIP_CHECK(hipMemcpyAsync(hb.data(), gb, hb.size() * 8, hipMemcpyDeviceToHost, w.stream));
    w.sync();
    double s = 0.0;
    for (size_t i = 0; i < ha.size(); ++i) s += ha[i] * hb[i];
    return std::max(s, 0.0);
  }

  static std::vector<int> initial_columns(Ctx &w, const DTT &y0) {
    Scope sc(w.arena);
    const int m = std::min(y0.r, y0.n2);
    double *Qb = w.arena.dalloc((size_t)y0.n2 * std::max(m, 1));
    int k = 0;
    orth(w, y0.B, y0.n2, y0.r, y0.n2, w.drop(), Qb, &k);
    if (k == 0) return {0};
    return maxvol_host(w, Qb, y0.n2, k, y0.n2, 1.05, 100);
  }

  // relative error |f - Y|_F / |Y|_F of a cross result Y on 16 seeded columns outside J
  double validate(Ctx &w, const FiberSpec &fs, int n1, int n2, const DTT &y,
                  const std::vector<int> &J, uint64_t key) {
    Scope sc(w.arena);
    const std::vector<int> Jv = kick_indices(J, n2, 16, key ^ 0x76A11DA7E5ull);
    const int nv = (int)Jv.size();
    if (nv == 0) return 0.0;
    int *Jd = w.arena.ialloc(nv);
    HIP_CHECK(hipMemcpyAsync(Jd, Jv.data(), nv * sizeof(int), hipMemcpyHostToDevice, w.stream));
    double *Fv = w.arena.dalloc((size_t)n1 * nv), *Yv = w.arena.dalloc((size_t)n1 * nv);
    double *G = w.arena.dalloc((size_t)nv * std::max(y.r, 1));
    fiber_cols(w, fs, n1, Jd, nv, Fv);
    gather_rows(w, G, nv, y.B, y.n2, Jd, nv, y.r);
    gemm2(w, false, true, n1, nv, y.r, 1.0, y.A, y.n1, G, nv, 0.0, Yv, n1);
    std::vector<double> f((size_t)n1 * nv), yy((size_t)n1 * nv);
    HIP_CHECK(hipMemcpyAsync(f.data(), Fv, f.size() * 8, hipMemcpyDeviceToHost, w.stream));
    HIP_CHECK(hipMemcpyAsync(yy.data(), Yv, yy.size() * 8, hipMemcpyDeviceToHost, w.stream));
    w.sync();
    double d2 = 0.0, y2 = 0.0;
    for (size_t i = 0; i < f.size(); ++i) {
      d2 += (f[i] - yy[i]) * (f[i] - yy[i]);
      y2 += yy[i] * yy[i];
    }
    return y2 > 0.0 ? std::sqrt(d2 / y2) : std::sqrt(d2);
  }

  // cross into the preallocated `out` (capacity r_max).  Pivots: the same site's columns of
  // the previous step (or maxvol of the starting TT), refined by the maxvol sweeps; with the
  // learned proposer, its top-K columns and one sweep when the validation check passes.
  bool site_ready(int site) const {
    return p.graph && site >= 0 && site < kSites && site_have[site];
  }

  // graph mode: the cross from the site's device column set (set by maxvol of the starting
  // TT on the site's first, eager, call)
  void cross_graph(Ctx &w, const FiberSpec &fs, int n1, int n2, const DTT &y0, int site,
                   DTT &out) {
    TT_REQUIRE(site >= 0 && site < kSites, "graph mode: cross site out of range");
    int *Jd = site_J + (size_t)site * (site_cap + 1), *nJ = Jd + site_cap;
    if (!site_have[site]) {
      TT_REQUIRE(!w.capturing, "graph mode: a cross site without pivots during capture");
      std::vector<int> J0 = initial_columns(w, y0);
      TT_REQUIRE((int)J0.size() <= site_cap, "graph mode: starting columns exceed r_max");
      std::vector<int> h(site_cap + 1, 0);
      std::copy(J0.begin(), J0.end(), h.begin());
      h[site_cap] = (int)J0.size();
      HIP_CHECK(hipMemcpyAsync(Jd, h.data(), h.size() * sizeof(int), hipMemcpyHostToDevice,
                               w.stream));
      w.sync();
      site_have[site] = 1;
    }
    const uint64_t key = (uint64_t)site;
    cross_fixed(w, fs, n1, n2, Jd, nJ, site_cap, eps_in, p.r_max, p.cross_sweeps, p.cross_kick,
                key, dev_step, out);
    sweeps_run += p.cross_sweeps;
  }

  void cross(Ctx &w, const FiberSpec &fs, int n1, int n2, const DTT &y0, int site, DTT &out) {
    if (p.graph) {
      cross_graph(w, fs, n1, n2, y0, site, out);
      return;
    }
    std::vector<int> J0;
    double ref = -1.0;
    if (piv_mode == TT_PIV_REPLAY) {
      std::pair<std::vector<int>, std::vector<int>> ji;
      {
        std::lock_guard<std::mutex> lk(mu);
        auto it = replay.find({step_index, site});
        if (it == replay.end())
          throw Error(TT_EINVAL, "replay: no pivots for step " + std::to_string(step_index) +
                                     ", site " + std::to_string(site));
        ji = it->second;
      }
      skeleton_tt(w, fs, n1, n2, ji.first, ji.second, eps_in, p.r_max, out);
      std::lock_guard<std::mutex> lk(mu);
      piv[site] = ji.first;
      last_piv[site] = ji;
      return;
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      auto it = piv.find(site);
      if (it != piv.end()) J0 = it->second;
      auto ie = ref_err.find(site);
      if (ie != ref_err.end()) ref = ie->second;
    }
    const bool have_prev = !J0.empty();
    if (J0.empty()) J0 = initial_columns(w, y0);
    const uint64_t key = ((uint64_t)site << 32) | (uint64_t)(step_index & 0xFFFFFFFFll);
    std::vector<int> J;
    Scope sc(w.arena);
    bf16_t *Xb = nullptr;
    if (pm && (piv_mode == TT_PIV_LOG || piv_mode == TT_PIV_LEARNED) && have_prev &&
        (int)J0.size() <= 128) {
      int *Jd = w.arena.ialloc(J0.size());
      HIP_CHECK(hipMemcpyAsync(Jd, J0.data(), J0.size() * sizeof(int), hipMemcpyHostToDevice,
                               w.stream));
      Xb = static_cast<bf16_t *>(w.arena.alloc((size_t)n2 * PM_F * sizeof(bf16_t)));
      pivot_features(w, y0.B, n2, y0.r, y0.n2, Jd, (int)J0.size(), nullptr, Xb);
    }
    const bool propose = (piv_mode == TT_PIV_LEARNED && Xb) ||
                         (piv_mode == TT_PIV_KICKS && have_prev && (int)J0.size() <= 128);
    if (propose && (acc_rel < 0.0 || ref >= 0.0)) {
      // the previous pivots, then up to K = min(r_max, |J_prev| + kick) columns they miss,
      // within the factorization width: the proposer's best scores, or (ablation) fresh
      // SplitMix64 columns
      const int K = std::min(std::min(p.r_max, (int)J0.size() + p.cross_kick), n2);
      std::vector<int> top;
      if (piv_mode == TT_PIV_LEARNED) {
        Scope s2(w.arena);
        float *sc_dev = static_cast<float *>(w.arena.alloc((size_t)n2 * sizeof(float)));
        pm->forward(w, Xb, n2, sc_dev, nullptr, nullptr);
        int *Kd = w.arena.ialloc(K);
        topk_indices(w, sc_dev, n2, K, Kd);
        top.resize(K);
        HIP_CHECK(hipMemcpyAsync(top.data(), Kd, K * sizeof(int), hipMemcpyDeviceToHost,
                                 w.stream));
        w.sync();
      } else {
        top = kick_indices(J0, n2, std::max(0, K - (int)J0.size()), key ^ 0x4B1C5ull);
      }
      std::vector<int> Jp = J0;
      for (int j : top) {
        if ((int)Jp.size() >= qr_max_cols()) break;
        if (std::find(Jp.begin(), Jp.end(), j) == Jp.end()) Jp.push_back(j);
      }
      std::vector<int> Il;
      cross_tt(w, fs, n1, n2, Jp, eps_in, p.r_max, 1, 0, key, out, &J, &Il);
      const double err = validate(w, fs, n1, n2, out, J, key);
      const double bar = acc_rel >= 0.0 ? std::max(acc_abs, (1.0 + acc_rel) * ref) : acc_abs;
      std::lock_guard<std::mutex> lk(mu);
      sweeps_run += 1;
      if (err <= bar) {
        learned++;
        max_learned_err = std::max(max_learned_err, err);
        piv[site] = J;
        last_piv[site] = {J, Il};
        return;
      }
      fallbacks++;
    }
    std::vector<int> I;
    cross_tt(w, fs, n1, n2, J0, eps_in, p.r_max, p.cross_sweeps, p.cross_kick, key, out, &J,
             &I);
    double err = -1.0;
    if (piv_mode != TT_PIV_MAXVOL) err = validate(w, fs, n1, n2, out, J, key);
    if (piv_mode == TT_PIV_LOG && Xb) {
      int *Jd = w.arena.ialloc(J.size());
      HIP_CHECK(hipMemcpyAsync(Jd, J.data(), J.size() * sizeof(int), hipMemcpyHostToDevice,
                               w.stream));
      pm->append(w, Xb, Jd, (int)J.size(), n2);
    }
    std::lock_guard<std::mutex> lk(mu);
    sweeps_run += p.cross_sweeps;
    if (err >= 0.0) ref_err[site] = err;
    piv[site] = J;
    last_piv[site] = {J, I};
  }

  static double time_factor(const DevTerm &tm, double tt) {
    return tm.amp * std::cos(tm.omega * tt + tm.phase);
  }

  // ---- reconstruction -------------------------------------------------------------
  // direction d (the first core of Qv runs along axis d); ghost terms of exact axes become
  // extra columns after the state's r
  void states_upwind(Ctx &w, const DTT *Qv, int d, double tt, DTT *qm, DTT *qp) {
    const int nf = nf_ax[d];
    for (int v = 0; v < 3; ++v) {
      const int nat = d == 0 ? v : (v == 0 ? 0 : 3 - v);   // natural variable index
      std::vector<const DevTerm *> gh;
      for (const DevTerm &tm : terms)
        if (tm.var == nat && tm.where != TT_TERM_FORCING) gh.push_back(&tm);
      const DTT &q = Qv[v];
      const int J = (int)gh.size(), R = q.r + J;
      DTT m = alloc(w, nf, n * nq, R);
      DTT pl = m;
      pl.A = w.arena.dalloc((size_t)nf * R);
      m.r = pl.r = R;
      recon_face(w, q.A, n, q.r, rule_ax[d], SIGN_NORMAL[v], st, m.A, pl.A, nf);
      recon_quad(w, q.B, n, q.r, rule_ax[1 - d], SIGN_TANGENT[v], st, m.B);  // shared core
      if (J) {
        double *Nx = w.arena.dalloc((size_t)(n + 6) * J), *Tx = w.arena.dalloc((size_t)(n + 6) * J);
        for (int j = 0; j < J; ++j) {
          const DevTerm &tm = *gh[j];
          const int ax = (tm.where == TT_TERM_X_LO || tm.where == TT_TERM_X_HI) ? 0 : 1;
          const double *nc = ax == d ? tm.e : tm.o, *tc = ax == d ? tm.o : tm.e;
          copy_scale(w, Nx + (size_t)j * (n + 6), n + 6, nc, n + 6, n + 6, 1,
                     time_factor(tm, tt));
          copy_scale(w, Tx + (size_t)j * (n + 6), n + 6, tc, n + 6, n + 6, 1, 1.0);
        }
        recon_face(w, Nx, n, J, Ghost::Explicit, 1.0, st, m.A + (size_t)q.r * nf,
                   pl.A + (size_t)q.r * nf, nf);
        recon_quad(w, Tx, n, J, Ghost::Explicit, 1.0, st, m.B + (size_t)q.r * n * nq);
      }
      qm[v] = m;
      qp[v] = pl;
    }
  }

  // Algorithms 2 and 3 for one variable and one side, into `out` (n_f x n*nq, cap r_max)
  // Exact boundaries: on the normal axis the ghost terms are further columns of Algorithm 2's
  // input; on the tangent axis Algorithm 3 needs the Step-1 values at the 6 tangent ghost
  // cells, where the field is the ghost terms alone: they are evaluated directly (the same
  // fiber function at those 6 rows of an extended tangent core) and appended to the Step-1
  // TT as 6 columns whose tangent factors are unit vectors at those rows.
  void weno_state(Ctx &w, const DTT &q, int v, int side, int site_base, int d, double tt,
                  DTT &out) {
    const int nf = nf_ax[d];
    const double eps_w = (1.0 / n) * (1.0 / n);
    const int site = site_base + 16 + v * 4 + side;
    const int nat = d == 0 ? v : (v == 0 ? 0 : 3 - v);
    std::vector<const DevTerm *> gh;
    for (const DevTerm &tm : terms)
      if (tm.var == nat && tm.where != TT_TERM_FORCING) gh.push_back(&tm);
    const int J = (int)gh.size();
    const bool normal_exact = rule_ax[d] == Ghost::Zero, tangent_exact = rule_ax[1 - d] ==
                                                                          Ghost::Zero;
    const int R = q.r + (normal_exact ? J : 0);
    double *Ae = w.arena.dalloc((size_t)(n + 6) * R);
    ghost_extend(w, q.A, n, q.r, rule_ax[d], SIGN_NORMAL[v], Ae);
    const double *B1 = q.B;
    if (normal_exact && J) {
      double *Bf = w.arena.dalloc((size_t)n * R);
      copy_scale(w, Bf, n, q.B, n, n, q.r, 1.0);
      for (int j = 0; j < J; ++j) {
        copy_scale(w, Ae + (size_t)(q.r + j) * (n + 6), n + 6, gh[j]->e, n + 6, n + 6, 1,
                   time_factor(*gh[j], tt));
        copy_scale(w, Bf + (size_t)(q.r + j) * n, n, gh[j]->o + 3, n, n, 1, 1.0);
      }
      B1 = Bf;
    }
    FiberSpec f1;
    f1.fn = side == 0 ? TT_FN_WENO_FACE_M : TT_FN_WENO_FACE_P;
    f1.n_in = 1;
    f1.in[0] = {Ae, B1, n + 6, n, R};
    f1.eps_w = eps_w;
    f1.wt = &wt;
    DTT vt = alloc(w, nf, n, p.r_max);
    cross(w, f1, nf, n, q, site, vt);
    DTT y0 = alloc(w, nf, n * nq, vt.r);
    y0.r = vt.r;
    copy_scale(w, y0.A, nf, vt.A, nf, nf, vt.r, 1.0);
    gather_rows(w, y0.B, n * nq, vt.B, n, rep_idx, n * nq, vt.r);
    const double *A2 = vt.A;
    int r2 = vt.r;
    double *Be;
    if (tangent_exact) {
      r2 = vt.r + 6;
      double *Ax = w.arena.dalloc((size_t)nf * r2);
      Be = w.arena.dalloc((size_t)(n + 6) * r2);
      copy_scale(w, Ax, nf, vt.A, nf, nf, vt.r, 1.0);
      fill_value(w, Be, n + 6, n + 6, vt.r, 0.0);
      copy_scale(w, Be + 3, n + 6, vt.B, n, n, vt.r, 1.0);
      copy_scale(w, Be + (size_t)vt.r * (n + 6), n + 6, unit6, n + 6, n + 6, 6, 1.0);
      double *V = Ax + (size_t)vt.r * nf;
      if (J) {
        // the ghost field: normal factors (extended by the normal rule) times tangent columns
        // (explicit, zero inside the domain), evaluated at the 6 tangent ghost rows
        double *Gn = w.arena.dalloc((size_t)(n + 6) * J), *Gt = w.arena.dalloc((size_t)(n + 6) * J);
        for (int j = 0; j < J; ++j) {
          copy_scale(w, Gn + (size_t)j * (n + 6), n + 6, gh[j]->o, n + 6, n + 6, 1,
                     time_factor(*gh[j], tt));
          copy_scale(w, Gt + (size_t)j * (n + 6), n + 6, gh[j]->e, n + 6, n + 6, 1, 1.0);
        }
        FiberSpec fg = f1;
        fg.in[0] = {Gn, Gt, n + 6, n + 6, J};
        fiber_cols(w, fg, nf, ghost_rows6, 6, V);
      } else {
        fill_value(w, V, nf, nf, 6, 0.0);
      }
      A2 = Ax;
    } else {
      Be = w.arena.dalloc((size_t)(n + 6) * vt.r);
      ghost_extend(w, vt.B, n, vt.r, rule_ax[1 - d], SIGN_TANGENT[v], Be);
    }
    FiberSpec f2;
    f2.fn = TT_FN_WENO_QUAD;
    f2.n_in = 1;
    f2.in[0] = {A2, Be, nf, n + 6, r2};
    f2.eps_w = eps_w;
    f2.nq = nq;
    f2.wt = &wt;
    cross(w, f2, nf, n * nq, y0, site + 2, out);
  }

  // ---- nonlinear flux pieces ----------------------------------------------------------
  // one side: 1/h (Algorithm 1), u, w, P1, P2 -> F2 = round(P1 + g/2 P2), F3 = round(m o w)
  // 1/h of one side: cross of the pointwise reciprocal or Algorithm 1, into rh (cap r_max)
  void reciprocal(Ctx &w, const DTT &h, int recip_site, int chain, DTT &rh) {
    if (p.graph && p.recip == 0) {
      reciprocal_fixed(w, h, eps_in, p.taylor_terms, p.r_max, rh);
      last_terms = p.taylor_terms;   // every term is formed; Err stays on the device
      return;
    }
    if (p.recip == 1) {
      FiberSpec fr;
      fr.fn = TT_FN_RECIP;
      fr.n_in = 1;
      fr.in[0] = {h.A, h.B, h.n1, h.n2, h.r};
      cross(w, fr, h.n1, h.n2, h, recip_site, rh);
    } else {
      double err = 0;
      int terms = 0;
      Ctx *a = (exec == pool.get() && aux[chain]) ? aux[chain].get() : nullptr;
      if (a) {
        a->fp32 = w.fp32;
        a->qr = w.qr;
      }
      reciprocal_tt(w, h, eps_in, p.taylor_terms, p.r_max, rh, &err, &terms, a);
      std::lock_guard<std::mutex> lk(mu);
      last_err = err;
      last_terms = terms;
    }
  }

  DTT finish(Ctx &w, const DTT &Fh, int d, DTT &o) {
    o.r = Fh.r;
    face_diff(w, Fh.A, nf_ax[d], n, Fh.r, periodic_ax[d], 1.0, o.A, n);
    quad_sum(w, Fh.B, n, nq, Fh.r, st, o.B);
    return o;
  }

  // dF[d][v] (n x n, cap r_max): flux differences of both directions, d = 0 x, d = 1 y
  // (the y result is in transposed orientation)
  void fluxes(const DTT (*QD)[3], int stage, double tt, DTT (*dF)[3]) {
    const int sb[2] = {(0 * 3 + stage) << 6, (1 * 3 + stage) << 6};
    DTT qm[2][3], qp[2][3];
    if (p.scheme != 55) {
      for (int d = 0; d < 2; ++d) states_upwind(c, QD[d], d, tt, qm[d], qp[d]);
      c.sync();
    } else {
      for (int d = 0; d < 2; ++d)
        for (int v = 0; v < 3; ++v) {
          qm[d][v] = alloc(c, nf_ax[d], n * nq, p.r_max);
          qp[d][v] = alloc(c, nf_ax[d], n * nq, p.r_max);
        }
      c.sync();
      std::vector<Pool::Task> tasks;
      for (int d = 0; d < 2; ++d)
        for (int v = 0; v < 3; ++v)
          for (int side = 0; side < 2; ++side)
            tasks.push_back([this, &QD, &qm, &qp, &sb, d, v, side, tt](Ctx &w) {
              weno_state(w, QD[d][v], v, side, sb[d], d, tt, side == 0 ? qm[d][v] : qp[d][v]);
            });
      run_tasks(std::move(tasks));
    }
    if (!p.nonlinear) {
      const double g = p.g, H = p.H0, cw = std::sqrt(g * H);
      for (int d = 0; d < 2; ++d) {
        DTT Fh[3];
        Fh[0] = add(c, {{0.5 * H, qm[d][1]}, {0.5 * H, qp[d][1]}, {-0.5 * cw, qp[d][0]},
                        {0.5 * cw, qm[d][0]}});
        Fh[1] = add(c, {{0.5 * g, qm[d][0]}, {0.5 * g, qp[d][0]}, {-0.5 * cw, qp[d][1]},
                        {0.5 * cw, qm[d][1]}});
        Fh[2] = add(c, {{-0.5 * cw, qp[d][2]}, {0.5 * cw, qm[d][2]}});
        for (int v = 0; v < 3; ++v) {
          dF[d][v] = alloc(c, n, n, Fh[v].r);
          finish(c, Fh[v], d, dF[d][v]);
        }
      }
      return;
    }
    if (p.flux == TT_FLUX_LF_CROSS) {
      // LF-cross: the whole LLF flux vector of direction d by one cross over the face index
      // and (component, quadrature column), then split by component
      for (int d = 0; d < 2; ++d)
        for (int v = 0; v < 3; ++v) dF[d][v] = alloc(c, n, n, p.r_max);
      DTT Fv[2];
      for (int d = 0; d < 2; ++d) Fv[d] = alloc(c, nf_ax[d], 3 * n * nq, p.r_max);
      c.sync();
      std::vector<Pool::Task> tasks;
      for (int d = 0; d < 2; ++d)
        tasks.push_back([this, &qm, &qp, &Fv, &dF, &sb, d](Ctx &w) {
          const int nf = nf_ax[d], n2 = n * nq;
          // starting columns: the normal momentum's (else h's) second core for each component
          const DTT &ys = norm2(w, qm[d][1]) > 0.0 ? qm[d][1] : qm[d][0];
          DTT y0{nf, 3 * n2, ys.r, ys.A, w.arena.dalloc((size_t)3 * n2 * ys.r)};
          for (int k = 0; k < 3; ++k)
            copy_scale(w, y0.B + (size_t)k * n2, 3 * n2, ys.B, n2, n2, ys.r, 1.0);
          FiberSpec fs;
          fs.fn = TT_FN_LLF_FLUX;
          fs.n_in = 6;
          const DTT *in[6] = {&qm[d][0], &qm[d][1], &qm[d][2], &qp[d][0], &qp[d][1], &qp[d][2]};
          for (int k = 0; k < 6; ++k) fs.in[k] = {in[k]->A, in[k]->B, in[k]->n1, in[k]->n2, in[k]->r};
          fs.g = p.g;
          fs.ncol = n2;
          cross(w, fs, nf, 3 * n2, y0, sb[d] + 4, Fv[d]);
          for (int v = 0; v < 3; ++v) {
            DTT Fh{nf, n2, Fv[d].r, Fv[d].A, w.arena.dalloc((size_t)n2 * std::max(Fv[d].r, 1))};
            copy_scale(w, Fh.B, n2, Fv[d].B + (size_t)v * n2, 3 * n2, n2, Fv[d].r, 1.0);
            finish(w, Fh, d, dF[d][v]);
          }
        });
      run_tasks(std::move(tasks));
      return;
    }
    // phase A, per direction d and side s (h, m = momentum along d, t = the other one):
    //   A1: rh = 1/h, P2 = round(h o h), and the two lambda crosses
    //   A2: u = round(m o rh), w = round(t o rh)
    //   A3: F2 = round(round(m o u) + g/2 P2), F3 = round(m o w)
    // Each value is the same rounding of the same operands as in one sequential chain; the
    // split only lets independent roundings run on different workers.
    DTT F[2][2][3], rh[2][2], P2[2][2], U[2][2], Wv[2][2];
    for (int d = 0; d < 2; ++d)
      for (int s = 0; s < 2; ++s) {
        F[d][s][0] = s == 0 ? qm[d][1] : qp[d][1];
        F[d][s][1] = alloc(c, nf_ax[d], n * nq, p.r_max);
        F[d][s][2] = alloc(c, nf_ax[d], n * nq, p.r_max);
        rh[d][s] = alloc(c, nf_ax[d], n * nq, p.r_max);
        P2[d][s] = alloc(c, nf_ax[d], n * nq, p.r_max);
        U[d][s] = alloc(c, nf_ax[d], n * nq, p.r_max);
        Wv[d][s] = alloc(c, nf_ax[d], n * nq, p.r_max);
      }
    DTT lam[2];
    for (int d = 0; d < 2; ++d) lam[d] = alloc(c, nf_ax[d], n * nq, p.r_max);
    c.sync();
    auto side = [&](int d, int s) { return s == 0 ? qm[d] : qp[d]; };
    {
      std::vector<Pool::Task> tasks;
      for (int d = 0; d < 2; ++d)
        for (int s = 0; s < 2; ++s)
          tasks.push_back([this, &side, &rh, &sb, d, s](Ctx &w) {
            reciprocal(w, side(d, s)[0], sb[d] + 8 + s, d * 2 + s, rh[d][s]);
          });
      for (int d = 0; d < 2; ++d)
        tasks.push_back([this, &qm, &qp, &lam, &sb, d](Ctx &w) {
          // (the starting TT matters only for a site's first cross)
          const DTT &y0 = site_ready(sb[d]) || norm2(w, qm[d][1]) > 0.0 ? qm[d][1] : qm[d][0];
          FiberSpec fl;
          fl.fn = TT_FN_LLF_LAMBDA;
          fl.n_in = 4;
          const DTT *in[4] = {&qm[d][0], &qm[d][1], &qp[d][0], &qp[d][1]};
          for (int k = 0; k < 4; ++k) fl.in[k] = {in[k]->A, in[k]->B, in[k]->n1, in[k]->n2, in[k]->r};
          fl.g = p.g;
          cross(w, fl, nf_ax[d], n * nq, y0, sb[d], lam[d]);
        });
      for (int d = 0; d < 2; ++d)
        for (int s = 0; s < 2; ++s)
          tasks.push_back([this, &side, &P2, d, s](Ctx &w) {
            const DTT &h = side(d, s)[0];
            round_tt(w, had(w, h, h), eps_in, p.r_max, P2[d][s], nullptr);
          });
      run_tasks(std::move(tasks));
    }
    {
      std::vector<Pool::Task> tasks;
      for (int d = 0; d < 2; ++d)
        for (int s = 0; s < 2; ++s) {
          tasks.push_back([this, &side, &rh, &U, d, s](Ctx &w) {
            round_tt(w, had(w, side(d, s)[1], rh[d][s]), eps_in, p.r_max, U[d][s], nullptr);
          });
          tasks.push_back([this, &side, &rh, &Wv, d, s](Ctx &w) {
            round_tt(w, had(w, side(d, s)[2], rh[d][s]), eps_in, p.r_max, Wv[d][s], nullptr);
          });
        }
      run_tasks(std::move(tasks));
    }
    {
      std::vector<Pool::Task> tasks;
      for (int d = 0; d < 2; ++d)
        for (int s = 0; s < 2; ++s) {
          tasks.push_back([this, &side, &U, &P2, &F, d, s](Ctx &w) {
            DTT P1 = rnd(w, had(w, side(d, s)[1], U[d][s]));
            round_tt(w, add(w, {{1.0, P1}, {0.5 * p.g, P2[d][s]}}), eps_in, p.r_max, F[d][s][1],
                     nullptr);
          });
          tasks.push_back([this, &side, &Wv, &F, d, s](Ctx &w) {
            round_tt(w, had(w, side(d, s)[1], Wv[d][s]), eps_in, p.r_max, F[d][s][2], nullptr);
          });
        }
      run_tasks(std::move(tasks));
    }
    // phase B: dissipation, LLF flux and finish, per direction and variable
    for (int d = 0; d < 2; ++d)
      for (int v = 0; v < 3; ++v) dF[d][v] = alloc(c, n, n, p.r_max);
    {
      std::vector<Pool::Task> tasks;
      for (int d = 0; d < 2; ++d)
        for (int v = 0; v < 3; ++v)
          tasks.push_back([this, &qm, &qp, &F, &lam, &dF, d, v](Ctx &w) {
            DTT dq = add(w, {{1.0, qp[d][v]}, {-1.0, qm[d][v]}});
            DTT D = rnd(w, had(w, lam[d], dq));
            DTT Fh = rnd(w, add(w, {{0.5, F[d][0][v]}, {0.5, F[d][1][v]}, {-0.5, D}}));
            finish(w, Fh, d, dF[d][v]);
          });
      run_tasks(std::move(tasks));
    }
  }

  // out[v] = round(Q[v] + dt L(Q)[v]); out buffers allocated by the caller (cap r_max)
  void euler(const DTT *Qv, double dt, int stage, double tt, DTT *out) {
    Scope sc(c.arena);
    DTT QD[2][3] = {{Qv[0], Qv[1], Qv[2]},
                    {transposed(Qv[0]), transposed(Qv[2]), transposed(Qv[1])}};
    DTT dF[2][3];
    fluxes(QD, stage, tt, dF);
    DTT G[3] = {transposed(dF[1][0]), transposed(dF[1][2]), transposed(dF[1][1])};
    const double dx = 1.0 / n;
    std::vector<Pool::Task> tasks;
    for (int v = 0; v < 3; ++v)
      tasks.push_back([this, Qv, &dF, &G, dt, dx, tt, out, v](Ctx &w) {
        std::vector<std::pair<double, DTT>> sum{{1.0, Qv[v]}, {-dt / dx, dF[0][v]},
                                                {-dt / dx, G[v]}};
        if (p.f != 0.0 && v == 1) sum.push_back({dt * p.f, Qv[2]});
        if (p.f != 0.0 && v == 2) sum.push_back({-dt * p.f, Qv[1]});
        for (const DevTerm &tm : terms)
          if (tm.var == v && tm.where == TT_TERM_FORCING)
            sum.push_back({dt * time_factor(tm, tt), DTT{n, n, 1, tm.e, tm.o}});
        round_tt(w, add(w, sum), eps_q[v], p.r_max, out[v], nullptr);
      });
    c.sync();
    run_tasks(std::move(tasks));
  }

  void combine(const DTT *A, double a, const DTT *B, double b, DTT *out) {
    std::vector<Pool::Task> tasks;
    for (int v = 0; v < 3; ++v)
      tasks.push_back([this, A, B, a, b, out, v](Ctx &w) {
        round_tt(w, add(w, {{a, A[v]}, {b, B[v]}}), eps_q[v], p.r_max, out[v], nullptr);
      });
    c.sync();
    run_tasks(std::move(tasks));
  }

  // Largest wave speed of direction d over the cells, for the explicit step's CFL condition:
  // |m/h| + sqrt(g h) with m the momentum along d, estimated on the TTs without forming the
  // field by rook pivoting on the pointwise function (fibers of TT_FN_LLF_LAMBDA with both
  // sides equal): from every maxvol column of h's second core, a walk from that column's
  // largest entry alternates the largest entry of the current row and column until the value
  // stops growing (at most 8 alternations); the best walk wins.  A lower bound of the true
  // maximum (a rook-pivot local maximum).  Linear SWE: sqrt(g H).
  double max_speed(int d) {
    if (!p.nonlinear) return std::sqrt(p.g * p.H0);
    Scope sc(c.arena);
    const DTT &h = Q[0], &m = Q[1 + d];
    FiberSpec fs;
    fs.fn = TT_FN_LLF_LAMBDA;
    fs.n_in = 4;
    fs.in[0] = fs.in[2] = {h.A, h.B, n, n, h.r};
    fs.in[1] = fs.in[3] = {m.A, m.B, n, n, m.r};
    fs.g = p.g;
    const std::vector<int> J0 = initial_columns(c, h);
    const int nj = (int)J0.size();
    int *Jd = c.arena.ialloc(nj), *one = c.arena.ialloc(1);
    double *C = c.arena.dalloc((size_t)n * nj), *vec = c.arena.dalloc(n);
    HIP_CHECK(hipMemcpyAsync(Jd, J0.data(), nj * sizeof(int), hipMemcpyHostToDevice, c.stream));
    auto read = [&](const double *dev, size_t len) {
      std::vector<double> h(len);
      HIP_CHECK(hipMemcpyAsync(h.data(), dev, len * sizeof(double), hipMemcpyDeviceToHost,
                               c.stream));
      c.sync();
      return h;
    };
    fiber_cols(c, fs, n, Jd, nj, C);
    const std::vector<double> Ch = read(C, (size_t)n * nj);
    auto argmax = [](const double *v, int len) {
      int a = 0;
      for (int t = 1; t < len; ++t)
        if (v[t] > v[a]) a = t;
      return a;
    };
    auto fetch = [&](bool row, int idx) {
      HIP_CHECK(hipMemcpyAsync(one, &idx, sizeof(int), hipMemcpyHostToDevice, c.stream));
      if (row) fiber_rows(c, fs, n, one, 1, vec);
      else fiber_cols(c, fs, n, one, 1, vec);
      return read(vec, n);
    };
    double best = -HUGE_VAL;
    for (int k = 0; k < nj; ++k) {
      int i = argmax(Ch.data() + (size_t)k * n, n);
      double v = Ch[(size_t)k * n + i];
      for (int alt = 0; alt < 8; ++alt) {
        const std::vector<double> row = fetch(true, i);
        const int jj = argmax(row.data(), n);
        if (row[jj] <= v) break;
        v = row[jj];
        const std::vector<double> col = fetch(false, jj);
        const int ii = argmax(col.data(), n);
        if (col[ii] <= v) break;
        v = col[ii];
        i = ii;
      }
      if (v > best) best = v;
    }
    if (!std::isfinite(best)) throw Error(TT_ENONFINITE, "max_speed: non-finite wave speed");
    return best;
  }

  // Section 4.4's tolerances from the state at the start of the step (TT_EPS_PAPER)
  void set_tolerances() {
    if (p.eps_rule != TT_EPS_PAPER) {
      eps_in = eps_q[0] = eps_q[1] = eps_q[2] = p.eps;
      return;
    }
    const double dx = 1.0 / n;
    const int order = p.scheme == 3 ? 3 : 5;
    const double base = p.c_eps * std::pow(dx, order - 0.5);   // V = 1
    double l2[3], top = 0.0;
    for (int v = 0; v < 3; ++v) {
      l2[v] = dx * norm_tt(c, Q[v]);
      top = std::max(top, l2[v]);
    }
    eps_in = top > 0.0 ? base / top : 1e-3;
    for (int v = 0; v < 3; ++v) eps_q[v] = l2[v] > 0.0 ? std::min(1e-3, base / l2[v]) : 1e-3;
  }

  void step(double dt) {
    if (p.graph) {
      step_graph(dt);
      return;
    }
    step_body(dt);
    ++step_index;
    t += dt;
  }

  // graph mode: one eager fixed-shape step sets the static ranks and every cross site's
  // pivots; the next step (and the first after a change of dt) is captured, and every step
  // launches the captured graph.  The kernels' scalar arguments (dt, tolerances) are part of
  // the graph; the step count the kicks use lives on the device.
  void step_graph(double dt) {
    TT_REQUIRE(c.timer.name.empty(), "graph mode: kernel timing is not available");
    if (!warm) {
      step_body(dt);
      ++step_index;
      t += dt;
      // one eager step sets the static ranks; a second one at those shapes lets the GEMM
      // tile autotuner (when on) time every shape class the captured step will meet
      warm = ++eager_steps >= (gemm_autotune_on() ? 2 : 1);
      return;
    }
    if (!gexec || dt != graph_dt || c.arena.mark() != graph_mark) capture(dt);
    HIP_CHECK(hipGraphLaunch(gexec, c.stream));
    ++graph_launches;
    const Counters &g = graph_cnt;
    c.cnt.roundings += g.roundings;
    c.cnt.crosses += g.crosses;
    c.cnt.flops += g.flops;
    c.cnt.bytes += g.bytes;
    sweeps_run += graph_sweeps;
    ++step_index;
    t += dt;
  }

  // the host counters of the solver's context and its branches, summed
  Counters all_counters() const {
    Counters t = c.cnt;
    for (auto &b : branch) {
      const Counters &w = b->cnt;
      t.roundings += w.roundings;
      t.crosses += w.crosses;
      t.flops += w.flops;
      t.bytes += w.bytes;
      t.warnings |= w.warnings;
    }
    return t;
  }

  void set_capturing(bool on) {
    c.capturing = on;
    for (auto &b : branch) b->capturing = on;
  }

  int fixed_status_all() {
    int w = fixed_status(c);
    for (auto &b : branch) w |= fixed_status(*b);
    return w;
  }

  void capture(double dt) {
    if (gexec) {
      HIP_CHECK(hipStreamSynchronize(c.stream));
      (void)hipGraphExecDestroy(gexec);
      gexec = nullptr;
    }
    if (graph) {
      (void)hipGraphDestroy(graph);
      graph = nullptr;
    }
    std::vector<Counters> saved{c.cnt};
    for (auto &b : branch) saved.push_back(b->cnt);
    const Counters before = all_counters();
    auto restore = [&]() {
      c.cnt = saved[0];
      for (size_t b = 0; b < branch.size(); ++b) branch[b]->cnt = saved[b + 1];
    };
    const long long sw = sweeps_run;
    const size_t mark = c.arena.mark();
    hipGraph_t g = nullptr;
    HIP_CHECK(hipStreamBeginCapture(c.stream, hipStreamCaptureModeRelaxed));
    set_capturing(true);
    try {
      step_body(dt);
    } catch (...) {
      set_capturing(false);
      if (hipStreamEndCapture(c.stream, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
      restore();
      sweeps_run = sw;
      throw;
    }
    set_capturing(false);
    HIP_CHECK(hipStreamEndCapture(c.stream, &g));
    graph = g;
    HIP_CHECK(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
    const Counters after = all_counters();
    graph_cnt = Counters{};
    graph_cnt.roundings = after.roundings - before.roundings;
    graph_cnt.crosses = after.crosses - before.crosses;
    graph_cnt.flops = after.flops - before.flops;
    graph_cnt.bytes = after.bytes - before.bytes;
    graph_sweeps = sweeps_run - sw;
    restore();
    sweeps_run = sw;
    graph_dt = dt;
    graph_mark = mark;
  }

  void step_body(double dt) {
    Scope sc(c.arena);
    set_tolerances();
    DTT Q1[3], F1[3], Q2[3], F2[3], Qn[3];
    for (int v = 0; v < 3; ++v) {
      Q1[v] = alloc(c, n, n, p.r_max);
      F1[v] = alloc(c, n, n, p.r_max);
      Q2[v] = alloc(c, n, n, p.r_max);
      F2[v] = alloc(c, n, n, p.r_max);
      Qn[v] = alloc(c, n, n, p.r_max);
    }
    // stage times of SSP-RK3: t, t + dt, t + dt/2
    euler(Q, dt, 0, t, Q1);
    euler(Q1, dt, 1, t + dt, F1);
    combine(Q, 0.75, F1, 0.25, Q2);
    euler(Q2, dt, 2, t + 0.5 * dt, F2);
    combine(Q, 1.0 / 3.0, F2, 2.0 / 3.0, Qn);
    for (int v = 0; v < 3; ++v) {
      copy_scale(c, Q[v].A, n, Qn[v].A, n, n, Qn[v].r, 1.0);
      copy_scale(c, Q[v].B, n, Qn[v].B, n, n, Qn[v].r, 1.0);
      Q[v].r = Qn[v].r;
    }
    if (p.graph) inc_step(c, dev_step);
    c.sync();
  }

  // replace the separable terms: ghost terms get their exact-axis column (zero inside the
  // domain) and their other factor extended by the other axis's rule, both n + 6 rows
  void set_terms(const tt_fv_term *tv, int count) {
    TT_REQUIRE(!p.graph || count == 0,
               "tt_fv_set_terms: graph mode has no time-dependent terms (their factors would "
               "be fixed in the captured step)");
    TT_REQUIRE(count >= 0 && (count == 0 || tv), "tt_fv_set_terms: bad term list");
    const size_t col = (size_t)n + 6;
    std::vector<double> host((size_t)count * 2 * col, 0.0);
    std::vector<DevTerm> nt;
    for (int k = 0; k < count; ++k) {
      const tt_fv_term &a = tv[k];
      TT_REQUIRE(a.var >= 0 && a.var < 3, "tt_fv_set_terms: var must be 0, 1 or 2");
      TT_REQUIRE(a.where >= TT_TERM_FORCING && a.where <= TT_TERM_Y_HI,
                 "tt_fv_set_terms: unknown where");
      TT_REQUIRE(a.X && a.Y, "tt_fv_set_terms: null factor");
      TT_REQUIRE(std::isfinite(a.amp) && std::isfinite(a.omega) && std::isfinite(a.phase),
                 "tt_fv_set_terms: non-finite time factor");
      double *e = host.data() + (size_t)k * 2 * col, *o = e + col;
      if (a.where == TT_TERM_FORCING) {
        std::copy(a.X, a.X + n, e);
        std::copy(a.Y, a.Y + n, o);
      } else {
        const int ax = (a.where == TT_TERM_X_LO || a.where == TT_TERM_X_HI) ? 0 : 1;
        TT_REQUIRE(rule_ax[ax] == Ghost::Zero,
                   "tt_fv_set_terms: ghost terms need an exact boundary on their axis");
        const bool lo = a.where == TT_TERM_X_LO || a.where == TT_TERM_Y_LO;
        const double *g = ax == 0 ? a.X : a.Y, *other = ax == 0 ? a.Y : a.X;
        for (int i = 0; i < 3; ++i) e[lo ? i : n + 3 + i] = g[i];
        // the other factor along axis 1 - ax: its rule; walls negate the momentum normal to it
        const int b = 1 - ax;
        const double sign = (b == 0 && a.var == 1) || (b == 1 && a.var == 2) ? -1.0 : 1.0;
        for (int q = -3; q < n + 3; ++q) {
          double v;
          if (q >= 0 && q < n) v = other[q];
          else if (rule_ax[b] == Ghost::Periodic) v = other[((q % n) + n) % n];
          else v = sign * other[q < 0 ? -1 - q : 2 * n - 1 - q];
          o[q + 3] = v;
        }
      }
      nt.push_back({a.var, a.where, a.amp, a.omega, a.phase, nullptr, nullptr});
    }
    c.sync();
    if (term_mem) HIP_CHECK(hipFree(term_mem));
    term_mem = nullptr;
    terms.clear();
    if (count) {
      HIP_CHECK(hipMalloc((void **)&term_mem, host.size() * sizeof(double)));
      HIP_CHECK(hipMemcpy(term_mem, host.data(), host.size() * sizeof(double),
                          hipMemcpyHostToDevice));
      for (int k = 0; k < count; ++k) {
        nt[k].e = term_mem + (size_t)k * 2 * col;
        nt[k].o = nt[k].e + col;
      }
    }
    terms = std::move(nt);
  }
};

Solver *solver_create(const tt_fv_params *p, const tt_matrix q0[3], void *stream,
                      size_t arena_bytes) {
  TT_REQUIRE(p && q0, "tt_fv_init: null argument");
  TT_REQUIRE(p->n >= 6, "tt_fv_init: n must be >= 6");
  TT_REQUIRE(p->scheme == 3 || p->scheme == 5 || p->scheme == 55, "tt_fv_init: bad scheme");
  TT_REQUIRE(p->r_max >= 1 && p->r_max <= 64, "tt_fv_init: r_max must be in [1, 64]");
  TT_REQUIRE(p->eps >= 0.0, "tt_fv_init: eps < 0");
  TT_REQUIRE(p->eps_rule == TT_EPS_FIXED || p->eps_rule == TT_EPS_PAPER,
             "tt_fv_init: unknown eps_rule");
  TT_REQUIRE(p->bc_x >= 0 && p->bc_x <= TT_BC_EXACT && p->bc_y >= 0 && p->bc_y <= TT_BC_EXACT,
             "tt_fv_init: unknown boundary kind");
  TT_REQUIRE(p->flux == TT_FLUX_PRODUCTS || p->flux == TT_FLUX_LF_CROSS,
             "tt_fv_init: unknown flux method");
  TT_REQUIRE(p->cross_enrich == TT_ENRICH_KICKS || p->cross_enrich == TT_ENRICH_RESIDUAL,
             "tt_fv_init: unknown cross enrichment");
  TT_REQUIRE(p->flux != TT_FLUX_LF_CROSS || (p->cross_sweeps >= 1 && p->cross_kick >= 0),
             "tt_fv_init: bad cross parameters");
  TT_REQUIRE(!(p->bc_x == TT_BC_EXACT && p->bc_y == TT_BC_EXACT),
             "tt_fv_init: at most one axis can have exact boundaries");
  TT_REQUIRE(std::isfinite(p->t0), "tt_fv_init: t0 not finite");
  TT_REQUIRE(p->eps_rule != TT_EPS_PAPER || (p->c_eps > 0.0 && std::isfinite(p->c_eps)),
             "tt_fv_init: c_eps must be positive with TT_EPS_PAPER");
  TT_REQUIRE(!p->nonlinear || p->taylor_terms >= 1 || p->recip == 1,
             "tt_fv_init: taylor_terms < 1");
  TT_REQUIRE(p->recip == 0 || p->recip == 1, "tt_fv_init: recip must be 0 or 1");
  TT_REQUIRE(p->workers >= -1 && p->workers <= 16, "tt_fv_init: workers must be in [-1, 16]");
  TT_REQUIRE(p->precision == TT_PREC_F64 || p->precision == TT_PREC_F32,
             "tt_fv_init: unknown precision");
  TT_REQUIRE(p->qr == TT_QR_AUTO || p->qr == TT_QR_CHOLESKY || p->qr == TT_QR_HOUSEHOLDER,
             "tt_fv_init: unknown QR method");
  TT_REQUIRE(p->cross_drop >= 0.0 && p->cross_drop < 1.0, "tt_fv_init: cross_drop out of [0, 1)");
  TT_REQUIRE(p->recip == 0 || (p->cross_sweeps >= 1 && p->cross_kick >= 0),
             "tt_fv_init: bad cross parameters");
  TT_REQUIRE(p->scheme != 55 || (p->cross_sweeps >= 1 && p->cross_kick >= 0),
             "tt_fv_init: bad cross parameters");
  TT_REQUIRE(p->graph == 0 || p->graph == 1, "tt_fv_init: graph must be 0 or 1");
  TT_REQUIRE(p->graph_iters >= 0 && p->graph_iters <= 8, "tt_fv_init: graph_iters in [0, 8]");
  if (p->graph) {
    // every decision of these paths has a device-side form; the others read the host
    TT_REQUIRE(p->scheme == 3 || p->scheme == 5, "graph mode: Upwind3 or Upwind5 only");
    TT_REQUIRE(p->eps_rule == TT_EPS_FIXED, "graph mode: fixed eps only");
    TT_REQUIRE(p->flux == TT_FLUX_PRODUCTS, "graph mode: the product flux only");
    TT_REQUIRE(p->cross_enrich == TT_ENRICH_KICKS, "graph mode: seeded kicks only");
    TT_REQUIRE(p->bc_x != TT_BC_EXACT && p->bc_y != TT_BC_EXACT,
               "graph mode: no exact-solution boundaries");
    TT_REQUIRE(!p->nonlinear || (p->cross_sweeps >= 1 && p->cross_kick >= 0),
               "tt_fv_init: bad cross parameters");
    TT_REQUIRE(2 * p->r_max < p->n, "graph mode: n must exceed 2 r_max");
  }
  for (int v = 0; v < 3; ++v) {
    TT_REQUIRE(q0[v].n1 == p->n && q0[v].n2 == p->n, "tt_fv_init: state shape != n x n");
    TT_REQUIRE(q0[v].rank >= 1 && q0[v].rank <= p->r_max, "tt_fv_init: state rank out of range");
    TT_REQUIRE(q0[v].g1 && q0[v].g2, "tt_fv_init: null core");
  }
  Solver *s = new Solver();
  try {
    s->p = *p;
    s->c.stream = (hipStream_t)stream;
    s->c.fp32 = p->precision == TT_PREC_F32;
    s->c.qr = p->qr;
    s->c.cross_drop = p->cross_drop;
    s->c.enrich = p->cross_enrich;
    const size_t ab = arena_bytes ? arena_bytes : ((size_t)4 << 30);
    s->c.arena.init(ab);
    int dev = 0;
    HIP_CHECK(hipGetDevice(&dev));
    const int nw = p->graph ? 0 : p->workers == 0 ? 8 : p->workers;
    if (p->graph) {
      // the step is captured on a stream of the solver's own (the caller's may be the null
      // stream); the initial state was copied on the caller's stream, which is synchronised
      // before the first step
      HIP_CHECK(hipStreamSynchronize(s->c.stream));
      s->user_stream = s->c.stream;
      HIP_CHECK(hipStreamCreateWithFlags(&s->own_stream, hipStreamNonBlocking));
      HIP_CHECK(hipEventCreateWithFlags(&s->user_ev, hipEventDisableTiming));
      s->c.stream = s->own_stream;
      s->c.fixed = true;
      s->c.householder = true;   // no host-side check of a Cholesky QR in a graph
      // the range finder cannot add iterations on demand: two subspace iterations keep the
      // leak of the discarded directions at the dynamic path's level at a binding rank cap
      const int gi = p->graph_iters > 0 ? p->graph_iters : (s->c.fp32 ? 1 : 2);
      s->c.power_iters = gi;
      // branches: 4 by default; a member made for an ensemble (workers = -1) keeps one chain,
      // since graphs with branches replayed side by side do not overlap each other, while
      // single-chain graphs on their own streams do (measured)
      const int nb = p->workers > 0 ? p->workers : p->workers == 0 ? 4 : 1;
      // split-K arrival counters now: their first use must not put a memset into a graph
      if (nb > 1) {
        HIP_CHECK(hipEventCreateWithFlags(&s->fork_ev, hipEventDisableTiming));
        for (int b = 0; b < nb; ++b) {
          auto w = std::make_unique<Ctx>();
          HIP_CHECK(hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking));
          w->arena.init(std::max(ab / 2, (size_t)64 << 20));
          w->fixed = true;
          w->householder = true;
          w->power_iters = gi;
          w->prepare();
          s->branch.push_back(std::move(w));
          hipEvent_t e;
          HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
          s->join_ev.push_back(e);
        }
      }
      s->site_cap = p->r_max;
      s->site_have.assign(Solver::kSites, 0);
      s->site_J = s->c.arena.ialloc((size_t)Solver::kSites * (s->site_cap + 1));
      s->dev_step = static_cast<long long *>(s->c.arena.alloc(sizeof(long long)));
      HIP_CHECK(hipMemsetAsync(s->site_J, 0,
                               (size_t)Solver::kSites * (s->site_cap + 1) * sizeof(int),
                               s->c.stream));
      HIP_CHECK(hipMemsetAsync(s->dev_step, 0, sizeof(long long), s->c.stream));
    }
    if (nw > 0) {
      s->pool = std::make_unique<Pool>(nw, ab, dev);
      s->exec = s->pool.get();
      // helper streams for the Taylor partial sums; a single worker keeps every kernel of
      // the step on one stream
      if (nw > 1 && p->nonlinear && p->recip == 0)
        for (auto &a : s->aux) {
          a = std::make_unique<Ctx>();
          HIP_CHECK(hipStreamCreateWithFlags(&a->stream, hipStreamNonBlocking));
          a->arena.init((size_t)512 << 20);
          a->prepare(std::max((int)Ctx::kTermEvents, p->taylor_terms));
        }
    }
    s->st = derive_stencils(p->scheme == 3 ? 3 : 5);
    s->wt = derive_weno_tables();
    s->n = p->n;
    s->nq = s->st.nq;
    for (int a = 0; a < 2; ++a) {
      const int kind = (a == 0 ? p->bc_x : p->bc_y) ? (a == 0 ? p->bc_x : p->bc_y)
                                                    : (p->periodic ? TT_BC_PERIODIC : TT_BC_WALL);
      s->rule_ax[a] = kind == TT_BC_PERIODIC ? Ghost::Periodic
                      : kind == TT_BC_WALL   ? Ghost::Wall
                                             : Ghost::Zero;
      s->periodic_ax[a] = kind == TT_BC_PERIODIC;
      s->nf_ax[a] = s->periodic_ax[a] ? p->n : p->n + 1;
    }
    s->t = p->t0;
    if (s->rule_ax[0] == Ghost::Zero || s->rule_ax[1] == Ghost::Zero) {
      const int n6 = p->n + 6;
      std::vector<int> rows{0, 1, 2, p->n + 3, p->n + 4, p->n + 5};
      std::vector<double> unit((size_t)n6 * 6, 0.0);
      for (int k = 0; k < 6; ++k) unit[(size_t)k * n6 + rows[k]] = 1.0;
      s->ghost_rows6 = s->c.arena.ialloc(6);
      s->unit6 = s->c.arena.dalloc(unit.size());
      HIP_CHECK(hipMemcpyAsync(s->ghost_rows6, rows.data(), 6 * sizeof(int),
                               hipMemcpyHostToDevice, s->c.stream));
      HIP_CHECK(hipMemcpyAsync(s->unit6, unit.data(), unit.size() * sizeof(double),
                               hipMemcpyHostToDevice, s->c.stream));
      s->c.sync();
    }
    for (int v = 0; v < 3; ++v) {
      s->Q[v] = Solver::alloc(s->c, p->n, p->n, p->r_max);
      s->Q[v].r = q0[v].rank;
      HIP_CHECK(hipMemcpyAsync(s->Q[v].A, q0[v].g1, (size_t)p->n * q0[v].rank * 8,
                               hipMemcpyDeviceToDevice, s->c.stream));
      HIP_CHECK(hipMemcpyAsync(s->Q[v].B, q0[v].g2, (size_t)p->n * q0[v].rank * 8,
                               hipMemcpyDeviceToDevice, s->c.stream));
    }
    std::vector<int> rep((size_t)p->n * s->nq);
    for (int j = 0; j < p->n; ++j)
      for (int m = 0; m < s->nq; ++m) rep[(size_t)j * s->nq + m] = j;
    s->rep_idx = s->c.arena.ialloc(rep.size());
    HIP_CHECK(hipMemcpyAsync(s->rep_idx, rep.data(), rep.size() * sizeof(int),
                             hipMemcpyHostToDevice, s->c.stream));
    s->c.prepare();   // nothing of the context is allocated later, in a step
    s->c.sync();
    s->set_tolerances();
  } catch (...) {
    delete s;
    throw;
  }
  return s;
}

void solver_max_speed(Solver *s, double out[2]) {
  out[0] = s->max_speed(0);
  out[1] = s->max_speed(1);
}

// dt = cfl / (s_x / dx + s_y / dy), dx = dy = 1/n
double solver_cfl_dt(Solver *s, double cfl) {
  double sp[2];
  solver_max_speed(s, sp);
  TT_REQUIRE(sp[0] + sp[1] > 0.0, "tt_fv_cfl_dt: zero wave speed");
  return cfl / ((sp[0] + sp[1]) * s->n);
}

void solver_set_terms(Solver *s, const tt_fv_term *terms, int count) {
  s->set_terms(terms, count);
}

void solver_step(Solver *s, double dt, int nsteps) {
  TT_REQUIRE(nsteps >= 0 && std::isfinite(dt), "tt_fv_step: bad dt or nsteps");
  TT_REQUIRE(s->exec || s->p.graph,
             "tt_fv_step: solver made with workers = -1 steps only inside an ensemble");
  s->after_user();
  for (int k = 0; k < nsteps; ++k) s->step(dt);
  if (s->p.graph) s->fixed_status_all();
}

// ---- ensemble: members share one pool; host threads take members in cost order --------
struct Ensemble {
  std::unique_ptr<Pool> pool;
  std::vector<hipStream_t> gstreams;   // graph mode: streams the members' graphs replay on
  ~Ensemble() {
    for (hipStream_t st : gstreams) {
      (void)hipStreamSynchronize(st);
      (void)hipStreamDestroy(st);
    }
  }
};

// Graph mode: each member's first step runs eagerly and its next step is captured, on
// `concurrency` host threads (members on their own streams); then every member's graph is
// launched for the remaining steps on one of `concurrency` streams (chosen longest-processing-
// time first), one host thread per stream, with no host round trip until the end.
void ensemble_step_graph(Ensemble *e, Solver *const *members, int count, const double *dts,
                         int nsteps, int concurrency) {
  std::vector<int> order(count), rem(count, nsteps);
  for (int i = 0; i < count; ++i) order[i] = i;
  auto cost = [&](int i) {
    const double r = members[i]->p.r_max, n = members[i]->n;
    return n * r * r * r * r;
  };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) > cost(b); });
  // prepare: eager first steps and captures, in parallel over members
  {
    std::mutex qm;
    size_t next = 0;
    std::exception_ptr err;
    auto worker = [&]() {
      for (;;) {
        int idx;
        {
          std::lock_guard<std::mutex> lk(qm);
          if (next >= order.size() || err) return;
          idx = order[next++];
        }
        try {
          Solver *m = members[idx];
          TT_REQUIRE(std::isfinite(dts[idx]), "tt_ens_step: bad dt");
          while (rem[idx] > 0 && !m->warm) {
            m->step_graph(dts[idx]);
            --rem[idx];
          }
          if (rem[idx] > 0 &&
              (!m->gexec || dts[idx] != m->graph_dt || m->c.arena.mark() != m->graph_mark))
            m->capture(dts[idx]);
          HIP_CHECK(hipStreamSynchronize(m->c.stream));
        } catch (...) {
          std::lock_guard<std::mutex> lk(qm);
          if (!err) err = std::current_exception();
          return;
        }
      }
    };
    std::vector<std::thread> th;
    int dev = 0;
    HIP_CHECK(hipGetDevice(&dev));
    for (int t = 0; t < std::min(concurrency, count); ++t)
      th.emplace_back([&, dev]() {
        (void)hipSetDevice(dev);
        worker();
      });
    for (auto &t : th) t.join();
    if (err) std::rethrow_exception(err);
  }
  const int ns = std::min(concurrency, count);
  while ((int)e->gstreams.size() < ns) {
    hipStream_t st;
    HIP_CHECK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    e->gstreams.push_back(st);
  }
  // members to streams: the least loaded stream takes the next most expensive member
  std::vector<int> sid(count, 0);
  std::vector<double> load(ns, 0.0);
  for (int i : order) {
    const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    sid[i] = k;
    load[k] += cost(i);
  }
  // one host thread per stream launches its members' graphs, step by step
  {
    std::vector<std::thread> th;
    std::vector<std::exception_ptr> errs(ns);
    int dev = 0;
    HIP_CHECK(hipGetDevice(&dev));
    for (int k = 0; k < ns; ++k)
      th.emplace_back([&, k, dev]() {
        (void)hipSetDevice(dev);
        try {
          int most = 0;
          for (int i : order)
            if (sid[i] == k) most = std::max(most, rem[i]);
          for (int step = 0; step < most; ++step)
            for (int i : order) {
              if (sid[i] != k || step >= rem[i]) continue;
              Solver *m = members[i];
              HIP_CHECK(hipGraphLaunch(m->gexec, e->gstreams[k]));
              ++m->graph_launches;
              const Counters &g = m->graph_cnt;
              m->c.cnt.roundings += g.roundings;
              m->c.cnt.crosses += g.crosses;
              m->c.cnt.flops += g.flops;
              m->c.cnt.bytes += g.bytes;
              m->sweeps_run += m->graph_sweeps;
              ++m->step_index;
              m->t += dts[i];
            }
          HIP_CHECK(hipStreamSynchronize(e->gstreams[k]));
        } catch (...) {
          errs[k] = std::current_exception();
        }
      });
    for (auto &t : th) t.join();
    for (auto &x : errs)
      if (x) std::rethrow_exception(x);
  }
  for (int i = 0; i < count; ++i) members[i]->fixed_status_all();
}

Ensemble *ensemble_create(int workers, size_t arena_bytes) {
  TT_REQUIRE(workers >= 1 && workers <= 32, "tt_ens_create: workers must be in [1, 32]");
  int dev = 0;
  HIP_CHECK(hipGetDevice(&dev));
  Ensemble *e = new Ensemble();
  e->pool = std::make_unique<Pool>(workers, arena_bytes ? arena_bytes : ((size_t)1 << 30), dev);
  return e;
}

void ensemble_destroy(Ensemble *e) { delete e; }

void ensemble_step(Ensemble *e, Solver *const *members, int count, const double *dts,
                   int nsteps, int concurrency) {
  TT_REQUIRE(count >= 1 && members && dts, "tt_ens_step: no members");
  TT_REQUIRE(concurrency >= 1 && concurrency <= 256, "tt_ens_step: concurrency in [1, 256]");
  for (int i = 0; i < count; ++i) {
    TT_REQUIRE(members[i], "tt_ens_step: null member");
    TT_REQUIRE(std::isfinite(dts[i]), "tt_ens_step: bad dt");
  }
  int ngraph = 0;
  for (int i = 0; i < count; ++i) ngraph += members[i]->p.graph ? 1 : 0;
  TT_REQUIRE(ngraph == 0 || ngraph == count,
             "tt_ens_step: members must all be in graph mode or none");
  if (ngraph) {
    ensemble_step_graph(e, members, count, dts, nsteps, concurrency);
    return;
  }
  // longest-processing-time first: a Hadamard rounding costs ~ n r^4
  std::vector<int> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  auto cost = [&](int i) {
    const double r = members[i]->p.r_max, n = members[i]->n;
    return n * r * r * r * r;
  };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) > cost(b); });
  std::vector<Pool *> saved(count);
  for (int i = 0; i < count; ++i) {
    saved[i] = members[i]->exec;
    members[i]->exec = e->pool.get();
  }
  std::mutex qm;
  size_t next = 0;
  std::exception_ptr err;
  auto worker = [&]() {
    for (;;) {
      int idx;
      {
        std::lock_guard<std::mutex> lk(qm);
        if (next >= order.size() || err) return;
        idx = order[next++];
      }
      try {
        for (int k = 0; k < nsteps; ++k) members[idx]->step(dts[idx]);
      } catch (...) {
        std::lock_guard<std::mutex> lk(qm);
        if (!err) err = std::current_exception();
        return;
      }
    }
  };
  std::vector<std::thread> th;
  const int nt = std::min(concurrency, count);
  int dev = 0;
  HIP_CHECK(hipGetDevice(&dev));
  for (int t = 0; t < nt; ++t)
    th.emplace_back([&, dev]() {
      (void)hipSetDevice(dev);
      worker();
    });
  for (auto &t : th) t.join();
  for (int i = 0; i < count; ++i) members[i]->exec = saved[i];
  if (err) std::rethrow_exception(err);
}

void solver_get_state(Solver *s, tt_matrix q[3]) {
  s->after_user();   // the caller's buffers may still be written on its stream
  for (int v = 0; v < 3; ++v) {
    TT_REQUIRE(q[v].n1 == s->n && q[v].n2 == s->n && q[v].cap >= s->Q[v].r,
               "tt_fv_get_state: output too small");
    HIP_CHECK(hipMemcpyAsync(q[v].g1, s->Q[v].A, (size_t)s->n * s->Q[v].r * 8,
                             hipMemcpyDeviceToDevice, s->c.stream));
    HIP_CHECK(hipMemcpyAsync(q[v].g2, s->Q[v].B, (size_t)s->n * s->Q[v].r * 8,
                             hipMemcpyDeviceToDevice, s->c.stream));
    q[v].rank = s->Q[v].r;
  }
  s->c.sync();
}

void solver_stats(Solver *s, tt_fv_stats *o) {
  o->steps = s->step_index;
  for (int v = 0; v < 3; ++v) o->ranks[v] = s->Q[v].r;
  o->graph_launches = s->graph_launches;
  if (s->p.graph) {
    // the static rank of a fixed-shape state holds zero columns after the device's rank
    Scope sc(s->c.arena);
    int *rk = s->c.arena.ialloc(3);
    for (int v = 0; v < 3; ++v) count_rank(s->c, s->Q[v].B, s->n, s->Q[v].r, rk + v);
    HIP_CHECK(hipMemcpyAsync(o->ranks, rk, 3 * sizeof(int), hipMemcpyDeviceToHost, s->c.stream));
    HIP_CHECK(hipStreamSynchronize(s->c.stream));
    for (int v = 0; v < 3; ++v) o->ranks[v] = std::max(o->ranks[v], 1);
    s->c.cnt.warnings |= s->fixed_status_all();
  }
  Counters t = s->c.cnt;
  const int npool = s->pool ? s->pool->size() : 0;
  std::vector<const Counters *> cs;
  for (int i = 0; i < npool; ++i) cs.push_back(&s->pool->ctx(i).cnt);
  for (auto &a : s->aux)
    if (a) cs.push_back(&a->cnt);
  for (auto &b : s->branch) cs.push_back(&b->cnt);
  long long jcap = s->c.jacobi_capped();
  for (auto &b : s->branch) jcap += b->jacobi_capped();
  for (int i = 0; i < npool; ++i) jcap += s->pool->ctx(i).jacobi_capped();
  for (auto &a : s->aux)
    if (a) jcap += a->jacobi_capped();
  for (const Counters *wc : cs) {
    const Counters &w = *wc;
    t.sketch_fallbacks += w.sketch_fallbacks;
    t.qr_redos += w.qr_redos;
    t.sketch_unconverged += w.sketch_unconverged;
    t.roundings += w.roundings;
    t.crosses += w.crosses;
    t.flops += w.flops;
    t.bytes += w.bytes;
    t.warnings |= w.warnings;
    t.extra_power_iters += w.extra_power_iters;
  }
  o->cross_sweeps_run = s->sweeps_run;
  o->learned_crosses = s->learned;
  o->learned_fallbacks = s->fallbacks;
  o->max_learned_err = s->max_learned_err;
  o->roundings = t.roundings;
  o->crosses = t.crosses;
  o->last_taylor_terms = s->last_terms;
  o->last_taylor_err = s->last_err;
  o->warnings = t.warnings | (jcap > 0 ? TT_WJACOBI : 0);
  o->sketch_fallbacks = t.sketch_fallbacks;
  o->sketch_unconverged = t.sketch_unconverged;
  o->jacobi_capped = jcap;
  o->qr_redos = t.qr_redos;
  o->eps_inner = s->eps_in;
  o->time = s->t;
  for (int v = 0; v < 3; ++v) o->eps_var[v] = s->eps_q[v];
  o->flops = t.flops;
  o->bytes = t.bytes;
  std::vector<KernelTimer *> tm{&s->c.timer};
  for (int i = 0; i < npool; ++i) tm.push_back(&s->pool->ctx(i).timer);
  for (auto &a : s->aux)
    if (a) tm.push_back(&a->timer);
  const int nt = (int)tm.size();
  o->timed_ms = 0;
  o->timed_launches = 0;
  o->timed_flops = 0;
  o->timed_bytes = 0;
  for (int i = 0; i < nt; ++i) {
    o->timed_ms += tm[i]->ms;
    o->timed_launches += tm[i]->launches;
    o->timed_flops += tm[i]->flops;
    o->timed_bytes += tm[i]->bytes;
  }
}

void solver_time_kernel(Solver *s, const char *name, int every) {
  std::vector<Ctx *> cs{&s->c};
  for (int i = 0; s->pool && i < s->pool->size(); ++i) cs.push_back(&s->pool->ctx(i));
  for (auto &a : s->aux)
    if (a) cs.push_back(a.get());
  for (Ctx *c : cs) {
    c->sync();
    c->timer.name = name;
    c->timer.every = every;
    c->timer.ms = c->timer.flops = c->timer.bytes = 0;
    c->timer.launches = 0;
    c->timer.seen = 0;
  }
}

void solver_set_pivots(Solver *s, int mode, PivotModel *pm) {
  TT_REQUIRE(!s->p.graph || mode == TT_PIV_MAXVOL,
             "tt_fv_set_pivots: graph mode runs plain maxvol crosses only");
  std::lock_guard<std::mutex> lk(s->mu);
  s->piv_mode = mode;
  s->pm = pm;
}

void solver_set_acceptance(Solver *s, double abs_tol, double rel_slack) {
  std::lock_guard<std::mutex> lk(s->mu);
  s->acc_abs = abs_tol;
  s->acc_rel = rel_slack;
}

void solver_replay_pivots(Solver *s, long long step, int site, const int *J, int nJ,
                          const int *I, int nI) {
  TT_REQUIRE(step >= 0 && site >= 0, "tt_fv_replay_pivots: negative step or site");
  TT_REQUIRE(nJ >= 1 && nJ <= qr_max_cols() && nI >= 0 && nI <= nJ && J && (I || nI == 0),
             "tt_fv_replay_pivots: need 1 <= nJ <= 96 and 0 <= nI <= nJ");
  std::lock_guard<std::mutex> lk(s->mu);
  s->replay[{step, site}] = {std::vector<int>(J, J + nJ), std::vector<int>(I, I + nI)};
}

int solver_get_pivots(Solver *s, int site, int *J, int capJ, int *nJ, int *I, int capI,
                      int *nI) {
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->last_piv.find(site);
  if (it == s->last_piv.end()) {
    *nJ = 0;
    *nI = 0;
    return 0;
  }
  const auto &ji = it->second;
  TT_REQUIRE((int)ji.first.size() <= capJ && (int)ji.second.size() <= capI,
             "tt_fv_get_pivots: output capacity too small");
  std::copy(ji.first.begin(), ji.first.end(), J);
  std::copy(ji.second.begin(), ji.second.end(), I);
  *nJ = (int)ji.first.size();
  *nI = (int)ji.second.size();
  return 1;
}

void solver_destroy(Solver *s) { delete s; }

}  // namespace ttfv
