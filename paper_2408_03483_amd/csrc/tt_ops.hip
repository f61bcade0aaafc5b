// Host-side TT algorithms built from the device kernels: rounding (Section 3.2),
// the Taylor reciprocal (Algorithm 1), and the alternating maxvol cross (Section 3.3).
//
// Rounding of X = A B^T (rank R) to (eps, rmax):
//   * R small (R <= sketch width and both modes): QR of both cores, M = Ra Rb^T, SVD of M
//     (the two-core form of orthogonalise-then-truncated-SVD);
//   * R large (e.g. Hadamard products, R = r_x r_y): a randomized range finder (Halko,
//     Martinsson and Tropp 2011) replaces the R x R SVD: Y = X Omega with a Gaussian
//     Omega of `width` columns (default 2 rmax), `power_iters` subspace iterations, Qa = orth(Y),
//     W = X^T Qa = Qb Rb, M = Rb^T; SVD of M.  Only GEMMs touch the n x R cores; the
//     factorizations are of width <= 96.
//   The rank k is the smallest with sqrt(sum_{i>=k} s_i^2) <= eps ||s|| capped at rmax.
//   Output gauge: A' = Qa U_k (orthonormal columns), B' = Qb M^T U_k (carries Sigma).
#include "common.h"
#include "rules.h"

#include <algorithm>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <exception>
#include <mutex>
#include <thread>
#include <unordered_set>

namespace ttfv {

namespace {

// small reads go through the context's pinned staging buffer: a copy into pageable memory
// is staged by the runtime and costs a longer round trip on this path of every rounding
std::vector<double> to_host(Ctx &c, const double *dev, size_t n) {
  TT_REQUIRE(!c.capturing, "graph capture: a step read a device value on the host");
  std::vector<double> h(n);
  double *st = n && n <= Ctx::kPinnedDoubles ? c.pinned_staging() : nullptr;
  if (st) {
    HIP_CHECK(hipMemcpyAsync(st, dev, n * sizeof(double), hipMemcpyDeviceToHost, c.stream));
    c.sync();
    std::copy(st, st + n, h.begin());
    return h;
  }
  if (n) HIP_CHECK(hipMemcpyAsync(h.data(), dev, n * sizeof(double), hipMemcpyDeviceToHost,
                                  c.stream));
  c.sync();
  return h;
}

// Kept rank of a truncation (rules.h: the rule the fixed-shape kernels take too)
int trunc_rank(const std::vector<double> &s, double eps, int rmax, double floor_rel,
               bool *capped) {
  const int m = (int)s.size();
  std::vector<double> tail(m + 1, 0.0);
  return rule_trunc_rank(s.data(), m, eps, rmax, floor_rel, tail.data(), capped);
}

// SVD of an m x m core (not transposed).  From m = 48 on, a pivoted QR first grades the
// matrix, which cuts the Jacobi sweeps on strongly graded spectra (the orthogonalisations of
// the cross iterations, exact roundings of sums of decaying TTs) from about 20 to about 7.
void small_svd(Ctx &c, const double *M, int m, double *US, double *sg, double floor_rel) {
  if (m >= 48 && m <= QR_MAXM) svd_pivoted(c, M, m, US, sg, floor_rel);
  else jacobi_svd(c, M, m, US, sg, false, floor_rel);
}

// Norm floor of a rounding's Jacobi SVD, relative to ||M||_F: columns below it take no
// rotations, so the kept part can differ from the exact truncated SVD by about the floor.
// eps / 100 keeps a rounding within its tolerance; the cap at 1e-13 keeps it at round-off
// level as well, which the rank-capped dam break needs (it amplifies a 5e-10 change of one
// step's state into 1e-7 over the next step, so an eps / 100 floor at eps = 1e-8 moves its
// result by 1e-7 from the exact rounding's).
double jacobi_floor(double eps) { return std::min(1e-2 * eps, 1e-13); }

void require_finite(const std::vector<double> &s, const char *what) {
  for (double v : s)
    if (!std::isfinite(v))
      throw Error(TT_ENONFINITE, std::string(what) + ": non-finite singular value");
}

void zero_tt(Ctx &c, DTT &y) {
  fill_value(c, y.A, y.n1, y.n1, 1, 0.0);
  fill_value(c, y.B, y.n2, y.n2, 1, 0.0);
  y.r = 1;
}

uint64_t g_sketch_seed = 0x5EED5EED12345ull;

// number of orthonormal directions orth keeps: those above drop * s_0, or exactly `want`
// (a replayed skeleton fixes its width), which must all be nonzero
int kept_directions(const std::vector<double> &s, double drop, int want) {
  const int m = (int)s.size();
  if (want >= 0) {
    TT_REQUIRE(want <= m && (want == 0 || s[want - 1] > 0.0),
               "orth: the columns have fewer nonzero directions than requested");
    return want;
  }
  return rule_kept_directions(s.data(), m, drop);
}

}  // namespace

namespace {

// Runs f with Cholesky QR; when that leaves non-finite singular values (a Cholesky QR that
// ended without orthonormal columns sets its Q and R to NaN), runs f again with Householder
// QR, which reports a truly non-finite input as before.
template <typename F>
auto with_qr_fallback(Ctx &c, F &&f) -> decltype(f()) {
  if (c.householder) return f();
  try {
    return f();
  } catch (const Error &e) {
    if (e.code != TT_ENONFINITE) throw;
  }
  c.cnt.qr_redos++;
  c.householder = true;
  try {
    auto r = f();
    c.householder = false;
    return r;
  } catch (...) {
    c.householder = false;
    throw;
  }
}

int round_impl(Ctx &c, const DTT &x, double eps, int rmax, DTT &y,
               std::vector<double> *sig_out);

}  // namespace

int round_tt(Ctx &c, const DTT &x, double eps, int rmax, DTT &y, std::vector<double> *sig_out) {
  if (c.fixed) {
    TT_REQUIRE(!sig_out, "fixed shapes: a rounding does not return its singular values");
    return round_fixed(c, x, eps, rmax, y);
  }
  const long long r0 = c.cnt.roundings;
  return with_qr_fallback(c, [&]() {
    c.cnt.roundings = r0;     // a redone rounding counts once
    return round_impl(c, x, eps, rmax, y, sig_out);
  });
}

namespace {

int round_impl(Ctx &c, const DTT &x, double eps, int rmax, DTT &y,
               std::vector<double> *sig_out) {
  TT_REQUIRE(x.r >= 1 && rmax >= 1, "round: empty input or rmax < 1");
  TT_REQUIRE(x.n1 == y.n1 && x.n2 == y.n2, "round: shape mismatch");
  c.cnt.roundings++;
  Scope sc(c.arena);
  const int n1 = x.n1, n2 = x.n2, R = x.r;
  const int qmax = qr_max_cols();
  int width = c.sketch_width > 0 ? c.sketch_width : std::min(QR_MAXM, std::max(2 * rmax, 16));
  width = std::min(width, qmax);
  const int mn = std::min(n1, n2);

  const double *Qa = nullptr, *Qb = nullptr;
  // The second output core is Qb M^T U_k.  Qb is only formed for tiny modes: on the exact
  // path Qb M^T = Qb Rb Ra^T = x.B Ra^T, and on the range finder Qb M^T = Qb Rb = W with
  // W = X^T Qa, so those paths need only the R factor of the second QR.
  const double *Bsrc = nullptr, *Ra_exact = nullptr;
  int bsrc_cols = 0;
  double *M = nullptr;
  bool Mt = false;           // M holds the transpose of the core to decompose
  double *US = nullptr, *sg = nullptr;   // SVD of M once computed
  std::vector<double> s_host;            // its singular values on the host, when fetched
  int sketch_warn = 0;                   // TT_WSKETCH when the range finder did not converge
  int m = 0;
  if (R <= width && R <= mn) {
    m = R;
    double *qa = c.arena.dalloc((size_t)n1 * m), *ra = c.arena.dalloc((size_t)m * m);
    double *rb = c.arena.dalloc((size_t)m * m);
    tsqr(c, x.A, n1, m, n1, qa, n1, ra, m);
    tsqr(c, x.B, n2, m, n2, nullptr, 0, rb, m);                        // R only
    M = c.arena.dalloc((size_t)m * m);
    gemm2(c, false, true, m, m, m, 1.0, ra, m, rb, m, 0.0, M, m);     // Ra Rb^T
    Qa = qa;
    Bsrc = x.B;
    bsrc_cols = m;
    Ra_exact = ra;
  } else if (mn <= width && mn <= qmax) {
    // tiny modes: materialise the full matrix on the smaller side
    if (n2 <= n1) {
      // X = (A B^T) I: A' = A B^T (n1 x n2), B' = I (n2 x n2)
      m = n2;
      double *F = c.arena.dalloc((size_t)n1 * n2);
      gemm2(c, false, true, n1, n2, R, 1.0, x.A, n1, x.B, n2, 0.0, F, n1);
      double *qa = c.arena.dalloc((size_t)n1 * m), *ra = c.arena.dalloc((size_t)m * m);
      tsqr(c, F, n1, m, n1, qa, n1, ra, m);
      double *qb = c.arena.dalloc((size_t)n2 * m);
      fill_value(c, qb, n2, n2, m, 0.0);
      {
        std::vector<double> eye((size_t)m * m, 0.0);
        for (int i = 0; i < m; ++i) eye[(size_t)i * m + i] = 1.0;
        HIP_CHECK(hipMemcpyAsync(qb, eye.data(), eye.size() * 8, hipMemcpyHostToDevice, c.stream));
        c.sync();
      }
      M = ra;
      Qa = qa;
      Qb = qb;
    } else {
      m = n1;
      double *F = c.arena.dalloc((size_t)n2 * n1);                  // X^T = B A^T
      gemm2(c, false, true, n2, n1, R, 1.0, x.B, n2, x.A, n1, 0.0, F, n2);
      double *qb = c.arena.dalloc((size_t)n2 * m), *rb = c.arena.dalloc((size_t)m * m);
      tsqr(c, F, n2, m, n2, qb, n2, rb, m);
      double *qa = c.arena.dalloc((size_t)n1 * m);
      {
        std::vector<double> eye((size_t)m * m, 0.0);
        for (int i = 0; i < m; ++i) eye[(size_t)i * m + i] = 1.0;
        HIP_CHECK(hipMemcpyAsync(qa, eye.data(), eye.size() * 8, hipMemcpyHostToDevice, c.stream));
        c.sync();
      }
      M = c.arena.dalloc((size_t)m * m);
      transpose(c, M, m, rb, m, m, m);                               // X = I Rb^T Qb^T
      Qa = qa;
      Qb = qb;
    }
  } else {
    // randomized range finder with subspace iterations; more iterations are run while the
    // estimated leak (s_m / s_k)^(2q+1) s_k of the discarded directions is above 1e-13 s_0
    m = std::min(width, mn);
    double *Om = c.arena.dalloc((size_t)n2 * m);
    // the test matrix depends only on the shape, so a rounding gives the same result on any
    // stream or worker (and run to run)
    fill_gauss(c, Om, n2, m, n2,
               g_sketch_seed ^ ((uint64_t)n1 * 0x9E3779B97F4A7C15ull) ^ ((uint64_t)n2 << 20) ^
                   ((uint64_t)R << 40) ^ (uint64_t)m);
    double *T = c.arena.dalloc((size_t)R * m);
    double *Y = c.arena.dalloc((size_t)n1 * m);
    double *Z = c.arena.dalloc((size_t)n2 * m);
    double *qa = c.arena.dalloc((size_t)n1 * m), *qz = c.arena.dalloc((size_t)n2 * m);
    double *rb = c.arena.dalloc((size_t)m * m);
    double *rtmp = c.arena.dalloc((size_t)m * m);
    gemm(c, true, R, m, n2, 1.0, x.B, n2, Om, n2, 0.0, T, R);          // B^T Omega
    gemm(c, false, n1, m, R, 1.0, x.A, n1, T, R, 0.0, Y, n1);          // Y = X Omega
    int q = 0;
    const int qlim = std::max(c.power_iters, c.sketch_max_iters);
    bool unconverged = false;
    for (;;) {
      for (; q < c.power_iters; ++q) {
        tsqr(c, Y, n1, m, n1, qa, n1, rtmp, m);
        gemm(c, true, R, m, n1, 1.0, x.A, n1, qa, n1, 0.0, T, R);      // A^T Qy
        gemm(c, false, n2, m, R, 1.0, x.B, n2, T, R, 0.0, Z, n2);      // X^T Qy
        tsqr(c, Z, n2, m, n2, qz, n2, rtmp, m);
        gemm(c, true, R, m, n2, 1.0, x.B, n2, qz, n2, 0.0, T, R);      // B^T Qz
        gemm(c, false, n1, m, R, 1.0, x.A, n1, T, R, 0.0, Y, n1);      // Y = X Qz
      }
      tsqr(c, Y, n1, m, n1, qa, n1, rtmp, m);
      gemm(c, true, R, m, n1, 1.0, x.A, n1, qa, n1, 0.0, T, R);        // A^T Qa
      gemm(c, false, n2, m, R, 1.0, x.B, n2, T, R, 0.0, Z, n2);        // W = X^T Qa
      tsqr(c, Z, n2, m, n2, nullptr, 0, rb, m);                        // W = Qb Rb (R only)
      M = rb;                                                          // X ~ Qa Rb^T Qb^T
      Mt = true;                                                       // (M^T held)
      // singular values of Rb estimate those of X on the captured subspace
      if (!US) {
        US = c.arena.dalloc((size_t)m * m);
        sg = c.arena.dalloc((size_t)m);
      }
      jacobi_svd(c, M, m, US, sg, Mt, jacobi_floor(eps));
      s_host = to_host(c, sg, m);
      const std::vector<double> &s = s_host;
      if (s[0] == 0.0) break;
      const int k = trunc_rank(s, eps, rmax, jacobi_floor(eps), nullptr);
      if (k >= m) break;
      // (a) the sketch reached round-off: beyond m - p the captured spectrum is below
      //     1e-14 s_0, so with oversampling p the range error is at that level;
      // (b) otherwise the subspace iteration has contracted the discarded directions by
      //     (s_m / s_k)^(2q+1); what they can still leak into the kept part is at most that
      //     factor times s_k, which must be below 1e-13 s_0.
      const int pover = std::max(8, m / 4);
      if (m - pover > k && s[m - pover] <= 1e-14 * s[0]) break;
      const double ratio = s[m - 1] / s[k - 1];
      if (std::pow(ratio, 2 * q + 1) * s[k - 1] <= 1e-13 * s[0]) break;
      if (q >= qlim) {
        unconverged = true;
        break;
      }
      US = nullptr;   // basis changes below: the SVD must be recomputed
      s_host.clear();
      // one more subspace iteration from the current basis: Y = X (X^T Qa) = X Z
      tsqr(c, Z, n2, m, n2, qz, n2, rtmp, m);
      gemm(c, true, R, m, n2, 1.0, x.B, n2, qz, n2, 0.0, T, R);
      gemm(c, false, n1, m, R, 1.0, x.A, n1, T, R, 0.0, Y, n1);
      ++q;
      c.cnt.extra_power_iters++;
    }
    if (unconverged) {
      // the discarded directions may still leak more than 1e-13 s_0 into the kept part:
      // redo the rounding exactly (QR of both cores and SVD of Ra Rb^T) when the input rank
      // fits the factorization width, else keep the sketch's answer and say so
      if (R <= qmax && R <= mn) {
        c.cnt.sketch_fallbacks++;
        c.cnt.roundings--;
        const int saved = c.sketch_width;
        c.sketch_width = R;
        int w = 0;
        try {
          w = round_tt(c, x, eps, rmax, y, sig_out);
        } catch (...) {
          c.sketch_width = saved;
          throw;
        }
        c.sketch_width = saved;
        return w;
      }
      c.cnt.sketch_unconverged++;
      sketch_warn = TT_WSKETCH;
    }
    Qa = qa;
    Bsrc = Z;
    bsrc_cols = m;
  }
  // SVD of the m x m core
  if (!US) {
    US = c.arena.dalloc((size_t)m * m);
    sg = c.arena.dalloc((size_t)m);
    if (Mt) jacobi_svd(c, M, m, US, sg, true, jacobi_floor(eps));
    else small_svd(c, M, m, US, sg, jacobi_floor(eps));
  }
  // the range finder's last check already brought these singular values to the host
  std::vector<double> s = s_host.empty() ? to_host(c, sg, m) : std::move(s_host);
  require_finite(s, "round");
  int warn = sketch_warn;
  if (s[0] == 0.0) {
    zero_tt(c, y);
    if (sig_out) sig_out->assign(1, 0.0);
    c.cnt.warnings |= warn;
    return warn;
  }
  bool capped = false;
  const int k = trunc_rank(s, eps, rmax, jacobi_floor(eps), &capped);
  if (capped) warn |= TT_WRANKCAP;
  double *U = c.arena.dalloc((size_t)m * k);
  normalise_cols(c, US, sg, m, k, U);
  gemm(c, false, n1, k, m, 1.0, Qa, n1, U, m, 0.0, y.A, n1);
  if (Bsrc && !Ra_exact) {
    gemm(c, false, n2, k, bsrc_cols, 1.0, Bsrc, n2, U, m, 0.0, y.B, n2);  // W U_k
  } else {
    double *W = c.arena.dalloc((size_t)m * k);
    if (Ra_exact)
      gemm(c, true, m, k, m, 1.0, Ra_exact, m, U, m, 0.0, W, m);        // Ra^T U_k
    else
      gemm(c, true, m, k, m, 1.0, M, m, U, m, 0.0, W, m);               // M^T U_k
    gemm(c, false, n2, k, bsrc_cols ? bsrc_cols : m, 1.0, Bsrc ? Bsrc : Qb, n2, W, m, 0.0, y.B,
         n2);
  }
  y.r = k;
  if (sig_out) sig_out->assign(s.begin(), s.begin() + k);
  c.cnt.warnings |= warn;
  return warn;
}

}  // namespace

size_t round_arena_bound(int n1, int n2, int R, int rmax) {
  auto al = [](size_t d) { return ((d * sizeof(double)) + 255) & ~(size_t)255; };
  const int qmax = qr_max_cols();
  const int width = std::min(std::min(QR_MAXM, std::max(2 * rmax, 16)), qmax);
  const int mn = std::min(n1, n2), nmax = std::max(n1, n2);
  const size_t N1 = n1, N2 = n2, RR = R;
  size_t persist = 0, transient = 0;
  auto tr = [&](size_t b) { transient = std::max(transient, b); };
  // the last part of every path: U_k, and W of the exact path, plus an SVD's pivoted-QR scratch
  auto tail = [&](int m) {
    const size_t mm = (size_t)m * m;
    persist += 4 * al(mm) + al(m);                 // US, sg, U, W
    tr(3 * al(mm) + gemm_arena_bytes(m, m, m));
    tr(gemm_arena_bytes(n1, m, m));
    tr(gemm_arena_bytes(n2, m, m));
    tr(gemm_arena_bytes(m, m, m));
  };
  // exact path (also the redo of an unconverged range finder)
  if (R <= qmax && R <= mn) {
    const size_t m = R;
    persist += al(N1 * m) + 3 * al(m * m);
    tr(tsqr_arena_bytes(n1, R));
    tr(tsqr_arena_bytes(n2, R));
    tail(R);
  }
  if (R <= width && R <= mn) return persist + transient + 64 * 256;
  if (mn <= width && mn <= qmax) {
    const size_t m = mn;
    persist += al(N1 * N2) + 2 * al((N1 + N2) * m) + 2 * al(m * m);
    tr(gemm_arena_bytes(nmax, mn, R));
    tr(tsqr_arena_bytes(nmax, mn));
    tail(mn);
    return persist + transient + 64 * 256;
  }
  const int m = std::min(width, mn);
  const size_t M = m;
  // Omega, T, Y, Z, Qa, Qz, Rb, Rtmp; and a fresh (US, sg) per convergence check, at most
  // one per subspace iteration up to the default limit of 8
  persist += al(N2 * M) + al(RR * M) + al(N1 * M) + al(N2 * M) + al(N1 * M) + al(N2 * M) +
             2 * al(M * M) + 10 * (al(M * M) + al(M));
  tr(gemm_arena_bytes(R, m, n2));
  tr(gemm_arena_bytes(n1, m, R));
  tr(gemm_arena_bytes(R, m, n1));
  tr(gemm_arena_bytes(n2, m, R));
  tr(tsqr_arena_bytes(n1, m));
  tr(tsqr_arena_bytes(n2, m));
  tail(m);
  return persist + transient + 64 * 256;
}

namespace {
void orth_impl(Ctx &c, const double *C, int n, int m, int ldc, double drop, double *Q,
               int *k_out, int want);
}

void orth(Ctx &c, const double *C, int n, int m, int ldc, double drop, double *Q, int *k_out,
          int want) {
  with_qr_fallback(c, [&]() {
    orth_impl(c, C, n, m, ldc, drop, Q, k_out, want);
    return 0;
  });
}

namespace {

void orth_impl(Ctx &c, const double *C, int n, int m, int ldc, double drop, double *Q,
               int *k_out, int want) {
  Scope sc(c.arena);
  TT_REQUIRE(m >= 1, "orth: no columns");
  if (m <= n) {
    TT_REQUIRE(m <= qr_max_cols(), "orth: too many columns");
    double *q = c.arena.dalloc((size_t)n * m), *r = c.arena.dalloc((size_t)m * m);
    tsqr(c, C, n, m, ldc, q, n, r, m);
    double *US = c.arena.dalloc((size_t)m * m), *sg = c.arena.dalloc(m);
    small_svd(c, r, m, US, sg, 1e-2 * drop);
    std::vector<double> s = to_host(c, sg, m);
    require_finite(s, "orth");
    const int k = kept_directions(s, drop, want);
    *k_out = k;
    if (k == 0) return;
    double *U = c.arena.dalloc((size_t)m * k);
    normalise_cols(c, US, sg, m, k, U);
    gemm(c, false, n, k, m, 1.0, q, n, U, m, 0.0, Q, n);
    return;
  }
  // wide: range(C) = range(R^T) where C^T = Qt Rt
  TT_REQUIRE(n <= qr_max_cols(), "orth: too many rows");
  double *Ct = c.arena.dalloc((size_t)m * n);
  transpose(c, Ct, m, C, ldc, n, m);
  double *qt = c.arena.dalloc((size_t)m * n), *rt = c.arena.dalloc((size_t)n * n);
  tsqr(c, Ct, m, n, m, qt, m, rt, n);
  double *Rt = c.arena.dalloc((size_t)n * n);
  transpose(c, Rt, n, rt, n, n, n);
  double *US = c.arena.dalloc((size_t)n * n), *sg = c.arena.dalloc(n);
  small_svd(c, Rt, n, US, sg, 1e-2 * drop);
  std::vector<double> s = to_host(c, sg, n);
  require_finite(s, "orth");
  const int k = kept_directions(s, drop, want);
  *k_out = k;
  if (k == 0) return;
  normalise_cols(c, US, sg, n, k, Q);
}

}  // namespace

namespace {

// Partial sums y_k = round(y_{k-1} + dy_k) of Algorithm 1 on a helper thread with its own
// stream: dy_k (made on the caller's stream) is handed over with an event recorded after it,
// so the sums run while the caller forms dy_{k+1}.  The operations and their operands are
// those of the one-thread loop, so the result is the same.
struct SumPipe {
  Ctx &a;
  int n1, n2, rmax;
  double eps;
  DTT ycur, ynext;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<std::pair<DTT, hipEvent_t>> q;
  bool done = false;
  int warn = 0;
  std::exception_ptr err;
  std::thread th;

  SumPipe(Ctx &aux, int n1_, int n2_, int rmax_, double eps_, int device)
      : a(aux), n1(n1_), n2(n2_), rmax(rmax_), eps(eps_) {
    const int cap = std::max(rmax, 1);
    ycur = DTT{n1, n2, 1, a.arena.dalloc((size_t)n1 * cap), a.arena.dalloc((size_t)n2 * cap)};
    ynext = DTT{n1, n2, 0, a.arena.dalloc((size_t)n1 * cap), a.arena.dalloc((size_t)n2 * cap)};
    fill_value(a, ycur.A, n1, n1, 1, 1.0);
    fill_value(a, ycur.B, n2, n2, 1, 1.0);
    th = std::thread([this, device]() {
      (void)hipSetDevice(device);
      run();
    });
  }

  // the helper context's term events, one per term of this call (made at its creation)
  size_t next_ev = 0;

  void push(const DTT &dy, hipStream_t producer) {
    TT_REQUIRE(next_ev < a.term_ev.size(), "reciprocal: more terms than the helper's events");
    hipEvent_t e = a.term_ev[next_ev++];
    HIP_CHECK(hipEventRecord(e, producer));
    {
      std::lock_guard<std::mutex> lk(mu);
      q.push_back({dy, e});
    }
    cv.notify_one();
  }

  void finish() {
    {
      std::lock_guard<std::mutex> lk(mu);
      done = true;
    }
    cv.notify_one();
    if (th.joinable()) th.join();
  }

  ~SumPipe() { finish(); }

  void run() {
    for (;;) {
      std::pair<DTT, hipEvent_t> item;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [this] { return done || !q.empty(); });
        if (q.empty()) break;
        item = q.front();
        q.pop_front();
      }
      try {
        if (!err) {
          HIP_CHECK(hipStreamWaitEvent(a.stream, item.second, 0));
          Scope sc(a.arena);
          const DTT &dy = item.first;
          const int Rs = ycur.r + dy.r;
          DTT s{n1, n2, Rs, a.arena.dalloc((size_t)n1 * Rs), a.arena.dalloc((size_t)n2 * Rs)};
          copy_scale(a, s.A, n1, ycur.A, n1, n1, ycur.r, 1.0);
          copy_scale(a, s.A + (size_t)n1 * ycur.r, n1, dy.A, n1, n1, dy.r, 1.0);
          copy_scale(a, s.B, n2, ycur.B, n2, n2, ycur.r, 1.0);
          copy_scale(a, s.B + (size_t)n2 * ycur.r, n2, dy.B, n2, n2, dy.r, 1.0);
          warn |= round_tt(a, s, eps, rmax, ynext, nullptr);
          std::swap(ycur, ynext);
        }
      } catch (...) {
        if (!err) err = std::current_exception();
      }
    }
    (void)hipStreamSynchronize(a.stream);
  }
};

}  // namespace

// Randomized range finder on a dense matrix (Halko, Martinsson and Tropp, SIAM Review 2011):
// Y = F Omega with a seeded Gaussian Omega of m = min(96, n1, n2) columns; Qa = orth(Y);
// W = F^T Qa = Qw Rw; F ~ Qa Qa^T F = Qa Rw^T Qw^T, whose SVD comes from the m x m Rw^T.
// Subspace iterations (Y = F orth(W)) continue until the discarded directions can leak at most
// 1e-13 s_0 into the kept part, as in the rounding's range finder.  The tolerance counts the
// energy outside the sketch: the kept rank k is the smallest with
// sum_{i >= k} s_i^2 + (||F||^2 - sum s^2) <= eps^2 ||F||^2, where the difference counts only
// above 1e-13 ||F||^2 (the resolution of a difference of two sums of squares).  Output gauge as the rounding's:
// A = Qa U_k (orthonormal columns), B = W U_k (carries Sigma).
int compress_dense(Ctx &c, const double *F, int n1, int n2, int ld, double eps, int rmax, DTT &y,
                   std::vector<double> *sig_out) {
  TT_REQUIRE(n1 >= 1 && n2 >= 1 && ld >= n1 && rmax >= 1 && eps >= 0.0,
             "tt_compress: bad arguments");
  Scope sc(c.arena);
  const int m = std::min(std::min(QR_MAXM, qr_max_cols()), std::min(n1, n2));
  double *cs = c.arena.dalloc(n2);
  colsumsq(c, F, n1, n2, ld, cs);
  const std::vector<double> csh = to_host(c, cs, n2);
  double total = 0.0;
  for (double v : csh) total += v;
  require_finite({total}, "compress");
  if (total == 0.0) {
    zero_tt(c, y);
    if (sig_out) sig_out->assign(1, 0.0);
    return 0;
  }
  double *Om = c.arena.dalloc((size_t)n2 * m), *Y = c.arena.dalloc((size_t)n1 * m);
  double *Qa = c.arena.dalloc((size_t)n1 * m), *W = c.arena.dalloc((size_t)n2 * m);
  double *Rt = c.arena.dalloc((size_t)m * m), *Rw = c.arena.dalloc((size_t)m * m);
  double *Qw = c.arena.dalloc((size_t)n2 * m);
  double *US = c.arena.dalloc((size_t)m * m), *sg = c.arena.dalloc(m);
  fill_gauss(c, Om, n2, m, n2, g_sketch_seed ^ ((uint64_t)n1 * 0x9E3779B97F4A7C15ull) ^
                                   ((uint64_t)n2 << 20) ^ (uint64_t)m ^ 0xC0FFEEull);
  gemm(c, false, n1, m, n2, 1.0, F, ld, Om, n2, 0.0, Y, n1);          // Y = F Omega
  const int qlim = std::max(c.power_iters, c.sketch_max_iters);
  std::vector<double> s;
  int warn = 0, k = 1;
  bool short_of_eps = false;
  for (int q = 0;; ++q) {
    tsqr(c, Y, n1, m, n1, Qa, n1, Rt, m);
    gemm(c, true, n2, m, n1, 1.0, F, ld, Qa, n1, 0.0, W, n2);          // W = F^T Qa
    tsqr(c, W, n2, m, n2, nullptr, 0, Rw, m);                          // W = Qw Rw
    jacobi_svd(c, Rw, m, US, sg, true, jacobi_floor(eps));             // SVD of Rw^T
    s = to_host(c, sg, m);
    require_finite(s, "compress");
    double captured = 0.0;
    for (double v : s) captured += v * v;
    // energy outside the sketch, counted when the difference of the two sums of squares can
    // resolve it (above 1e-13 of the total; below that the convergence test stands for it)
    const double diff = total - captured;
    const double outside = diff > 1e-13 * total ? diff : 0.0;
    const double thr = eps * eps * total;
    // smallest k whose discarded tail plus the energy outside the sketch is within eps
    std::vector<double> tail(m + 1, 0.0);
    for (int i = m - 1; i >= 0; --i) tail[i] = tail[i + 1] + s[i] * s[i];
    k = m;
    for (int kk = 1; kk <= m; ++kk)
      if (tail[kk] + outside <= thr) { k = kk; break; }
    const double fl = std::max(1e-17, jacobi_floor(eps)) * std::sqrt(captured);
    int kf = 0;
    while (kf < m && s[kf] > fl) ++kf;
    k = std::max(1, std::min(std::min(k, kf), rmax));
    // the cap or the sketch width, not eps, set k
    short_of_eps = tail[k] + outside > thr && (k == rmax || k == m);
    if (k < m && q >= c.power_iters) {
      const int pover = std::max(8, m / 4);
      if (m - pover > k && s[m - pover] <= 1e-14 * s[0]) break;
      if (std::pow(s[m - 1] / s[k - 1], 2 * q + 1) * s[k - 1] <= 1e-13 * s[0]) break;
    }
    if (k >= m && q >= c.power_iters) break;          // the sketch holds every direction kept
    if (q >= qlim) {
      warn |= TT_WSKETCH;
      c.cnt.sketch_unconverged++;
      break;
    }
    // one more subspace iteration, orthonormalising in between (Y = F (F^T Qa) directly
    // would square the spectrum and lose every direction below sqrt(u) of the largest)
    tsqr(c, W, n2, m, n2, Qw, n2, Rt, m);
    gemm(c, false, n1, m, n2, 1.0, F, ld, Qw, n2, 0.0, Y, n1);         // Y = F orth(F^T Qa)
    c.cnt.extra_power_iters++;
  }
  if (short_of_eps) warn |= TT_WRANKCAP;
  double *U = c.arena.dalloc((size_t)m * k);
  normalise_cols(c, US, sg, m, k, U);
  gemm(c, false, n1, k, m, 1.0, Qa, n1, U, m, 0.0, y.A, n1);
  gemm(c, false, n2, k, m, 1.0, W, n2, U, m, 0.0, y.B, n2);
  y.r = k;
  if (sig_out) sig_out->assign(s.begin(), s.begin() + k);
  c.cnt.warnings |= warn;
  return warn;
}

double norm_tt(Ctx &c, const DTT &x) {
  if (x.r == 0) return 0.0;
  Scope sc(c.arena);
  const int r = x.r;
  double *G = c.arena.dalloc(2 * (size_t)r * r);
  gemm(c, true, r, r, x.n1, 1.0, x.A, x.n1, x.A, x.n1, 0.0, G, r);
  gemm(c, true, r, r, x.n2, 1.0, x.B, x.n2, x.B, x.n2, 0.0, G + (size_t)r * r, r);
  std::vector<double> h = to_host(c, G, 2 * (size_t)r * r);
  double s = 0.0;
  for (size_t i = 0; i < (size_t)r * r; ++i) s += h[i] * h[(size_t)r * r + i];
  return std::sqrt(std::max(s, 0.0));
}

int reciprocal_tt(Ctx &c, const DTT &x, double eps, int K, int rmax, DTT &y, double *err_out,
                  int *terms_out, Ctx *aux) {
  TT_REQUIRE(K >= 1, "reciprocal: max_terms < 1");
  Scope sc(c.arena);
  const int n1 = x.n1, n2 = x.n2;
  const double N = (double)n1 * (double)n2;
  // x_avg = sum(x) / N, sum(x) = (1^T A)(B^T 1)
  double *cs = c.arena.dalloc(2 * (size_t)x.r);
  colsum(c, x.A, n1, x.r, n1, cs);
  colsum(c, x.B, n2, x.r, n2, cs + x.r);
  std::vector<double> h = to_host(c, cs, 2 * (size_t)x.r);
  double total = 0.0;
  for (int a = 0; a < x.r; ++a) total += h[a] * h[x.r + a];
  const double xavg = total / N;
  TT_REQUIRE(xavg != 0.0 && std::isfinite(xavg), "reciprocal: mean of x is zero or not finite");
  // x~ = round(1 - x / x_avg)
  const int cap = std::max(rmax, 1);
  DTT xt{n1, n2, 0, c.arena.dalloc((size_t)n1 * cap), c.arena.dalloc((size_t)n2 * cap)};
  {
    Scope s2(c.arena);
    DTT t{n1, n2, x.r + 1, c.arena.dalloc((size_t)n1 * (x.r + 1)),
          c.arena.dalloc((size_t)n2 * (x.r + 1))};
    fill_value(c, t.A, n1, n1, 1, 1.0);
    fill_value(c, t.B, n2, n2, 1, 1.0);
    copy_scale(c, t.A + n1, n1, x.A, n1, n1, x.r, -1.0 / xavg);
    copy_scale(c, t.B + n2, n2, x.B, n2, n2, x.r, 1.0);
    round_tt(c, t, eps, rmax, xt, nullptr);
  }
  DTT dy{n1, n2, 1, c.arena.dalloc((size_t)n1 * cap), c.arena.dalloc((size_t)n2 * cap)};
  DTT dy2{n1, n2, 0, c.arena.dalloc((size_t)n1 * cap), c.arena.dalloc((size_t)n2 * cap)};
  fill_value(c, dy.A, n1, n1, 1, 1.0);
  fill_value(c, dy.B, n2, n2, 1, 1.0);
  if (aux) {
    // the terms dy_k each keep their own buffers until the helper has added them
    int dev = 0;
    HIP_CHECK(hipGetDevice(&dev));
    Scope sa(aux->arena);
    SumPipe pipe(*aux, n1, n2, rmax, eps, dev);
    double err = 1.0, err1 = 1.0, err2 = 1.0;   // the last three term sizes
    int terms = 1, warn = 0;
    DTT prev = dy;
    while (err > eps && terms < K) {
      DTT next{n1, n2, 0, c.arena.dalloc((size_t)n1 * cap), c.arena.dalloc((size_t)n2 * cap)};
      {
        Scope s3(c.arena);
        const int R = prev.r * xt.r;
        DTT p{n1, n2, R, c.arena.dalloc((size_t)n1 * R), c.arena.dalloc((size_t)n2 * R)};
        khatri_rao(c, p.A, n1, prev.A, prev.r, xt.A, xt.r);
        khatri_rao(c, p.B, n2, prev.B, prev.r, xt.B, xt.r);
        std::vector<double> sdy;
        warn |= round_tt(c, p, eps, rmax, next, &sdy);
        double nrm2 = 0.0;
        for (double v : sdy) nrm2 += v * v;
        err2 = err1;
        err1 = err;
        err = std::sqrt(nrm2) / std::sqrt(N);
      }
      pipe.push(next, c.stream);
      prev = next;
      ++terms;
      if (terms >= 3 && err > err1 && err1 > err2) {
        pipe.finish();
        throw Error(TT_EDOMAIN, "reciprocal: the Taylor terms grow, |1 - x/mean| >= 1");
      }
    }
    pipe.finish();
    if (pipe.err) std::rethrow_exception(pipe.err);
    warn |= pipe.warn;
    copy_scale(c, y.A, n1, pipe.ycur.A, n1, n1, pipe.ycur.r, 1.0 / xavg);
    copy_scale(c, y.B, n2, pipe.ycur.B, n2, n2, pipe.ycur.r, 1.0);
    y.r = pipe.ycur.r;
    c.sync();
    if (err > eps) warn |= TT_WNOCONV;
    if (err_out) *err_out = err;
    if (terms_out) *terms_out = terms;
    c.cnt.warnings |= warn;
    return warn;
  }
  // y is accumulated in the caller's buffers; start at 1
  fill_value(c, y.A, n1, n1, 1, 1.0);
  fill_value(c, y.B, n2, n2, 1, 1.0);
  y.r = 1;
  double err = 1.0, err1 = 1.0, err2 = 1.0;   // the last three term sizes
  int terms = 1, warn = 0;
  while (err > eps && terms < K) {
    Scope s3(c.arena);
    const int R = dy.r * xt.r;
    DTT p{n1, n2, R, c.arena.dalloc((size_t)n1 * R), c.arena.dalloc((size_t)n2 * R)};
    khatri_rao(c, p.A, n1, dy.A, dy.r, xt.A, xt.r);
    khatri_rao(c, p.B, n2, dy.B, dy.r, xt.B, xt.r);
    std::vector<double> sdy;
    warn |= round_tt(c, p, eps, rmax, dy2, &sdy);
    std::swap(dy, dy2);
    const int Rs = y.r + dy.r;
    DTT s{n1, n2, Rs, c.arena.dalloc((size_t)n1 * Rs), c.arena.dalloc((size_t)n2 * Rs)};
    copy_scale(c, s.A, n1, y.A, n1, n1, y.r, 1.0);
    copy_scale(c, s.A + (size_t)n1 * y.r, n1, dy.A, n1, n1, dy.r, 1.0);
    copy_scale(c, s.B, n2, y.B, n2, n2, y.r, 1.0);
    copy_scale(c, s.B + (size_t)n2 * y.r, n2, dy.B, n2, n2, dy.r, 1.0);
    warn |= round_tt(c, s, eps, rmax, y, nullptr);
    double nrm2 = 0.0;
    for (double v : sdy) nrm2 += v * v;
    err2 = err1;
    err1 = err;
    err = std::sqrt(nrm2) / std::sqrt(N);
    ++terms;
    if (terms >= 3 && err > err1 && err1 > err2)
      throw Error(TT_EDOMAIN, "reciprocal: the Taylor terms grow, |1 - x/mean| >= 1");
  }
  copy_scale(c, y.A, n1, y.A, n1, n1, y.r, 1.0 / xavg);
  if (err > eps) warn |= TT_WNOCONV;
  if (err_out) *err_out = err;
  if (terms_out) *terms_out = terms;
  c.cnt.warnings |= warn;
  return warn;
}

std::vector<int> maxvol_host(Ctx &c, const double *Q, int n, int r, int ldq, double tau,
                             int maxit) {
  Scope sc(c.arena);
  int *rows = c.arena.ialloc(r);
  maxvol_dev(c, Q, n, r, ldq, tau, maxit, rows);
  std::vector<int> h(r);
  HIP_CHECK(hipMemcpyAsync(h.data(), rows, r * sizeof(int), hipMemcpyDeviceToHost, c.stream));
  c.sync();
  return h;
}

uint64_t splitmix64_next(uint64_t &state) { return rule_splitmix64(state); }

// seeded fresh columns outside `have_v` (rules.h: the rule the fixed-shape kernels take too)
std::vector<int> kick_indices(const std::vector<int> &have_v, int n, int count, uint64_t key) {
  std::vector<int> J;
  J.reserve(have_v.size() + std::max(count, 0));
  for (int j : have_v)
    if (std::find(J.begin(), J.end(), j) == J.end()) J.push_back(j);
  const int have = (int)J.size();
  J.resize(have + std::max(count, 0));
  const int added = count > 0 ? rule_kicks(J.data(), have, n, count, key) : 0;
  return std::vector<int>(J.begin() + have, J.begin() + have + added);
}

namespace {

// G1 = Qc Qc[I]^-1 (Qc: n1 x rc orthonormal columns, I: rc rows), G2^T = RwT, then rounding
int skeleton_round(Ctx &c, const double *Qc, int n1, int n2, int rc, const int *Id,
                   double *RwT, double eps, int rmax, DTT &y) {
  Scope sc(c.arena);
  double *QI = c.arena.dalloc((size_t)rc * rc), *QIi = c.arena.dalloc((size_t)rc * rc);
  gather_rows(c, QI, rc, Qc, n1, Id, rc, rc);
  small_inverse(c, QI, rc, rc, QIi);
  double *G1 = c.arena.dalloc((size_t)n1 * rc);
  gemm(c, false, n1, rc, rc, 1.0, Qc, n1, QIi, rc, 0.0, G1, n1);
  DTT sk{n1, n2, rc, G1, RwT};
  return round_tt(c, sk, eps, rmax, y, nullptr);
}

}  // namespace

// Residual-based column enrichment (in the spirit of AMEn's, Section 3.3): 4 x count candidate
// columns outside J drawn by the kick generator, the current skeleton's interpolant
// Qc Qc[I]^-1 f(I, j) of each (RwT = f(I, :)^T), and the count candidates with the largest
// residual norms |f(:, j) - interpolant| (ties to the earlier candidate; residuals below 1e-12
// of the largest candidate column's norm, round-off, count as ties at zero).
std::vector<int> residual_columns(Ctx &c, const FiberSpec &fs, int n1, int n2, const double *Qc,
                                  int rc, const int *Id, const double *RwT,
                                  const std::vector<int> &J, int count, uint64_t key) {
  const std::vector<int> cand =
      kick_indices(J, n2, std::min(4 * count, n2 - (int)J.size()), key);
  const int nc = (int)cand.size();
  if (nc == 0) return {};
  Scope sc(c.arena);
  int *Cd = c.arena.ialloc(nc);
  HIP_CHECK(hipMemcpyAsync(Cd, cand.data(), nc * sizeof(int), hipMemcpyHostToDevice, c.stream));
  double *Fs = c.arena.dalloc((size_t)n1 * nc);
  fiber_cols(c, fs, n1, Cd, nc, Fs);
  double *cn = c.arena.dalloc(nc);
  colsumsq(c, Fs, n1, nc, n1, cn);                                  // candidate column norms^2
  const std::vector<double> c2 = to_host(c, cn, nc);
  double *QI = c.arena.dalloc((size_t)rc * rc), *QIinv = c.arena.dalloc((size_t)rc * rc);
  gather_rows(c, QI, rc, Qc, n1, Id, rc, rc);                        // Qc[I]
  small_inverse(c, QI, rc, rc, QIinv);
  double *Rs = c.arena.dalloc((size_t)nc * rc), *T = c.arena.dalloc((size_t)rc * nc);
  gather_rows(c, Rs, nc, RwT, n2, Cd, nc, rc);                      // f(I, cand)^T
  gemm2(c, false, true, rc, nc, rc, 1.0, QIinv, rc, Rs, nc, 0.0, T, rc);
  gemm(c, false, n1, nc, rc, -1.0, Qc, n1, T, rc, 1.0, Fs, n1);       // residual columns
  double *rs = c.arena.dalloc(nc);
  colsumsq(c, Fs, n1, nc, n1, rs);
  std::vector<double> r2 = to_host(c, rs, nc);
  // residuals at round-off (below 1e-12 of the largest candidate column) are ties at zero
  const double big = *std::max_element(c2.begin(), c2.end());
  for (double &v : r2)
    if (v <= 1e-24 * big) v = 0.0;
  std::vector<int> order(nc);
  for (int t = 0; t < nc; ++t) order[t] = t;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return r2[a] > r2[b]; });
  std::vector<int> out;
  for (int t = 0; t < std::min(count, nc); ++t) out.push_back(cand[order[t]]);
  return out;
}

int cross_tt(Ctx &c, const FiberSpec &fs, int n1, int n2, std::vector<int> J, double eps,
             int rmax, int sweeps, int kick, uint64_t key, DTT &y, std::vector<int> *J_out,
             std::vector<int> *I_out) {
  TT_REQUIRE(!J.empty(), "cross: empty starting column set");
  TT_REQUIRE(sweeps >= 1, "cross: sweeps < 1");
  c.cnt.crosses++;
  Scope sc(c.arena);
  const int jcap = std::max((int)J.size(), rmax) + kick * sweeps + 1;
  const int qmax = qr_max_cols();
  TT_REQUIRE(jcap <= qmax + kick * sweeps + 1, "cross: rank too large");
  int *Jd = c.arena.ialloc(jcap);
  int *Id = c.arena.ialloc(jcap);
  double *C = c.arena.dalloc((size_t)n1 * jcap);
  double *Qc = c.arena.dalloc((size_t)n1 * jcap);
  double *RwT = c.arena.dalloc((size_t)n2 * jcap);
  double *Qr = c.arena.dalloc((size_t)n2 * jcap);
  std::vector<int> I;
  int rc = 0;
  // fiber directions below this fraction of the largest are dropped: round-off level of
  // the QR's arithmetic unless the caller sets another
  const double drop = c.drop();
  auto zero_result = [&]() {
    zero_tt(c, y);
    if (J_out) *J_out = J;
    if (I_out) I_out->clear();
    return 0;
  };
  for (int s = 0; s < sweeps; ++s) {
    TT_REQUIRE((int)J.size() <= qmax, "cross: column set exceeds the factorization width");
    HIP_CHECK(hipMemcpyAsync(Jd, J.data(), J.size() * sizeof(int), hipMemcpyHostToDevice,
                             c.stream));
    fiber_cols(c, fs, n1, Jd, (int)J.size(), C);
    orth(c, C, n1, (int)J.size(), n1, drop, Qc, &rc);
    if (rc == 0) return zero_result();
    I = maxvol_host(c, Qc, n1, rc, n1, 1.05, 100);
    HIP_CHECK(hipMemcpyAsync(Id, I.data(), I.size() * sizeof(int), hipMemcpyHostToDevice,
                             c.stream));
    fiber_rows(c, fs, n2, Id, rc, RwT);
    if (s == sweeps - 1) break;
    int rr = 0;
    orth(c, RwT, n2, rc, n2, drop, Qr, &rr);
    if (rr == 0) return zero_result();
    J = maxvol_host(c, Qr, n2, rr, n2, 1.05, 100);
    if ((int)J.size() < rmax && kick > 0) {
      const int cnt = std::min(kick, rmax - (int)J.size());
      const uint64_t k2 = key + 1000003ull * (uint64_t)(s + 1);
      const std::vector<int> extra =
          c.enrich == 1 ? residual_columns(c, fs, n1, n2, Qc, rc, Id, RwT, J, cnt, k2)
                        : kick_indices(J, n2, cnt, k2);
      J.insert(J.end(), extra.begin(), extra.end());
    }
  }
  const int w = skeleton_round(c, Qc, n1, n2, rc, Id, RwT, eps, rmax, y);
  if (J_out) *J_out = J;
  if (I_out) *I_out = I;
  return w;
}

// ---- fixed shapes: the same algorithms with every decision on the device ---------------

int fixed_status(Ctx &c) {
  TT_REQUIRE(!c.capturing, "fixed shapes: status read during graph capture");
  int h[2] = {0, 0};
  HIP_CHECK(hipMemcpyAsync(h, c.arena.status() + FX_WARN, 2 * sizeof(int),
                           hipMemcpyDeviceToHost, c.stream));
  HIP_CHECK(hipStreamSynchronize(c.stream));
  if (h[0] || h[1]) {
    const int zero[2] = {0, 0};
    HIP_CHECK(hipMemcpyAsync(c.arena.status() + FX_WARN, zero, 2 * sizeof(int),
                             hipMemcpyHostToDevice, c.stream));
    HIP_CHECK(hipStreamSynchronize(c.stream));
  }
  if (h[1] & FX_ERR_NONFINITE)
    throw Error(TT_ENONFINITE, "fixed shapes: non-finite singular value");
  if (h[1] & FX_ERR_DOMAIN)
    throw Error(TT_EDOMAIN, "reciprocal: the Taylor terms grow, |1 - x/mean| >= 1");
  if (h[1] & FX_ERR_MEAN) throw Error(TT_EINVAL, "reciprocal: mean of x is zero or not finite");
  c.cnt.warnings |= h[0];
  return h[0];
}

// The exact path and the range finder of round_tt with the kept rank chosen on the device.
// The output keeps rank kout = min(rmax, m); its columns beyond the device's k are zero.
// Without a host check of the sketch's convergence, every input of rank R <= 96 (the
// factorisation width) takes the exact path, which the dynamic path also reaches when its
// range finder does not converge; larger ranks take the range finder with a fixed number of
// subspace iterations.
int round_fixed(Ctx &c, const DTT &x, double eps, int rmax, DTT &y, int *k_dev,
                double *ss_dev) {
  TT_REQUIRE(x.r >= 1 && rmax >= 1, "round: empty input or rmax < 1");
  TT_REQUIRE(x.n1 == y.n1 && x.n2 == y.n2, "round: shape mismatch");
  c.cnt.roundings++;
  Scope sc(c.arena);
  const int n1 = x.n1, n2 = x.n2, R = x.r;
  const int qmax = qr_max_cols();
  int width = c.sketch_width > 0 ? c.sketch_width : std::min(QR_MAXM, std::max(2 * rmax, 16));
  width = std::min(width, qmax);
  const int mn = std::min(n1, n2);
  const double *Qa = nullptr, *Bsrc = nullptr, *Ra_exact = nullptr;
  double *M = nullptr;
  bool Mt = false;
  int m = 0, q_used = -1;
  if ((R <= width || (c.sketch_width <= 0 && R <= qmax)) && R <= mn) {
    m = R;
    double *qa = c.arena.dalloc((size_t)n1 * m), *ra = c.arena.dalloc((size_t)m * m);
    double *rb = c.arena.dalloc((size_t)m * m);
    tsqr(c, x.A, n1, m, n1, qa, n1, ra, m);
    tsqr(c, x.B, n2, m, n2, nullptr, 0, rb, m);
    M = c.arena.dalloc((size_t)m * m);
    gemm2(c, false, true, m, m, m, 1.0, ra, m, rb, m, 0.0, M, m);     // Ra Rb^T
    Qa = qa;
    Bsrc = x.B;
    Ra_exact = ra;
  } else {
    TT_REQUIRE(mn > width, "fixed shapes: a mode no longer than the sketch width");
    m = std::min(width, mn);
    double *Om = c.arena.dalloc((size_t)n2 * m);
    fill_gauss(c, Om, n2, m, n2,
               g_sketch_seed ^ ((uint64_t)n1 * 0x9E3779B97F4A7C15ull) ^ ((uint64_t)n2 << 20) ^
                   ((uint64_t)R << 40) ^ (uint64_t)m);
    double *T = c.arena.dalloc((size_t)R * m);
    double *Y = c.arena.dalloc((size_t)n1 * m);
    double *Z = c.arena.dalloc((size_t)n2 * m);
    double *qa = c.arena.dalloc((size_t)n1 * m), *qz = c.arena.dalloc((size_t)n2 * m);
    double *rb = c.arena.dalloc((size_t)m * m), *rtmp = c.arena.dalloc((size_t)m * m);
    gemm(c, true, R, m, n2, 1.0, x.B, n2, Om, n2, 0.0, T, R);          // B^T Omega
    gemm(c, false, n1, m, R, 1.0, x.A, n1, T, R, 0.0, Y, n1);          // Y = X Omega
    const int iters = std::max(c.power_iters, 1);
    for (int q = 0; q < iters; ++q) {
      tsqr(c, Y, n1, m, n1, qa, n1, rtmp, m);
      gemm(c, true, R, m, n1, 1.0, x.A, n1, qa, n1, 0.0, T, R);
      gemm(c, false, n2, m, R, 1.0, x.B, n2, T, R, 0.0, Z, n2);        // X^T Qy
      tsqr(c, Z, n2, m, n2, qz, n2, rtmp, m);
      gemm(c, true, R, m, n2, 1.0, x.B, n2, qz, n2, 0.0, T, R);
      gemm(c, false, n1, m, R, 1.0, x.A, n1, T, R, 0.0, Y, n1);        // Y = X Qz
    }
    tsqr(c, Y, n1, m, n1, qa, n1, rtmp, m);
    gemm(c, true, R, m, n1, 1.0, x.A, n1, qa, n1, 0.0, T, R);
    gemm(c, false, n2, m, R, 1.0, x.B, n2, T, R, 0.0, Z, n2);          // W = X^T Qa
    tsqr(c, Z, n2, m, n2, nullptr, 0, rb, m);                          // R of W only
    M = rb;
    Mt = true;
    Qa = qa;
    Bsrc = Z;
    q_used = iters;
  }
  double *US = c.arena.dalloc((size_t)m * m), *sg = c.arena.dalloc((size_t)m);
  if (Mt) jacobi_svd(c, M, m, US, sg, true, jacobi_floor(eps));
  else small_svd(c, M, m, US, sg, jacobi_floor(eps));
  const int kout = std::min(rmax, m);
  double *U = c.arena.dalloc((size_t)m * kout);
  trunc_mask(c, sg, US, m, kout, 0, eps, jacobi_floor(eps), rmax, q_used, U, k_dev, ss_dev);
  gemm(c, false, n1, kout, m, 1.0, Qa, n1, U, m, 0.0, y.A, n1);
  if (!Ra_exact) {
    gemm(c, false, n2, kout, m, 1.0, Bsrc, n2, U, m, 0.0, y.B, n2);    // W U_k
  } else {
    double *W = c.arena.dalloc((size_t)m * kout);
    gemm(c, true, m, kout, m, 1.0, Ra_exact, m, U, m, 0.0, W, m);      // Ra^T U_k
    gemm(c, false, n2, kout, m, 1.0, Bsrc, n2, W, m, 0.0, y.B, n2);
  }
  y.r = kout;
  return 0;
}

void orth_fixed(Ctx &c, const double *C, int n, int m, int ldc, double drop, double *Q,
                int *k_dev) {
  TT_REQUIRE(m >= 1 && m <= n && m <= qr_max_cols(), "orth: need 1 <= m <= min(n, 96)");
  Scope sc(c.arena);
  double *q = c.arena.dalloc((size_t)n * m), *r = c.arena.dalloc((size_t)m * m);
  tsqr(c, C, n, m, ldc, q, n, r, m);
  double *US = c.arena.dalloc((size_t)m * m), *sg = c.arena.dalloc(m);
  small_svd(c, r, m, US, sg, 1e-2 * drop);
  double *U = c.arena.dalloc((size_t)m * m);
  trunc_mask(c, sg, US, m, m, 1, drop, 0.0, m, -1, U, k_dev, nullptr);
  gemm(c, false, n, m, m, 1.0, q, n, U, m, 0.0, Q, n);
}

int cross_fixed(Ctx &c, const FiberSpec &fs, int n1, int n2, int *Jd, int *nJ, int m,
                double eps, int rmax, int sweeps, int kick, uint64_t site,
                const long long *step_dev, DTT &y, int *k_dev) {
  TT_REQUIRE(sweeps >= 1, "cross: sweeps < 1");
  TT_REQUIRE(m >= 1 && m <= qr_max_cols() && m <= n1 && m <= n2,
             "fixed shapes: cross width must be in [1, min(n1, n2, 96)]");
  c.cnt.crosses++;
  Scope sc(c.arena);
  int *Id = c.arena.ialloc(m), *kc = c.arena.ialloc(1), *kr = c.arena.ialloc(1);
  double *C = c.arena.dalloc((size_t)n1 * m), *Qc = c.arena.dalloc((size_t)n1 * m);
  double *RwT = c.arena.dalloc((size_t)n2 * m), *Qr = c.arena.dalloc((size_t)n2 * m);
  const double drop = c.drop();
  for (int s = 0; s < sweeps; ++s) {
    fiber_cols(c, fs, n1, Jd, m, C);
    mask_cols(c, C, n1, n1, m, nJ);
    orth_fixed(c, C, n1, m, n1, drop, Qc, kc);
    maxvol_dev(c, Qc, n1, m, n1, 1.05, 100, Id, kc);
    fiber_rows(c, fs, n2, Id, m, RwT);
    mask_cols(c, RwT, n2, n2, m, kc);
    if (s == sweeps - 1) break;
    orth_fixed(c, RwT, n2, m, n2, drop, Qr, kr);
    maxvol_dev(c, Qr, n2, m, n2, 1.05, 100, Jd, kr);
    device_kicks(c, Jd, nJ, kr, n2, kick, rmax, site, step_dev, s);
  }
  // skeleton: G1 = Qc Qc[I]^-1 (leading kc block; the identity outside it), G2^T = RwT
  double *QI = c.arena.dalloc((size_t)m * m), *QIi = c.arena.dalloc((size_t)m * m);
  gather_rows(c, QI, m, Qc, n1, Id, m, m);
  qi_pad(c, QI, m, kc);
  small_inverse(c, QI, m, m, QIi);
  double *G1 = c.arena.dalloc((size_t)n1 * m);
  gemm(c, false, n1, m, m, 1.0, Qc, n1, QIi, m, 0.0, G1, n1);
  DTT sk{n1, n2, m, G1, RwT};
  return round_fixed(c, sk, eps, rmax, y, k_dev);
}

int reciprocal_fixed(Ctx &c, const DTT &x, double eps, int K, int rmax, DTT &y) {
  TT_REQUIRE(K >= 1, "reciprocal: max_terms < 1");
  Scope sc(c.arena);
  const int n1 = x.n1, n2 = x.n2;
  const double N = (double)n1 * (double)n2;
  double *cs = c.arena.dalloc(2 * (size_t)x.r), *xavg = c.arena.dalloc(1);
  colsum(c, x.A, n1, x.r, n1, cs);
  colsum(c, x.B, n2, x.r, n2, cs + x.r);
  mean_dev(c, cs, x.r, N, xavg);
  const int cap = std::max(rmax, 1);
  DTT xt{n1, n2, 0, c.arena.dalloc((size_t)n1 * cap), c.arena.dalloc((size_t)n2 * cap)};
  {
    Scope s2(c.arena);
    DTT t{n1, n2, x.r + 1, c.arena.dalloc((size_t)n1 * (x.r + 1)),
          c.arena.dalloc((size_t)n2 * (x.r + 1))};
    fill_value(c, t.A, n1, n1, 1, 1.0);
    fill_value(c, t.B, n2, n2, 1, 1.0);
    scale_dev(c, t.A + n1, n1, x.A, n1, n1, x.r, xavg, -1.0, 1);      // -x / x_avg
    copy_scale(c, t.B + n2, n2, x.B, n2, n2, x.r, 1.0);
    round_fixed(c, t, eps, rmax, xt);
  }
  DTT dy{n1, n2, 1, c.arena.dalloc((size_t)n1 * cap), c.arena.dalloc((size_t)n2 * cap)};
  DTT dy2{n1, n2, 0, c.arena.dalloc((size_t)n1 * cap), c.arena.dalloc((size_t)n2 * cap)};
  fill_value(c, dy.A, n1, n1, 1, 1.0);
  fill_value(c, dy.B, n2, n2, 1, 1.0);
  fill_value(c, y.A, n1, n1, 1, 1.0);
  fill_value(c, y.B, n2, n2, 1, 1.0);
  y.r = 1;
  double *hist = c.arena.dalloc(4), *ss = c.arena.dalloc(1);
  taylor_start(c, hist);
  if (K == 1) c.cnt.warnings |= TT_WNOCONV;   // the constant term alone: Err = 1 > eps
  for (int terms = 1; terms < K; ++terms) {
    Scope s3(c.arena);
    const int R = dy.r * xt.r;
    DTT p{n1, n2, R, c.arena.dalloc((size_t)n1 * R), c.arena.dalloc((size_t)n2 * R)};
    khatri_rao(c, p.A, n1, dy.A, dy.r, xt.A, xt.r);
    khatri_rao(c, p.B, n2, dy.B, dy.r, xt.B, xt.r);
    round_fixed(c, p, eps, rmax, dy2, nullptr, ss);
    std::swap(dy, dy2);
    const int Rs = y.r + dy.r;
    DTT s{n1, n2, Rs, c.arena.dalloc((size_t)n1 * Rs), c.arena.dalloc((size_t)n2 * Rs)};
    copy_scale(c, s.A, n1, y.A, n1, n1, y.r, 1.0);
    // the term enters while the series runs (hist[3] = 1); after the stop it enters times 0
    scale_dev(c, s.A + (size_t)n1 * y.r, n1, dy.A, n1, n1, dy.r, hist + 3, 1.0, 0);
    copy_scale(c, s.B, n2, y.B, n2, n2, y.r, 1.0);
    copy_scale(c, s.B + (size_t)n2 * y.r, n2, dy.B, n2, n2, dy.r, 1.0);
    round_fixed(c, s, eps, rmax, y);
    taylor_err(c, ss, N, eps, hist, terms + 1, terms + 1 == K);
  }
  scale_dev(c, y.A, n1, y.A, n1, n1, y.r, xavg, 1.0, 1);                // y / x_avg
  return 0;
}

int skeleton_tt(Ctx &c, const FiberSpec &fs, int n1, int n2, const std::vector<int> &J,
                const std::vector<int> &I, double eps, int rmax, DTT &y) {
  TT_REQUIRE(!J.empty() && (int)J.size() <= qr_max_cols(), "skeleton: |J| must be in [1, 96]");
  for (int j : J) TT_REQUIRE(j >= 0 && j < n2, "skeleton: column index out of range");
  for (int i : I) TT_REQUIRE(i >= 0 && i < n1, "skeleton: row index out of range");
  c.cnt.crosses++;
  Scope sc(c.arena);
  const int nj = (int)J.size();
  int *Jd = c.arena.ialloc(nj);
  double *C = c.arena.dalloc((size_t)n1 * nj);
  double *Qc = c.arena.dalloc((size_t)n1 * nj);
  HIP_CHECK(hipMemcpyAsync(Jd, J.data(), nj * sizeof(int), hipMemcpyHostToDevice, c.stream));
  fiber_cols(c, fs, n1, Jd, nj, C);
  if (I.empty()) {
    zero_tt(c, y);
    return 0;
  }
  int rc = 0;
  orth(c, C, n1, nj, n1, 0.0, Qc, &rc, (int)I.size());
  int *Id = c.arena.ialloc(rc);
  HIP_CHECK(hipMemcpyAsync(Id, I.data(), rc * sizeof(int), hipMemcpyHostToDevice, c.stream));
  double *RwT = c.arena.dalloc((size_t)n2 * rc);
  fiber_rows(c, fs, n2, Id, rc, RwT);
  return skeleton_round(c, Qc, n1, n2, rc, Id, RwT, eps, rmax, y);
}

}  // namespace ttfv
