// Rounding of a d-core tensor train (Section 3.1's TT definition, Section 3.2's rounding
// extended to d cores: the TT-SVD of Oseledets 2011), on the library's two-core primitives.
//
// Core k is r_k x n_k x r_{k+1} with the left rank index fastest, so its left unfolding
// ((r_k n_k) x r_{k+1}) and its right unfolding (r_k x (n_k r_{k+1})) are both column-major
// views of the same memory.
//   1. right-to-left orthogonalisation, k = d-1 .. 1: the right unfolding R_k = L Q^T with
//      Q^T's rows orthonormal, by a tall-skinny QR of R_k^T (or, when R_k has more rows than
//      columns, L = R_k and Q = I, which lowers the rank to n_k r_{k+1}); core k <- Q^T,
//      core k-1's left unfolding <- itself times L;
//   2. left-to-right truncation, k = 0 .. d-2: the two-core TT (core k's left unfolding,
//      core k+1's right unfolding transposed) is rounded by round_tt to the absolute accuracy
//      delta = eps / sqrt(d - 1) ||X|| (its relative tolerance delta / ||core k||, since the
//      cores around it are orthonormal) and rank <= rmax; its orthonormal left factor becomes
//      core k, its right factor (carrying Sigma) the right unfolding of core k+1.
#include "common.h"

#include <cmath>

namespace ttfv {

namespace {

double core_norm(Ctx &c, const double *G, int rows, int cols) {
  Scope sc(c.arena);
  double *cs = c.arena.dalloc(cols);
  colsumsq(c, G, rows, cols, rows, cs);
  std::vector<double> h(cols);
  HIP_CHECK(hipMemcpyAsync(h.data(), cs, cols * sizeof(double), hipMemcpyDeviceToHost,
                           c.stream));
  c.sync();
  double s = 0.0;
  for (double v : h) s += v;
  return std::sqrt(s);
}

}  // namespace

// in: d cores (device), modes n[d], ranks r[d + 1]; out: cores written into out[k] (room for
// rmax * n_k * rmax doubles each), ranks into r_out; kept singular values of every bond
// appended to sig (when not null).  Returns TT_W* bits.
int round_nd(Ctx &c, int d, const int *n, const int *r, const double *const *in, double eps,
             int rmax, double *const *out, int *r_out, std::vector<double> *sig) {
  TT_REQUIRE(d >= 2, "tt_round_nd: d must be >= 2");
  TT_REQUIRE(r[0] == 1 && r[d] == 1, "tt_round_nd: boundary ranks must be 1");
  for (int k = 0; k < d; ++k)
    TT_REQUIRE(n[k] >= 1 && r[k] >= 1 && r[k] <= QR_MAXM && r[k + 1] >= 1,
               "tt_round_nd: modes >= 1, ranks in [1, 96]");
  Scope sc(c.arena);
  std::vector<int> rk(r, r + d + 1);
  // work copies, each with room for its input size
  std::vector<double *> G(d);
  std::vector<size_t> room(d);
  for (int k = 0; k < d; ++k) {
    room[k] = (size_t)rk[k] * n[k] * rk[k + 1];
    G[k] = c.arena.dalloc(std::max(room[k], (size_t)1));
    copy_scale(c, G[k], rk[k] * n[k], in[k], rk[k] * n[k], rk[k] * n[k], rk[k + 1], 1.0);
  }
  // 1. right-to-left orthogonalisation
  for (int k = d - 1; k >= 1; --k) {
    Scope s2(c.arena);
    const int r0 = rk[k], m = n[k] * rk[k + 1];
    const int p = rk[k - 1] * n[k - 1];          // rows of core k-1's left unfolding
    double *T = c.arena.dalloc((size_t)m * r0);
    double *P = c.arena.dalloc((size_t)p * std::max(r0, m));
    if (m >= r0) {
      transpose(c, T, m, G[k], r0, r0, m);                                  // R_k^T (m x r0)
      double *Q = c.arena.dalloc((size_t)m * r0), *R = c.arena.dalloc((size_t)r0 * r0);
      tsqr(c, T, m, r0, m, Q, m, R, r0);
      transpose(c, G[k], r0, Q, m, m, r0);                                  // core k = Q^T
      gemm2(c, false, true, p, r0, r0, 1.0, G[k - 1], p, R, r0, 0.0, P, p);  // L = R^T
      copy_scale(c, G[k - 1], p, P, p, p, r0, 1.0);
    } else {
      // L = R_k (r0 x m), Q = I: core k-1 absorbs core k, whose rank drops to m
      gemm(c, false, p, m, r0, 1.0, G[k - 1], p, G[k], r0, 0.0, P, p);
      copy_scale(c, G[k - 1], p, P, p, p, m, 1.0);
      fill_value(c, G[k], m, m, m, 0.0);
      std::vector<double> eye((size_t)m * m, 0.0);
      for (int i = 0; i < m; ++i) eye[(size_t)i * m + i] = 1.0;
      HIP_CHECK(hipMemcpyAsync(G[k], eye.data(), eye.size() * sizeof(double),
                               hipMemcpyHostToDevice, c.stream));
      c.sync();
      rk[k] = m;
    }
  }
  const double total = core_norm(c, G[0], n[0], rk[1]);
  int warn = 0;
  if (!(total > 0.0)) {
    TT_REQUIRE(total == 0.0, "tt_round_nd: non-finite norm");
    for (int k = 0; k < d; ++k) {
      fill_value(c, out[k], n[k], n[k], 1, 0.0);
      r_out[k] = 1;
      if (sig && k < d - 1) sig->push_back(0.0);
    }
    r_out[d] = 1;
    return 0;
  }
  const double delta = eps / std::sqrt((double)(d - 1)) * total;
  // 2. left-to-right truncation through two-core roundings
  for (int k = 0; k + 1 < d; ++k) {
    Scope s2(c.arena);
    const int rows = rk[k] * n[k], r1 = rk[k + 1], m2 = n[k + 1] * rk[k + 2];
    double *Bt = c.arena.dalloc((size_t)m2 * r1);
    transpose(c, Bt, m2, G[k + 1], r1, r1, m2);                             // R_{k+1}^T
    const double nk = core_norm(c, G[k], rows, r1);
    DTT x{rows, m2, r1, G[k], Bt};
    const int cap = std::min(rmax, std::min(rows, std::max(r1, 1)));
    DTT y{rows, m2, 0, c.arena.dalloc((size_t)rows * std::max(cap, 1)),
          c.arena.dalloc((size_t)m2 * std::max(cap, 1))};
    std::vector<double> s;
    warn |= round_tt(c, x, nk > 0.0 ? delta / nk : 0.0, cap, y, &s);
    if (sig) sig->insert(sig->end(), s.begin(), s.end());
    const int kept = y.r;
    copy_scale(c, G[k], rows, y.A, rows, rows, kept, 1.0);                  // core k
    transpose(c, G[k + 1], kept, y.B, m2, m2, kept);                        // core k+1
    rk[k + 1] = kept;
  }
  for (int k = 0; k < d; ++k) {
    TT_REQUIRE(rk[k] <= rmax && rk[k + 1] <= rmax, "tt_round_nd: output rank above r_max");
    copy_scale(c, out[k], rk[k] * n[k], G[k], rk[k] * n[k], rk[k] * n[k], rk[k + 1], 1.0);
  }
  for (int k = 0; k <= d; ++k) r_out[k] = rk[k];
  c.sync();
  return warn;
}

}  // namespace ttfv
