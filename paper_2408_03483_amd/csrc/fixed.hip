// Fixed-shape execution: the decisions that the dynamic path takes on the host -- a
// rounding's kept rank, an orthogonalisation's kept directions, a cross's active columns and
// rows, the Taylor series' stopping test -- taken by small kernels instead.  Every TT keeps
// the static rank of its buffer and the columns beyond the rank chosen on the device are
// zero, so each TT has the value of the dynamic path's and a step is the same sequence of
// launches with the same shapes on every call: it can be captured in a HIP graph once and
// replayed.  The rank, kept-direction and kick rules are the host code's own (rules.h); the
// reciprocal's Err test follows the host loop's order.
#include "common.h"
#include "rules.h"

#include <cmath>

namespace ttfv {
namespace {

constexpr int TB = 256;

// Kept rank k (rule 0: the rounding's; rule 1: the orthogonalisation's), then
// U(:, j) = US(:, j) / s_j for j < k and 0 for k <= j < kcap (U: m x kcap).  With q >= 0 the
// SVD came from a range finder after q subspace iterations, and TT_WSKETCH is raised when its
// stopping test does not hold.  Non-finite singular values raise the error bit and keep
// nothing.  ss_out: sum of the kept s_j^2.
__global__ __launch_bounds__(TB) void k_trunc_mask(const double *__restrict__ sg,
                                                   const double *__restrict__ US, int m,
                                                   int kcap, int rule, double eps,
                                                   double floor_rel, int rmax, int q,
                                                   double *__restrict__ U, int *k_out,
                                                   double *ss_out, int *status) {
  __shared__ double tail[130];
  __shared__ int ks;
  if (threadIdx.x == 0) {
    bool bad = false;
    for (int i = 0; i < m; ++i)
      if (!isfinite(sg[i])) bad = true;
    int k = 0;
    if (bad) {
      atomicOr(&status[FX_ERRORS], FX_ERR_NONFINITE);
    } else if (rule == 1) {
      k = rule_kept_directions(sg, m, eps);
    } else if (sg[0] != 0.0) {
      bool capped = false;
      k = rule_trunc_rank(sg, m, eps, rmax, floor_rel, tail, &capped);
      if (capped) atomicOr(&status[FX_WARN], TT_WRANKCAP);
      if (q >= 0 && k < m) {
        const int pover = max(8, m / 4);
        bool conv = m - pover > k && sg[m - pover] <= 1e-14 * sg[0];
        if (!conv) {
          const double ratio = sg[m - 1] / sg[k - 1];
          double f = ratio;
          for (int t = 0; t < 2 * q; ++t) f *= ratio;
          conv = f * sg[k - 1] <= 1e-13 * sg[0];
        }
        if (!conv) atomicOr(&status[FX_WARN], TT_WSKETCH);
      }
    }
    k = min(k, kcap);
    ks = k;
    if (k_out) *k_out = k;
    if (ss_out) {
      double s = 0.0;
      for (int j = 0; j < k; ++j) s += sg[j] * sg[j];
      *ss_out = s;
    }
  }
  __syncthreads();
  const int k = ks;
  for (int idx = threadIdx.x; idx < m * kcap; idx += TB) {
    const int c = idx / m;
    const double s = c < k ? sg[c] : 0.0;
    U[idx] = s > 0.0 ? US[idx] / s : 0.0;
  }
}

// the block of QI (m x m) outside the leading k x k one becomes the identity
__global__ void k_qi_pad(double *__restrict__ QI, int m, const int *__restrict__ kd) {
  const int idx = blockIdx.x * TB + threadIdx.x;
  if (idx >= m * m) return;
  const int a = idx % m, b = idx / m, k = *kd;
  if (a >= k || b >= k) QI[idx] = a == b ? 1.0 : 0.0;
}

// zero columns k.. of X (rows x m, ld)
__global__ void k_mask_cols(double *__restrict__ X, int ld, int rows, const int *__restrict__ kd) {
  const int i = blockIdx.x * TB + threadIdx.x, c = blockIdx.y;
  if (i >= rows || c < *kd) return;
  X[(size_t)c * ld + i] = 0.0;
}

// nJ = *src, then the seeded fresh columns of a non-final sweep (rules.h, with the key
// (site << 32 | step) + 1000003 (sweep + 1) of the host's crosses) appended while nJ < rmax
__global__ void k_kicks(int *__restrict__ J, int *__restrict__ nJ, const int *__restrict__ src,
                        int n, int kick, int rmax, unsigned long long site,
                        const long long *__restrict__ step, int sweep) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int have = *src;
  int added = 0;
  if (have < rmax && kick > 0) {
    const uint64_t key = ((site << 32) | ((uint64_t)*step & 0xFFFFFFFFull)) +
                         1000003ull * (uint64_t)(sweep + 1);
    added = rule_kicks(J, have, n, min(kick, rmax - have), key);
  }
  *nJ = have + added;
}

// dst = alpha src with alpha = mul * s[0] (mode 0) or mul / s[0] (mode 1)
__global__ void k_scale_dev(double *__restrict__ dst, int ldd, const double *src, int lds,
                            int rows, const double *__restrict__ s, double mul, int mode) {
  const int i = blockIdx.x * TB + threadIdx.x, c = blockIdx.y;
  if (i >= rows) return;
  const double alpha = mode == 0 ? mul * s[0] : mul / s[0];
  dst[(size_t)c * ldd + i] = alpha * src[(size_t)c * lds + i];
}

// out = (sum_a cs[a] cs[r + a]) / N: the mean of a TT from its core column sums
__global__ void k_mean(const double *__restrict__ cs, int r, double N, double *__restrict__ out,
                       int *status) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double total = 0.0;
  for (int a = 0; a < r; ++a) total += cs[a] * cs[r + a];
  const double m = total / N;
  if (m == 0.0 || !isfinite(m)) atomicOr(&status[FX_ERRORS], FX_ERR_MEAN);
  out[0] = m;
}

// Taylor reciprocal, after the term of index `terms - 1` (hist: err, err1, err2, active):
// while active, Err = sqrt(sum s^2) / sqrt(N) of the term, the growth test, and the term is
// the last one added when Err <= eps
__global__ void k_taylor_err(const double *__restrict__ ss, double N, double eps,
                             double *__restrict__ hist, int terms, int last, int *status) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (hist[3] == 0.0) return;
  hist[2] = hist[1];
  hist[1] = hist[0];
  hist[0] = sqrt(ss[0]) / sqrt(N);
  if (terms >= 3 && hist[0] > hist[1] && hist[1] > hist[2])
    atomicOr(&status[FX_ERRORS], FX_ERR_DOMAIN);
  if (hist[0] <= eps) hist[3] = 0.0;
  else if (last) atomicOr(&status[FX_WARN], TT_WNOCONV);
}

__global__ void k_fill4(double *__restrict__ d, double a, double b, double c, double e) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    d[0] = a;
    d[1] = b;
    d[2] = c;
    d[3] = e;
  }
}

__global__ void k_inc_step(long long *step) {
  if (threadIdx.x == 0 && blockIdx.x == 0) step[0] += 1;
}

// leading nonzero columns of B (n x r): the rank a fixed-shape TT carries
__global__ __launch_bounds__(TB) void k_count_rank(const double *__restrict__ B, int n, int r,
                                                   int *__restrict__ out) {
  __shared__ int last;
  if (threadIdx.x == 0) last = 0;
  __syncthreads();
  for (int c = 0; c < r; ++c)
    for (int i = threadIdx.x; i < n; i += TB)
      if (B[(size_t)c * n + i] != 0.0) atomicMax(&last, c + 1);
  __syncthreads();
  if (threadIdx.x == 0) out[0] = last;
}

dim3 grid2f(int rows, int cols) { return dim3((rows + TB - 1) / TB, cols); }

}  // namespace

void trunc_mask(Ctx &c, const double *sg, const double *US, int m, int kcap, int rule,
                double eps, double floor_rel, int rmax, int q, double *U, int *k_out,
                double *ss_out) {
  TT_REQUIRE(m >= 1 && m <= 128 && kcap >= 1 && kcap <= m, "trunc_mask: bad sizes");
  hipLaunchKernelGGL(k_trunc_mask, dim3(1), dim3(TB), 0, c.stream, sg, US, m, kcap, rule, eps,
                     floor_rel, rmax, q, U, k_out, ss_out, c.arena.status());
}

void qi_pad(Ctx &c, double *QI, int m, const int *k_dev) {
  hipLaunchKernelGGL(k_qi_pad, dim3((m * m + TB - 1) / TB), dim3(TB), 0, c.stream, QI, m, k_dev);
}

void mask_cols(Ctx &c, double *X, int ld, int rows, int m, const int *k_dev) {
  if (rows <= 0 || m <= 0) return;
  hipLaunchKernelGGL(k_mask_cols, grid2f(rows, m), dim3(TB), 0, c.stream, X, ld, rows, k_dev);
}

void device_kicks(Ctx &c, int *J, int *nJ, const int *src, int n, int kick, int rmax,
                  uint64_t site, const long long *step_dev, int sweep) {
  hipLaunchKernelGGL(k_kicks, dim3(1), dim3(64), 0, c.stream, J, nJ, src, n, kick, rmax,
                     (unsigned long long)site, step_dev, sweep);
}

void scale_dev(Ctx &c, double *dst, int ldd, const double *src, int lds, int rows, int cols,
               const double *s, double mul, int mode) {
  if (rows <= 0 || cols <= 0) return;
  hipLaunchKernelGGL(k_scale_dev, grid2f(rows, cols), dim3(TB), 0, c.stream, dst, ldd, src, lds,
                     rows, s, mul, mode);
}

void mean_dev(Ctx &c, const double *cs, int r, double N, double *out) {
  hipLaunchKernelGGL(k_mean, dim3(1), dim3(64), 0, c.stream, cs, r, N, out, c.arena.status());
}

void taylor_start(Ctx &c, double *hist) {
  hipLaunchKernelGGL(k_fill4, dim3(1), dim3(64), 0, c.stream, hist, 1.0, 1.0, 1.0, 1.0);
}

void taylor_err(Ctx &c, const double *ss, double N, double eps, double *hist, int terms,
                bool last) {
  hipLaunchKernelGGL(k_taylor_err, dim3(1), dim3(64), 0, c.stream, ss, N, eps, hist, terms,
                     last ? 1 : 0, c.arena.status());
}

void inc_step(Ctx &c, long long *step) {
  hipLaunchKernelGGL(k_inc_step, dim3(1), dim3(64), 0, c.stream, step);
}

void count_rank(Ctx &c, const double *B, int n, int r, int *out) {
  hipLaunchKernelGGL(k_count_rank, dim3(1), dim3(TB), 0, c.stream, B, n, r, out);
}

}  // namespace ttfv
