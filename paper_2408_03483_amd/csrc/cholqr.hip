// Tall-skinny QR on the matrix cores by repeated Cholesky QR: for Y (n x m, m <= 96),
// Q_0 = Y, and pass p forms the Gram matrix G_p = Q_p^T Q_p, factors it G_p (+ s I) = R^T R
// (Cholesky), and multiplies Q_{p+1} = Q_p R^{-1}, until the columns are orthonormal.  The
// first passes add the diagonal shift s = 11 (m n + m (m + 1)) u tr(G) of shifted Cholesky
// QR (Fukaya, Kannan, Nakatsukasa, Zhang and Yamamoto 2020), which keeps the factorisation
// defined for any condition number and brings the columns close to orthonormal; unshifted
// passes then finish the orthogonalisation to round-off.  In an unshifted pass a pivot at or
// below 1e-18 of the trace marks its column null: the column has no direction the earlier
// columns lack, only round-off, so it is set to zero and its row of R is zero.  Exactly
// rank-deficient inputs (zero or repeated columns, Khatri-Rao cores of symmetric products,
// sketches of low-rank matrices) thus end with columns that are orthonormal or zero, and
// rows of R that are zero where the column is.  R is the product of the pass factors.
//
// Two launches per pass, with the kernel boundary as the only synchronisation between blocks
// (a device-scope fence inside a kernel writes back and invalidates the whole L2 on this
// chip, which measured slower than the launch it saves):
//   * slab kernel, at most 32 blocks of 64-row chunks: from pass 1 on the chunk of Q_{p-1}
//     times the multiplier W = R^{-1} of the previous pass (MFMA 16x16x4 FP64), written to Q
//     (in place from pass 2 on); every pass the chunks' Gram blocks (upper 16x16 blocks, MFMA,
//     accumulated in registers) as one partial per block;
//   * factor kernel, one block: the partials summed in block order (the result does not
//     depend on scheduling), then either convergence (|G - I| small: R out, done) or a
//     blocked Cholesky of G (16x16 diagonal blocks in one wavefront, panel and trailing
//     updates on the matrix cores), its inverse by block rows, W and the running R.
// The host launches a fixed number of passes; passes after convergence return at once.  When
// the last pass ends without orthonormal columns (measured on the CPU emulation of these
// passes: at most five are needed for condition numbers up to 1e30 and for the
// rank-deficient cases above) the arena's status word [1] is incremented and Q and R are set
// to NaN, so the caller's finiteness check redoes the operation with Householder QR.
#include "common.h"

#include <algorithm>
#include <cmath>

namespace ttfv {
namespace {

constexpr int CQ_NT = 256;     // 4 wavefronts
constexpr int CQ_RB = 64;      // rows of Y per block
constexpr int CQ_MAXB = 32;    // slab blocks per pass at most
constexpr double CQ_U = 1.1102230246251565e-16;   // unit round-off of FP64

typedef double v4d __attribute__((ext_vector_type(4)));

// 16x16x4 FP64 matrix-core step: lane l supplies A(l % 16, l / 16) and B(l / 16, l % 16);
// accumulator element v of lane l is D(l / 16 + 4 v, l % 16)
__device__ __forceinline__ v4d mma(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// value of lane `src` (uniform) in every lane
__device__ __forceinline__ double bcast(double x, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), src);
  return __hiloint2double(hi, lo);
}

// upper 16x16 blocks (a <= c) of a T x T block matrix, numbered row by row
template <int T>
__device__ __forceinline__ void upper_tile(int t, int &a, int &c) {
  a = 0;
  int w = T;
  while (t >= w) {
    t -= w;
    ++a;
    --w;
  }
  c = a + t;
}
// lower 16x16 blocks (t >= u) of the trailing part below block column k, numbered row by row
__device__ __forceinline__ void lower_pair(int q, int k, int &t, int &u) {
  t = k + 1;
  while (q >= t - k) {
    q -= t - k;
    ++t;
  }
  u = k + 1 + q;
}


template <int MP>
constexpr size_t cq_factor_lds_doubles() {
  return (size_t)2 * MP * (MP + 1);
}

// Slab kernel of one pass: block b takes `rpb` rows (in chunks of 64): pass >= 1 multiplies
// them by W and writes them to Q; every pass accumulates the chunks' Gram blocks (upper 16x16
// blocks, in registers) and writes the block's partial sums.  No cross-block traffic: the
// factor kernel launched next on the stream reads the partials.
template <int MP>
__global__ __launch_bounds__(CQ_NT) void k_cqr_slab(
    int n, int m, int pass, int rpb, const double *src, int ld_src, double *dst, int ld_dst,
    const double *__restrict__ Wg, double *__restrict__ part, const int *__restrict__ flags) {
  constexpr int T = MP / 16;
  constexpr int NTILE = T * (T + 1) / 2;
  constexpr int TPW = (NTILE + 3) / 4;   // Gram blocks per wavefront
  constexpr int LD = MP + 1;
  constexpr int SLD = CQ_RB + 1;
  extern __shared__ double lds[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  if (pass > 0 && (flags[0] | flags[1])) return;   // converged or given up in an earlier pass
  const int b = blockIdx.x;
  const int rbeg = b * rpb, rend = min(n, rbeg + rpb);
  double *S = lds;                     // 64 x MP chunk, ld SLD
  double *Ws = lds + (size_t)SLD * MP; // MP x MP, ld LD
  if (pass > 0)
    for (int e = tid; e < MP * MP; e += CQ_NT) Ws[(e % MP) + (e / MP) * LD] = Wg[e];
  v4d gacc[TPW];
#pragma unroll
  for (int q = 0; q < TPW; ++q) gacc[q] = v4d{0, 0, 0, 0};
  for (int r0 = rbeg; r0 < rend; r0 += CQ_RB) {
    const int rows = min(CQ_RB, rend - r0);
    for (int e = tid; e < CQ_RB * MP; e += CQ_NT) {
      const int r = e % CQ_RB, c = e / CQ_RB;
      double v = 0.0;
      if (r < rows && c < m) v = src[(size_t)(r0 + r) + (size_t)c * ld_src];
      S[r + c * SLD] = v;
    }
    __syncthreads();
    if (pass > 0) {
      v4d acc[T];
#pragma unroll
      for (int c = 0; c < T; ++c) acc[c] = v4d{0, 0, 0, 0};
      for (int k = 0; k < MP; k += 4) {
        const double a = S[(16 * wave + li) + (k + lk) * SLD];
#pragma unroll
        for (int c = 0; c < T; ++c) acc[c] = mma(a, Ws[(k + lk) + (16 * c + li) * LD], acc[c]);
      }
      __syncthreads();                 // every wave has read S
#pragma unroll
      for (int c = 0; c < T; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          S[(16 * wave + lk + 4 * v) + (16 * c + li) * SLD] = acc[c][v];
      __syncthreads();
      for (int e = tid; e < CQ_RB * MP; e += CQ_NT) {
        const int r = e % CQ_RB, c = e / CQ_RB;
        if (r < rows && c < m) dst[(size_t)(r0 + r) + (size_t)c * ld_dst] = S[r + c * SLD];
      }
    }
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
      const int t = wave + 4 * q;
      if (t >= NTILE) break;
      int a, c;
      upper_tile<T>(t, a, c);
      for (int k = 0; k < CQ_RB; k += 4)
        gacc[q] = mma(S[(k + lk) + (16 * a + li) * SLD], S[(k + lk) + (16 * c + li) * SLD],
                      gacc[q]);
    }
    __syncthreads();                   // before the next chunk overwrites S
  }
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
    const int t = wave + 4 * q;
    if (t >= NTILE) break;
    double *p = part + ((size_t)b * NTILE + t) * 256;
#pragma unroll
    for (int v = 0; v < 4; ++v) p[v * 64 + lane] = gacc[q][v];
  }
}

// Factor kernel of one pass (one block): G = the sum of the nb partials in block order, then
// the convergence check, or the Cholesky factor, its inverse, W and the running R.
template <int MP>
__global__ __launch_bounds__(CQ_NT) void k_cqr_factor(
    int n, int m, int pass, int last, int nb, double *__restrict__ Wg, double *__restrict__ Racc,
    const double *__restrict__ part, int *__restrict__ flags, int *__restrict__ fail_count,
    double *__restrict__ dst, int ld_dst, double *__restrict__ R, int ldr) {
  constexpr int T = MP / 16;
  constexpr int NTILE = T * (T + 1) / 2;
  constexpr int LD = MP + 1;
  extern __shared__ double lds[];
  __shared__ int s_bad, s_far;
  __shared__ double s_tr;
  __shared__ int s_null[MP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  if (pass > 0 && (flags[0] | flags[1])) return;

  // ---- the last block: G in LDS (full symmetric) ------------------------------------------
  double *G = lds;                     // MP x MP, ld LD: G, then L (lower) in place
  double *X = lds + (size_t)MP * LD;   // MP x MP, ld LD: L^{-1} (lower)
  {
    // thread tid owns elements tid + 256 t of every partial (t = its Gram block); the
    // partials are added in block order, QB of them loaded per round for all its elements
    constexpr int QB = NTILE <= 10 ? 4 : 2;
    double acc[NTILE];
#pragma unroll
    for (int t = 0; t < NTILE; ++t) acc[t] = 0.0;
    for (int q0 = 0; q0 < nb; q0 += QB) {
      double x[QB][NTILE];
#pragma unroll
      for (int u = 0; u < QB; ++u)
#pragma unroll
        for (int t = 0; t < NTILE; ++t)
          x[u][t] = q0 + u < nb ? part[((size_t)(q0 + u) * NTILE + t) * 256 + tid] : 0.0;
#pragma unroll
      for (int u = 0; u < QB; ++u)
#pragma unroll
        for (int t = 0; t < NTILE; ++t) acc[t] += x[u][t];
    }
    const int l = tid & 63, v = tid >> 6;
#pragma unroll
    for (int t = 0; t < NTILE; ++t) {
      int a, c;
      upper_tile<T>(t, a, c);
      const int i = 16 * a + (l >> 4) + 4 * v, j = 16 * c + (l & 15);
      G[i + j * LD] = acc[t];
      G[j + i * LD] = acc[t];
    }
  }
  if (tid == 0) {
    s_bad = 0;
    s_far = 0;
  }
  __syncthreads();
  if (tid == 0) {
    double tr = 0.0;
    for (int j = 0; j < m; ++j) tr += G[j + j * LD];
    s_tr = tr;
  }
  if (pass > 0) {
    // converged when the unit columns are orthonormal and the others are zero
    const double tol = 4.0 * m * CQ_U;
    int bad = 0, far = 0;
    for (int e = tid; e < m * m; e += CQ_NT) {
      const int i = e % m, j = e / m;
      if (i > j) continue;
      const double want = (i == j && G[j + j * LD] >= 0.5) ? 1.0 : 0.0;
      const double dv = fabs(G[i + j * LD] - want);
      if (!(dv <= tol)) bad = 1;       // a NaN counts as not converged
      if (!(dv <= 0.1)) far = 1;
    }
    if (bad) s_bad = 1;
    if (far) s_far = 1;
    __syncthreads();
    const double *Rp = Racc + (size_t)((pass - 1) & 1) * MP * MP;   // Y = Q_pass Rp
    if (!s_bad || pass == last) {
      const bool ok = !s_bad;
      if (ok) {
        for (int e = tid; e < m * m; e += CQ_NT) {
          const int i = e % m, j = e / m;
          const bool keep = i <= j && G[i + i * LD] >= 0.5;
          R[i + (size_t)j * ldr] = keep ? Rp[i + (size_t)j * MP] : 0.0;
        }
      } else {
        // not orthonormal after the last pass: Q and R become NaN, which the caller's
        // finiteness check of the singular values catches (it then uses Householder QR)
        const double qnan = __builtin_nan("");
        for (size_t e = tid; e < (size_t)n * m; e += CQ_NT)
          dst[(e % n) + (e / n) * (size_t)ld_dst] = qnan;
        for (int e = tid; e < m * m; e += CQ_NT) R[(e % m) + (size_t)(e / m) * ldr] = qnan;
      }
      if (tid == 0) {
        if (ok) {
          flags[0] = 1;
        } else {
          flags[1] = 1;
          atomicAdd(fail_count, 1);
        }
      }
      return;
    }
  }
  __syncthreads();
  const double tr = s_tr;
  const bool shifted = pass == 0 || (pass == 1 && s_far);
  const double shift = shifted ? 11.0 * ((double)m * n + (double)m * (m + 1)) * CQ_U * tr : 0.0;
  // a pivot at or below `guard` is a column with no new direction (in an unshifted pass the
  // columns are near unit norm, and 1e-18 of the trace separates real directions, which the
  // shifted passes have scaled up, from the round-off left in dependent columns)
  const double guard = (shifted ? 1e-30 : 1e-18) * tr;
  if (shift > 0.0)
    for (int j = tid; j < m; j += CQ_NT) G[j + j * LD] += shift;
  __syncthreads();

  // ---- blocked Cholesky G = L L^T (lower, in place) and the inverses of its diagonal blocks
  for (int bk = 0; bk < T; ++bk) {
    const int o = 16 * bk;
    if (wave == 0) {
      const int r = lane & 15;
      double a[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) a[c] = G[(o + r) + (o + c) * LD];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const double d = bcast(a[j], j);
        const bool nul = d <= guard;
        const double ljj = nul ? 1.0 : sqrt(d);
        const double inv = 1.0 / ljj;
        a[j] = r > j ? (nul ? 0.0 : a[j] * inv) : (r == j ? ljj : 0.0);
        if (lane == 0) s_null[o + j] = nul;
#pragma unroll
        for (int k = j + 1; k < 16; ++k) {
          const double lkj = bcast(a[j], k);
          if (r >= k) a[k] -= a[j] * lkj;
        }
      }
      if (lane < 16)
#pragma unroll
        for (int c = 0; c < 16; ++c) G[(o + r) + (o + c) * LD] = a[c];
      // column r of the inverse of the diagonal block, by forward substitution
      double x[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        double s = i == r ? 1.0 : 0.0;
#pragma unroll
        for (int k = 0; k < i; ++k) s -= bcast(a[k], i) * x[k];
        x[i] = s / bcast(a[i], i);
      }
      if (lane < 16)
#pragma unroll
        for (int i = 0; i < 16; ++i) X[(o + i) + (o + r) * LD] = x[i];
    }
    __syncthreads();
    // panel below the diagonal block: L(t, bk) = G(t, bk) X(bk, bk)^T, null columns zero
    for (int t = bk + 1 + wave; t < T; t += 4) {
      v4d acc = v4d{0, 0, 0, 0};
#pragma unroll
      for (int k = 0; k < 16; k += 4)
        acc = mma(G[(16 * t + li) + (o + k + lk) * LD], X[(o + li) + (o + k + lk) * LD], acc);
#pragma unroll
      for (int v = 0; v < 4; ++v)
        G[(16 * t + lk + 4 * v) + (o + li) * LD] = s_null[o + li] ? 0.0 : acc[v];
    }
    __syncthreads();
    // trailing update of the lower blocks (t, u), bk < u <= t: G(t, u) -= L(t, bk) L(u, bk)^T
    const int tr_n = T - bk - 1, npairs = tr_n * (tr_n + 1) / 2;
    for (int q = wave; q < npairs; q += 4) {
      int t, u;
      lower_pair(q, bk, t, u);
      v4d acc = v4d{0, 0, 0, 0};
#pragma unroll
      for (int k = 0; k < 16; k += 4)
        acc = mma(G[(16 * t + li) + (o + k + lk) * LD], G[(16 * u + li) + (o + k + lk) * LD],
                  acc);
#pragma unroll
      for (int v = 0; v < 4; ++v) G[(16 * t + lk + 4 * v) + (16 * u + li) * LD] -= acc[v];
    }
    __syncthreads();
  }

  // ---- L^{-1} below the diagonal, one block row at a time:
  //      X(I, c) = -X(I, I) sum_{c <= k < I} L(I, k) X(k, c)
  for (int I = 1; I < T; ++I) {
    for (int c = wave; c < I; c += 4) {
      v4d s = v4d{0, 0, 0, 0};
      for (int kb = c; kb < I; ++kb)
#pragma unroll
        for (int k = 0; k < 16; k += 4)
          s = mma(G[(16 * I + li) + (16 * kb + k + lk) * LD],
                  X[(16 * kb + k + lk) + (16 * c + li) * LD], s);
      // the accumulator layout is the B operand layout of the next product
      v4d x = v4d{0, 0, 0, 0};
#pragma unroll
      for (int q = 0; q < 4; ++q) x = mma(X[(16 * I + li) + (16 * I + 4 * q + lk) * LD], s[q], x);
#pragma unroll
      for (int v = 0; v < 4; ++v) X[(16 * I + lk + 4 * v) + (16 * c + li) * LD] = -x[v];
    }
    __syncthreads();
  }

  // ---- W = R^{-1} = (L^{-1})^T (upper) for the next pass; running R = L^T R_prev.  A null
  //      column gets a zero column of W and a zero row of R: it becomes exactly zero in the
  //      next pass and drops out of Y = Q R (its part is at the round-off of the pass)
  for (int e = tid; e < MP * MP; e += CQ_NT) {
    const int i = e % MP, j = e / MP;
    Wg[e] = (i <= j && !s_null[j]) ? X[j + i * LD] : 0.0;
  }
  double *Rn = Racc + (size_t)(pass & 1) * MP * MP;
  const double *Ro = Racc + (size_t)((pass + 1) & 1) * MP * MP;
  for (int t = wave; t < T * T; t += 4) {
    const int a = t % T, c = t / T;            // block (a, c) of the new R
    v4d acc = v4d{0, 0, 0, 0};
    if (a <= c) {
      if (pass == 0) {
#pragma unroll
        for (int v = 0; v < 4; ++v)
          acc[v] = G[(16 * c + li) + (16 * a + lk + 4 * v) * LD];   // L(c, a)^T
      } else {
        for (int kb = a; kb <= c; ++kb)
#pragma unroll
          for (int k = 0; k < 16; k += 4)
            acc = mma(G[(16 * kb + k + lk) + (16 * a + li) * LD],
                      Ro[(16 * kb + k + lk) + (size_t)(16 * c + li) * MP], acc);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 16 * a + lk + 4 * v, j = 16 * c + li;
      Rn[i + (size_t)j * MP] = (i <= j && !s_null[i]) ? acc[v] : 0.0;
    }
  }
  if (pass == 0 && tid == 0) {
    flags[0] = 0;
    flags[1] = 0;
  }
}

// rows per slab block: four chunks of 64, and at most CQ_MAXB blocks (the factor kernel
// reads one partial Gram matrix per block, so fewer blocks shorten its serial part)
int slab_rows(int n) {
  const int nb = std::max(1, std::min(CQ_MAXB, (n + 4 * CQ_RB - 1) / (4 * CQ_RB)));
  const int per = (n + nb - 1) / nb;
  return (per + CQ_RB - 1) / CQ_RB * CQ_RB;
}

template <int MP>
void launch_passes(Ctx &c, const double *Y, int n, int m, int ldy, double *Qb, int ldq,
                   double *R, int ldr) {
  constexpr int T = MP / 16, NTILE = T * (T + 1) / 2;
  const int rpb = slab_rows(n), nb = (n + rpb - 1) / rpb;
  double *W = c.arena.dalloc((size_t)MP * MP);
  double *Racc = c.arena.dalloc((size_t)2 * MP * MP);
  double *part = c.arena.dalloc((size_t)nb * NTILE * 256);
  int *flags = c.arena.ialloc(2);
  int *fails = c.arena.status() + 1;
  const size_t lds_s = ((size_t)(CQ_RB + 1) * MP + (size_t)MP * (MP + 1)) * sizeof(double);
  const size_t lds_f = cq_factor_lds_doubles<MP>() * sizeof(double);
  static bool attr_set = false;   // per instance; the attribute is process-wide
  if (!attr_set) {
    HIP_CHECK(hipFuncSetAttribute((const void *)k_cqr_slab<MP>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_s));
    HIP_CHECK(hipFuncSetAttribute((const void *)k_cqr_factor<MP>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_f));
    attr_set = true;
  }
  const int passes = c.cqr_passes;
  for (int p = 0; p < passes; ++p) {
    const double *src = p <= 1 ? Y : Qb;
    const int lsrc = p <= 1 ? ldy : ldq;
    {
      // the slab product (pass >= 1) and the slab Gram blocks
      TimedLaunch tl(c, "cholqr_slab",
                     (p > 0 ? 2.0 : 0.0) * n * (double)MP * MP + (double)n * MP * (MP + 16),
                     8.0 * ((p > 0 ? 2.0 : 1.0) * n * (double)m + (double)nb * NTILE * 256));
      TT_LAUNCH(c, k_cqr_slab<MP>, dim3(nb), dim3(CQ_NT), lds_s, n, m, p, rpb, src, lsrc, Qb,
                ldq, (const double *)W, part, (const int *)flags);
    }
    {
      TimedLaunch tl(c, "cholqr_factor", (double)MP * MP * MP,
                     8.0 * ((double)nb * NTILE * 256 + 3.0 * MP * MP));
      TT_LAUNCH(c, k_cqr_factor<MP>, dim3(1), dim3(CQ_NT), lds_f, n, m, p, passes - 1, nb, W,
                Racc, (const double *)part, flags, fails, Qb, ldq, R, ldr);
    }
  }
}

}  // namespace

size_t cholqr_arena_bytes(int n, int m, bool with_q) {
  if (m < 1 || n < m || m > QR_MAXM) return 0;
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t MP = (size_t)((m + 15) / 16) * 16, T = MP / 16, NTILE = T * (T + 1) / 2;
  const int rpb = slab_rows(n);
  const size_t nb = (n + rpb - 1) / rpb;
  size_t b = al(MP * MP * 8) + al(2 * MP * MP * 8) + al(nb * NTILE * 256 * 8) + al(8);
  if (!with_q) b += al((size_t)n * m * 8);
  return b;
}

void cholqr(Ctx &c, const double *Y, int n, int m, int ldy, double *Q, int ldq, double *R,
            int ldr) {
  TT_REQUIRE(m >= 1 && n >= m && m <= QR_MAXM, "cholqr: need n >= m >= 1 and m <= 96");
  TT_REQUIRE(R != nullptr, "cholqr: R is required");
  Scope sc(c.arena);
  double *Qb = Q;
  int lq = ldq;
  if (!Qb) {                              // R only: the passes still need a Q buffer
    Qb = c.arena.dalloc((size_t)n * m);
    lq = n;
  }
  TT_REQUIRE(Qb != Y, "cholqr: Q may not alias Y");
  const int MP = (m + 15) / 16 * 16;
  switch (MP) {
    case 16: launch_passes<16>(c, Y, n, m, ldy, Qb, lq, R, ldr); break;
    case 32: launch_passes<32>(c, Y, n, m, ldy, Qb, lq, R, ldr); break;
    case 48: launch_passes<48>(c, Y, n, m, ldy, Qb, lq, R, ldr); break;
    case 64: launch_passes<64>(c, Y, n, m, ldy, Qb, lq, R, ldr); break;
    case 80: launch_passes<80>(c, Y, n, m, ldy, Qb, lq, R, ldr); break;
    default: launch_passes<96>(c, Y, n, m, ldy, Qb, lq, R, ldr); break;
  }
  c.cnt.flops += 4.0 * n * (double)m * m;
  c.cnt.bytes += 8.0 * 3.0 * n * m;
}

}  // namespace ttfv
