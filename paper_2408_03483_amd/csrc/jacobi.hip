// Small dense factorizations kept in one workgroup's LDS:
//  * one-sided (Hestenes) Jacobi SVD of the m x m core matrix of a rounding (Section 3.2
//    truncates the SVD of G1 R): columns are rotated pairwise until mutually orthogonal,
//    giving U * Sigma column by column; a round-robin schedule makes the m/2 pair rotations
//    of a round independent, one wavefront per pair;
//  * Householder QR with column pivoting, which grades a matrix before the Jacobi SVD of its
//    triangular factor (far fewer sweeps on strongly graded spectra);
//  * Gauss-Jordan inverse with partial pivoting (skeleton of the cross, maxvol start).
#include "common.h"
#include "wave.h"

#include <algorithm>

namespace ttfv {
namespace {

constexpr int NT = 1024;

// hardware reciprocal and reciprocal square root refined by one Newton step (a rotation only
// needs c^2 + s^2 = 1 to round-off, which these give; correctly rounded division and square
// roots would lengthen the dependent chain of every round)
__device__ __forceinline__ double rcp_nr(double a) {
  const double x = __builtin_amdgcn_rcp(a);
  return fma(x, fma(-a, x, 1.0), x);
}
__device__ __forceinline__ double rsq_nr(double a) {
  const double y = __builtin_amdgcn_rsq(a);
  return y * fma(-0.5 * a * y, y, 1.5);
}
constexpr int WAVES = NT / 64;

// One group of LP lanes (8 or 16) per column pair: column entries i = lane + LP r.  A round
// is a dependent chain (loads, dot products, group reduction, rotation, stores, barrier),
// so its latency, not the issue rate, sets the time per round.
// Columns whose norm is below floor ||M||_F (at least 1e-17 ||M||_F) are left alone: for a
// rounding with tolerance eps the caller sets floor = eps / 100, below which a column can
// neither change the kept rank nor move the kept part by more than a fraction of eps.
template <int LP, int RS>
__global__ __launch_bounds__(NT) void k_jacobi(const double *__restrict__ M, int m,
                                               double *__restrict__ US,
                                               double *__restrict__ sig, int max_sweeps,
                                               int trans, double floor2, int accum,
                                               int *__restrict__ status) {
  extern __shared__ double sm[];
  const int mm = (m + 1) & ~1;
  double *S = sm;                               // mm columns of m rows
  double *nrm = sm + (size_t)mm * m;            // mm norms
  double *cn = nrm + mm;                        // squared column norms during the sweeps
  double *Jr = cn + mm;                         // accum: product of the rotations, mm x mm
  __shared__ int rotated;
  __shared__ double fro_part[NT / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int gid = threadIdx.x / LP, gl = threadIdx.x % LP;
  const int nt = blockDim.x, ngroups = nt / LP;
  double part = 0.0;
  for (int idx = threadIdx.x; idx < mm * m; idx += nt) {
    double v = 0.0;
    if (idx < m * m) v = trans ? M[(idx / m) + (size_t)(idx % m) * m] : M[idx];
    S[idx] = v;
    part += v * v;
  }
  if (accum)
    for (int idx = threadIdx.x; idx < mm * mm; idx += nt)
      Jr[idx] = (idx % mm) == (idx / mm) ? 1.0 : 0.0;
  part = wave_sum(part);
  if (lane == 0) fro_part[wave] = part;
  __syncthreads();
  double fro2 = 0.0;
  for (int w = 0; w < nt / 64; ++w) fro2 += fro_part[w];
  const double tiny = fmax(1e-34, floor2) * fro2;
  const double tol = sqrt((double)m) * 2.220446049250313e-16;
  const double tol2 = tol * tol;
  const int np = mm - 1;                        // round-robin over mm players, np rounds
  bool converged = false;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    if (threadIdx.x == 0) rotated = 0;
    // exact squared norms at the start of each sweep; within a sweep they follow the
    // rotations (a' = a - t g, b' = b + t g), so a round reduces only the cross product
    for (int col = gid; col < mm; col += ngroups) {
      const double *cc = S + (size_t)col * m;
      double acc[1] = {0.0};
#pragma unroll
      for (int r = 0; r < RS; ++r) {
        const int i = gl + LP * r;
        const double x = i < m ? cc[i] : 0.0;
        acc[0] += x * x;
      }
      group_sum_n<LP, 1>(acc);
      if (gl == 0) cn[col] = acc[0];
    }
    __syncthreads();
    for (int t = 0; t < np; ++t) {
      for (int k = gid; k < mm / 2; k += ngroups) {
        int a = k + t;
        if (a >= np) a -= np;
        int b = np - k + t;
        if (b >= np) b -= np;
        if (k == 0) b = np;
        const int p = min(a, b), q = max(a, b);
        double *cp = S + (size_t)p * m, *cq = S + (size_t)q * m;
        double xp[RS], xq[RS];
        double acc[1] = {0.0};
#pragma unroll
        for (int r = 0; r < RS; ++r) {
          const int i = gl + LP * r;
          xp[r] = i < m ? cp[i] : 0.0;
          xq[r] = i < m ? cq[i] : 0.0;
          acc[0] += xp[r] * xq[r];
        }
        group_sum_n<LP, 1>(acc);
        const double al = cn[p], be = cn[q], ga = acc[0];
        if (al > tiny && be > tiny && ga * ga > tol2 * al * be) {
          // tan of the rotation angle, t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)) with
          // zeta = (be - al) / (2 ga), written with one square root and one division
          const double d = be - al, g2 = 2.0 * ga;
          const double dd = fma(d, d, g2 * g2);
          const double r = dd * rsq_nr(dd);
          const double tt = (d >= 0.0 ? g2 : -g2) * rcp_nr(fabs(d) + r);
          const double c = rsq_nr(fma(tt, tt, 1.0)), s = c * tt;
#pragma unroll
          for (int r = 0; r < RS; ++r) {
            const int i = gl + LP * r;
            if (i < m) {
              cp[i] = c * xp[r] - s * xq[r];
              cq[i] = s * xp[r] + c * xq[r];
            }
          }
          if (accum) {
            double *jp = Jr + (size_t)p * mm, *jq = Jr + (size_t)q * mm;
#pragma unroll
            for (int r = 0; r < RS; ++r) {
              const int i = gl + LP * r;
              if (i < mm) {
                const double a = jp[i], b = jq[i];
                jp[i] = c * a - s * b;
                jq[i] = s * a + c * b;
              }
            }
          }
          if (gl == 0) {
            cn[p] = al - tt * ga;
            cn[q] = be + tt * ga;
            rotated = 1;
          }
        }
      }
      __syncthreads();
    }
    const int any = rotated;
    __syncthreads();
    if (!any) {
      converged = true;
      break;
    }
  }
  // stopped at the sweep cap while still rotating: count it (one lane; launches on a
  // stream run in order, so the count needs no atomic)
  if (!converged && threadIdx.x == 0) status[0] = status[0] + 1;
  // norms
  for (int cidx = wave; cidx < mm; cidx += nt / 64) {
    const double *cc = S + (size_t)cidx * m;
    double x0 = lane < m ? cc[lane] : 0.0, x1 = lane + 64 < m ? cc[lane + 64] : 0.0;
    double s2 = wave_sum(x0 * x0 + x1 * x1);
    if (lane == 0) nrm[cidx] = sqrt(s2);
  }
  __syncthreads();
  // rank by (norm desc, index asc) over the first m columns (the pad column is zero)
  for (int i = threadIdx.x; i < m; i += nt) {
    int rk = 0;
    const double ni = nrm[i];
    for (int j = 0; j < m; ++j) {
      const double nj = nrm[j];
      rk += (nj > ni) || (nj == ni && j < i);
    }
    sig[rk] = ni;
    if (accum)   // left singular vectors of the transpose held in S, scaled by the norms
      for (int r = 0; r < m; ++r) US[(size_t)rk * m + r] = Jr[(size_t)i * mm + r] * ni;
    else
      for (int r = 0; r < m; ++r) US[(size_t)rk * m + r] = S[(size_t)i * m + r];
  }
}

// Householder QR with column pivoting of an m x m matrix (m <= 96) in one workgroup,
// M P = Q2 R2, with Q2 formed explicitly (backward accumulation of the reflectors).  The
// pivot is the remaining column of largest norm below the current row (ties to the smallest
// index); the norms are recomputed exactly after every step instead of downdated.  The
// permutation is not returned: the left singular vectors of M are Q2 times those of R2.
// Wave 0 picks the pivot, swaps it in and forms the reflector; then groups of 16 lanes, one
// column each, apply it to the trailing columns: two barriers per column.
constexpr int QRCP_NT = 1024;
__global__ __launch_bounds__(QRCP_NT) void k_qrcp(const double *__restrict__ M, int m,
                                                  double *__restrict__ R2,
                                                  double *__restrict__ Q2) {
  extern __shared__ double sm[];
  double *A = sm;                               // m x m, column-major: R above, v below
  double *Qs = A + (size_t)m * m;               // m x m, the explicit Q2
  double *vn = Qs + (size_t)m * m;              // squared norms below the current row
  double *tau = vn + m;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int gid = threadIdx.x >> 4, gl = threadIdx.x & 15, ngroups = QRCP_NT / 16;
  for (int idx = threadIdx.x; idx < m * m; idx += QRCP_NT) A[idx] = M[idx];
  __syncthreads();
  for (int k = gid; k < m; k += ngroups) {
    double s2[1] = {0.0};
    for (int i = gl; i < m; i += 16) s2[0] += A[i + (size_t)k * m] * A[i + (size_t)k * m];
    row16_sum_n<1>(s2);
    if (gl == 0) vn[k] = s2[0];
  }
  __syncthreads();
  for (int j = 0; j < m; ++j) {
    double *aj = A + (size_t)j * m;
    if (wave == 0) {
      // pivot: largest squared norm, smallest index among equals
      double bv = -1.0;
      int bi = j;
      for (int k = j + lane; k < m; k += 64)
        if (vn[k] > bv) {
          bv = vn[k];
          bi = k;
        }
      const double mx = wave_max(bv);
      const unsigned long long hit = __ballot(bv == mx);
      if (hit) {
        // among the lanes that hold the maximum, the smallest index
        int best = m;
        unsigned long long h = hit;
        while (h) {
          const int l = __builtin_ctzll(h);
          h &= h - 1;
          best = min(best, __builtin_amdgcn_readlane(bi, l));
        }
        bi = best;
      } else {
        bi = j;   // no finite norm: keep the column (the caller sees the non-finite result)
      }
      if (bi != j) {
        double *ap = A + (size_t)bi * m;
        for (int i = lane; i < m; i += 64) {
          const double x = aj[i];
          aj[i] = ap[i];
          ap[i] = x;
        }
        __builtin_amdgcn_wave_barrier();
      }
      // reflector of column j over rows j .. m-1 (LAPACK's dlarfg convention)
      double ss = 0.0;
      for (int i = j + 1 + lane; i < m; i += 64) ss += aj[i] * aj[i];
      ss = wave_sum(ss);
      const double alpha = aj[j];
      double beta = alpha, t = 0.0, scal = 0.0;
      if (ss > 0.0) {
        const double nrm = sqrt(alpha * alpha + ss);
        beta = alpha >= 0.0 ? -nrm : nrm;
        t = (beta - alpha) / beta;
        scal = 1.0 / (alpha - beta);
      }
      __builtin_amdgcn_wave_barrier();
      for (int i = j + 1 + lane; i < m; i += 64) aj[i] *= scal;
      if (lane == 0) {
        aj[j] = beta;
        tau[j] = t;
      }
    }
    __syncthreads();
    const double t = tau[j];
    // apply the reflector to the columns right of j, then their squared norms below row j
    for (int k = j + 1 + gid; k < m; k += ngroups) {
      double *ak = A + (size_t)k * m;
      if (t != 0.0) {
        double w[1] = {0.0};
        for (int i = j + gl; i < m; i += 16) w[0] += (i == j ? 1.0 : aj[i]) * ak[i];
        row16_sum_n<1>(w);
        const double tw = t * w[0];
        for (int i = j + gl; i < m; i += 16) ak[i] -= tw * (i == j ? 1.0 : aj[i]);
      }
      double s2[1] = {0.0};
      for (int i = j + 1 + gl; i < m; i += 16) s2[0] += ak[i] * ak[i];
      row16_sum_n<1>(s2);
      if (gl == 0) vn[k] = s2[0];
    }
    __syncthreads();
  }
  for (int idx = threadIdx.x; idx < m * m; idx += QRCP_NT) {
    const int i = idx % m, c = idx / m;
    R2[idx] = i <= c ? A[idx] : 0.0;
    Qs[idx] = i == c ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int j = m - 1; j >= 0; --j) {   // Q2 = H_0 ... H_{m-1}: apply H_j to Q2(j:, j:)
    const double t = tau[j];
    const double *aj = A + (size_t)j * m;
    if (t != 0.0)
      for (int k = j + gid; k < m; k += ngroups) {
        double *qk = Qs + (size_t)k * m;
        double w[1] = {0.0};
        for (int i = j + gl; i < m; i += 16) w[0] += (i == j ? 1.0 : aj[i]) * qk[i];
        row16_sum_n<1>(w);
        const double tw = t * w[0];
        for (int i = j + gl; i < m; i += 16) qk[i] -= tw * (i == j ? 1.0 : aj[i]);
      }
    __syncthreads();
  }
  for (int idx = threadIdx.x; idx < m * m; idx += QRCP_NT) Q2[idx] = Qs[idx];
}

// Gauss-Jordan inverse of an m x m matrix (m <= 96) with partial pivoting
__global__ __launch_bounds__(NT) void k_inverse(const double *__restrict__ M, int m, int ldm,
                                                double *__restrict__ Minv) {
  extern __shared__ double sm[];
  const int w = 2 * m;
  double *T = sm;                    // row-major m x 2m
  __shared__ int piv;
  __shared__ double pv;
  for (int idx = threadIdx.x; idx < m * w; idx += NT) {
    const int i = idx / w, j = idx - i * w;
    T[idx] = j < m ? M[i + (size_t)j * ldm] : (j - m == i ? 1.0 : 0.0);
  }
  __syncthreads();
  for (int j = 0; j < m; ++j) {
    // pivot: largest |T(i, j)| over i >= j, ties to the smallest row (wave 0, m <= 128)
    if (threadIdx.x < 64) {
      double bv = -1.0;
      int bi = m;
      for (int i = j + (int)threadIdx.x; i < m; i += 64) {
        const double v = fabs(T[(size_t)i * w + j]);
        if (v > bv) { bv = v; bi = i; }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(bv, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
      }
      if (threadIdx.x == 0) piv = bi;
    }
    __syncthreads();
    const int pr = piv;
    if (pr != j)
      for (int c = threadIdx.x; c < w; c += NT) {
        const double tmp = T[(size_t)j * w + c];
        T[(size_t)j * w + c] = T[(size_t)pr * w + c];
        T[(size_t)pr * w + c] = tmp;
      }
    __syncthreads();
    if (threadIdx.x == 0) pv = T[(size_t)j * w + j];
    __syncthreads();
    const double inv = 1.0 / pv;
    for (int c = threadIdx.x; c < w; c += NT) T[(size_t)j * w + c] *= inv;
    __syncthreads();
    for (int idx = threadIdx.x; idx < m * w; idx += NT) {
      const int i = idx / w, c = idx - i * w;
      if (i == j) continue;
      const double f = T[(size_t)i * w + j];
      if (c != j) T[idx] -= f * T[(size_t)j * w + c];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < m; i += NT)
      if (i != j) T[(size_t)i * w + j] = 0.0;
    __syncthreads();
  }
  for (int idx = threadIdx.x; idx < m * m; idx += NT) {
    const int i = idx % m, j = idx / m;
    Minv[i + (size_t)j * m] = T[(size_t)i * w + m + j];
  }
}

__global__ void k_normalise(const double *__restrict__ US, const double *__restrict__ sig, int m,
                            int k, double *__restrict__ U) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * k) return;
  const int c = idx / m;
  const double s = sig[c];
  U[idx] = s > 0.0 ? US[idx] / s : 0.0;
}

template <typename K>
void set_lds(K kern, size_t bytes) {
  HIP_CHECK(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)bytes));
}

}  // namespace

void jacobi_svd(Ctx &c, const double *M, int m, double *US, double *sig, bool trans,
                double floor_rel, bool accumulate) {
  TT_REQUIRE(m >= 1 && m <= 128, "jacobi_svd: m out of range");
  TT_REQUIRE(!accumulate || m <= QR_MAXM, "jacobi_svd: accumulation needs m <= 96");
  const int mm = (m + 1) & ~1;
  const size_t lds = ((size_t)mm * m + 2 * mm + (accumulate ? (size_t)mm * mm : 0)) *
                     sizeof(double);
  TimedLaunch tl(c, "jacobi", 22.0 * m * m * m, 8.0 * (2.0 * m * m + m));
  // 16 lanes per pair (measured faster than 8 at m = 64); threads = pairs * lanes per pair
  auto launch = [&](auto kern, int lp) {
    const int nthreads = std::max(64, ((mm / 2) * lp + 63) / 64 * 64);
    set_lds(kern, lds);
    TT_LAUNCH(c, kern, dim3(1), dim3(nthreads), lds, M, m, US, sig, c.jacobi_max_sweeps,
              trans ? 1 : 0, floor_rel * floor_rel, accumulate ? 1 : 0, c.arena.status());
  };
  if (m <= 32) launch(k_jacobi<16, 2>, 16);
  else if (m <= 64) launch(k_jacobi<16, 4>, 16);
  else if (m <= 96) launch(k_jacobi<16, 6>, 16);
  else launch(k_jacobi<16, 8>, 16);
  c.cnt.flops += 22.0 * m * m * m;
}

void svd_pivoted(Ctx &c, const double *M, int m, double *US, double *sig, double floor_rel) {
  TT_REQUIRE(m >= 1 && m <= QR_MAXM, "svd_pivoted: m out of range");
  Scope sc(c.arena);
  double *R2 = c.arena.dalloc((size_t)m * m), *Q2 = c.arena.dalloc((size_t)m * m);
  double *UJ = c.arena.dalloc((size_t)m * m);
  const size_t lds = (2 * (size_t)m * m + 2 * (size_t)m) * sizeof(double);
  set_lds(k_qrcp, lds);
  hipLaunchKernelGGL(k_qrcp, dim3(1), dim3(QRCP_NT), lds, c.stream, M, m, R2, Q2);
  c.cnt.flops += 8.0 * m * m * m / 3.0;
  // one-sided Jacobi on R2^T with the rotations accumulated: R2 = J Sigma V^T
  jacobi_svd(c, R2, m, UJ, sig, true, floor_rel, true);
  gemm2(c, false, false, m, m, m, 1.0, Q2, m, UJ, m, 0.0, US, m);
}

void small_inverse(Ctx &c, const double *M, int m, int ldm, double *Minv) {
  TT_REQUIRE(m >= 1 && m <= 128, "small_inverse: m out of range");
  const size_t lds = (size_t)m * 2 * m * sizeof(double);
  set_lds(k_inverse, lds);
  hipLaunchKernelGGL(k_inverse, dim3(1), dim3(NT), lds, c.stream, M, m, ldm, Minv);
  c.cnt.flops += 2.0 * m * m * m;
}

void normalise_cols(Ctx &c, const double *US, const double *sig, int m, int k, double *U) {
  if (k <= 0) return;
  hipLaunchKernelGGL(k_normalise, dim3((m * k + 255) / 256), dim3(256), 0, c.stream, US, sig, m, k,
                     U);
}

}  // namespace ttfv
