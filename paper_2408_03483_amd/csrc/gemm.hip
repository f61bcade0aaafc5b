// FP64 GEMM for the dense core contractions of TT rounding (sketches, projections,
// back-multiplication): C = alpha * op(A) * B + beta * C with op = I or transpose.
//
// Tiling: 64 x 64 output tile per 256-thread block, K staged through LDS in slices of 16,
// 4 x 4 register micro-tile per thread (rows tx + 16u, columns ty + 16v, so LDS reads are
// conflict-free).  Tall-skinny contractions (few output tiles, long K) are split along K
// over blockIdx.z into partial tiles that a second kernel sums in a fixed order, so the
// result does not depend on scheduling.
#include "common.h"

#include <algorithm>

namespace ttfv {
namespace {

constexpr int BM = 64, BN = 64, BK = 16, NT = 256;

template <bool TA, bool TB>
__global__ __launch_bounds__(NT) void k_gemm(int M, int N, int K, int kchunk, double alpha,
                                             const double *__restrict__ A, int lda,
                                             const double *__restrict__ B, int ldb, double beta,
                                             double *__restrict__ C, int ldc,
                                             double *__restrict__ part) {
  __shared__ double As[BK][BM + 1];
  __shared__ double Bs[BK][BN + 1];
  const int bm = blockIdx.x * BM, bn = blockIdx.y * BN;
  const int k0 = blockIdx.z * kchunk;
  const int k1 = min(K, k0 + kchunk);
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  double acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;

  for (int kk = k0; kk < k1; kk += BK) {
#pragma unroll
    for (int t = tid; t < BM * BK; t += NT) {
      int i, k;
      if (!TA) { i = t & 63; k = t >> 6; }       // A(i, k): contiguous along i
      else     { k = t & 15; i = t >> 4; }       // A(k, i): contiguous along k
      const int gi = bm + i, gk = kk + k;
      double v = 0.0;
      if (gi < M && gk < k1) v = TA ? A[gk + (size_t)gi * lda] : A[gi + (size_t)gk * lda];
      As[k][i] = v;
    }
#pragma unroll
    for (int t = tid; t < BN * BK; t += NT) {
      int k, j;
      if (!TB) { k = t & 15; j = t >> 4; }       // B(k, j): contiguous along k
      else     { j = t & 63; k = t >> 6; }       // B(j, k) stored, contiguous along j
      const int gj = bn + j, gk = kk + k;
      double v = 0.0;
      if (gj < N && gk < k1) v = TB ? B[gj + (size_t)gk * ldb] : B[gk + (size_t)gj * ldb];
      Bs[k][j] = v;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < BK; ++k) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = As[k][tx + 16 * u];
#pragma unroll
      for (int v = 0; v < 4; ++v) b[v] = Bs[k][ty + 16 * v];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int gi = bm + tx + 16 * u;
    if (gi >= M) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int gj = bn + ty + 16 * v;
      if (gj >= N) continue;
      if (part) {
        part[((size_t)blockIdx.z * N + gj) * M + gi] = acc[u][v];
      } else {
        double out = alpha * acc[u][v];
        if (beta != 0.0) out += beta * C[gi + (size_t)gj * ldc];
        C[gi + (size_t)gj * ldc] = out;
      }
    }
  }
}

__global__ void k_splitk_reduce(int M, int N, int S, const double *__restrict__ part,
                                double alpha, double beta, double *__restrict__ C, int ldc) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)M * N) return;
  const int i = (int)(idx % M), j = (int)(idx / M);
  double s = 0.0;
  for (int z = 0; z < S; ++z) s += part[((size_t)z * N + j) * M + i];
  double out = alpha * s;
  if (beta != 0.0) out += beta * C[i + (size_t)j * ldc];
  C[i + (size_t)j * ldc] = out;
}

template <bool TA, bool TB>
void launch(Ctx &c, dim3 grid, int M, int N, int K, int kchunk, double alpha, const double *A,
            int lda, const double *B, int ldb, double beta, double *C, int ldc, double *part) {
  hipLaunchKernelGGL((k_gemm<TA, TB>), grid, dim3(NT), 0, c.stream, M, N, K, kchunk, alpha, A, lda,
                     B, ldb, beta, C, ldc, part);
}

void dispatch(Ctx &c, bool ta, bool tb, dim3 grid, int M, int N, int K, int kchunk, double alpha,
              const double *A, int lda, const double *B, int ldb, double beta, double *C, int ldc,
              double *part) {
  if (ta && tb) launch<true, true>(c, grid, M, N, K, kchunk, alpha, A, lda, B, ldb, beta, C, ldc, part);
  else if (ta) launch<true, false>(c, grid, M, N, K, kchunk, alpha, A, lda, B, ldb, beta, C, ldc, part);
  else if (tb) launch<false, true>(c, grid, M, N, K, kchunk, alpha, A, lda, B, ldb, beta, C, ldc, part);
  else launch<false, false>(c, grid, M, N, K, kchunk, alpha, A, lda, B, ldb, beta, C, ldc, part);
}

}  // namespace

void gemm(Ctx &c, bool transA, int M, int N, int K, double alpha, const double *A, int lda,
          const double *B, int ldb, double beta, double *C, int ldc) {
  gemm2(c, transA, false, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
}

void gemm2(Ctx &c, bool transA, bool transB, int M, int N, int K, double alpha, const double *A,
           int lda, const double *B, int ldb, double beta, double *C, int ldc) {
  if (M <= 0 || N <= 0) return;
  if (K <= 0) {  // C = beta * C
    copy_scale(c, C, ldc, C, ldc, M, N, beta);
    return;
  }
  const int tm = (M + BM - 1) / BM, tn = (N + BN - 1) / BN;
  const int tiles = tm * tn;
  int S = 1;
  if (tiles < 256 && K >= 512) {
    S = std::min((512 + tiles - 1) / tiles, K / 256);
    S = std::max(S, 1);
  }
  int kchunk = (K + S - 1) / S;
  kchunk = ((kchunk + BK - 1) / BK) * BK;
  S = (K + kchunk - 1) / kchunk;
  const double fl = 2.0 * M * N * K;
  const double by = 8.0 * ((double)M * K + (double)K * N + (double)M * N);
  c.cnt.flops += fl;
  c.cnt.bytes += by;
  TimedLaunch tl(c, "gemm", fl, by);
  if (S == 1) {
    dispatch(c, transA, transB, dim3(tm, tn, 1), M, N, K, kchunk, alpha, A, lda, B, ldb, beta, C,
             ldc, nullptr);
    return;
  }
  Scope sc(c.arena);
  double *part = c.arena.dalloc((size_t)S * M * N);
  dispatch(c, transA, transB, dim3(tm, tn, S), M, N, K, kchunk, alpha, A, lda, B, ldb, beta, C,
           ldc, part);
  const size_t tot = (size_t)M * N;
  hipLaunchKernelGGL(k_splitk_reduce, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                     c.stream, M, N, S, part, alpha, beta, C, ldc);
}

}  // namespace ttfv
