// GEMM for the dense core contractions of TT rounding (sketches, projections,
// back-multiplication): C = alpha * op(A) * B + beta * C with op = I or transpose, on the
// matrix cores (FP64 MFMA, or FP32 MFMA when the context computes contractions in FP32).
//
// Tiling: 64 x 64 or 64 x 128 output tile per 256-thread block, K staged through LDS in
// slices of 16.  Tall-skinny contractions (few output tiles, long K) are split along K over
// blockIdx.z into partial tiles; the last block to finish a tile (arrival counter) sums its
// partials in z order, so the result does not depend on scheduling.
#include "common.h"

#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <tuple>

namespace ttfv {
namespace {

constexpr int BM = 64, BK = 16, NT = 256;

// Matrix-core variant: the block tile is 64 x BN2 (BN2 = 64 or 128), four waves each own a
// 32 x (BN2/2) sub-tile built from 16x16 MFMA blocks (16x16x4, FP64 or FP32 operands with
// accumulation in the same type).  Operand layout of the 16x16x4 instructions: lane l
// supplies A(l % 16, l / 16) and B(l / 16, l % 16).  Result v of lane l is
// D(4 (l / 16) + v, l % 16) for FP32 and D(l / 16 + 4 v, l % 16) for FP64 (both checked).
// Operands are converted to T as they are staged in LDS; C and the split-K partials are FP64.
template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int v) { return lk + 4 * v; }
};
template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int v) { return 4 * lk + v; }
};

template <typename T, int BN2, bool TA, bool TB>
__global__ __launch_bounds__(NT) void k_gemm_mfma(int M, int N, int K, int kchunk, double alpha,
                                                  const double *__restrict__ A, int lda,
                                                  const double *__restrict__ B, int ldb,
                                                  double beta, double *__restrict__ C, int ldc,
                                                  double *__restrict__ part,
                                                  int *__restrict__ tile_cnt) {
  constexpr int TN = BN2 / 32;                   // 16-wide MFMA blocks per wave along N
  __shared__ T As[BK][BM + 4];
  __shared__ T Bs[BK][BN2 + 4];
  using V = typename Mfma<T>::v4;
  const int bm = blockIdx.x * BM, bn = blockIdx.y * BN2;
  const int k0 = blockIdx.z * kchunk;
  const int k1 = min(K, k0 + kchunk);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave & 1) * 32, wc = (wave >> 1) * (BN2 / 2);
  const int li = lane & 15, lk = lane >> 4;
  V acc[2][TN];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < TN; ++v) acc[u][v] = V{0, 0, 0, 0};

  // K-slices are fetched into registers two ahead of the one multiplied from LDS (two
  // register sets, so a slice's global loads have two slices of MFMA work to arrive)
  constexpr int QA = BM * BK / NT, QB = BN2 * BK / NT;
  double ra0[QA], rb0[QB], ra1[QA], rb1[QB];
  auto fetch = [&](int kk, double (&ra)[QA], double (&rb)[QB]) {
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int t = tid + NT * q;
      int i, k;
      if (!TA) { i = t & 63; k = t >> 6; }
      else     { k = t & 15; i = t >> 4; }
      const int gi = bm + i, gk = kk + k;
      double v = 0.0;
      if (gi < M && gk < k1) v = TA ? A[gk + (size_t)gi * lda] : A[gi + (size_t)gk * lda];
      ra[q] = v;
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const int t = tid + NT * q;
      int k, j;
      if (!TB) { k = t & 15; j = t >> 4; }
      else     { j = t % BN2; k = t / BN2; }
      const int gj = bn + j, gk = kk + k;
      double v = 0.0;
      if (gj < N && gk < k1) v = TB ? B[gj + (size_t)gk * ldb] : B[gk + (size_t)gj * ldb];
      rb[q] = v;
    }
  };
  auto stage = [&](const double (&ra)[QA], const double (&rb)[QB]) {
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int t = tid + NT * q;
      int i, k;
      if (!TA) { i = t & 63; k = t >> 6; }
      else     { k = t & 15; i = t >> 4; }
      As[k][i] = (T)ra[q];
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const int t = tid + NT * q;
      int k, j;
      if (!TB) { k = t & 15; j = t >> 4; }
      else     { j = t % BN2; k = t / BN2; }
      Bs[k][j] = (T)rb[q];
    }
  };
  auto mult = [&]() {
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      T a[2], b[TN];
#pragma unroll
      for (int u = 0; u < 2; ++u) a[u] = As[ks + lk][wr + 16 * u + li];
#pragma unroll
      for (int v = 0; v < TN; ++v) b[v] = Bs[ks + lk][wc + 16 * v + li];
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < TN; ++v) acc[u][v] = Mfma<T>::op(a[u], b[v], acc[u][v]);
    }
  };
  if (k0 < k1) fetch(k0, ra0, rb0);
  if (k0 + BK < k1) fetch(k0 + BK, ra1, rb1);
  for (int kk = k0; kk < k1; kk += 2 * BK) {
    stage(ra0, rb0);
    __syncthreads();
    if (kk + 2 * BK < k1) fetch(kk + 2 * BK, ra0, rb0);
    mult();
    __syncthreads();
    if (kk + BK >= k1) break;
    stage(ra1, rb1);
    __syncthreads();
    if (kk + 3 * BK < k1) fetch(kk + 3 * BK, ra1, rb1);
    mult();
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < TN; ++v) {
      const int gj = bn + wc + 16 * v + li;
      if (gj >= N) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gi = bm + wr + 16 * u + Mfma<T>::row(lk, e);
        if (gi >= M) continue;
        const double r = (double)acc[u][v][e];
        if (part) {
          part[((size_t)blockIdx.z * N + gj) * M + gi] = r;
        } else {
          double out = alpha * r;
          if (beta != 0.0) out += beta * C[gi + (size_t)gj * ldc];
          C[gi + (size_t)gj * ldc] = out;
        }
      }
    }
  if (!part) return;
  // split-K: the last block to finish this output tile sums the partials in z order (the
  // result does not depend on which block that is) and resets the tile's counter
  __shared__ int is_last;
  __threadfence();
  __syncthreads();
  if (tid == 0) {
    const int tile = blockIdx.x + blockIdx.y * gridDim.x;
    const int prev = atomicAdd(&tile_cnt[tile], 1);
    is_last = prev == (int)gridDim.z - 1;
    if (is_last) atomicExch(&tile_cnt[tile], 0);
  }
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  const int S = gridDim.z;
  for (int t = tid; t < BM * BN2; t += NT) {
    const int gi = bm + (t % BM), gj = bn + (t / BM);
    if (gi >= M || gj >= N) continue;
    double sum = 0.0;
    for (int z = 0; z < S; ++z) sum += part[((size_t)z * N + gj) * M + gi];
    double out = alpha * sum;
    if (beta != 0.0) out += beta * C[gi + (size_t)gj * ldc];
    C[gi + (size_t)gj * ldc] = out;
  }
}

template <typename T, int BN2, bool TA, bool TB>
void launch(Ctx &c, dim3 grid, int M, int N, int K, int kchunk, double alpha, const double *A,
            int lda, const double *B, int ldb, double beta, double *C, int ldc, double *part) {
  TT_LAUNCH(c, (k_gemm_mfma<T, BN2, TA, TB>), grid, dim3(NT), 0, M, N, K, kchunk, alpha, A,
            lda, B, ldb, beta, C, ldc, part, part ? c.tile_counters() : (int *)nullptr);
}

template <typename T, int BN2>
void dispatch(Ctx &c, bool ta, bool tb, dim3 grid, int M, int N, int K, int kchunk, double alpha,
              const double *A, int lda, const double *B, int ldb, double beta, double *C, int ldc,
              double *part) {
  if (ta && tb) launch<T, BN2, true, true>(c, grid, M, N, K, kchunk, alpha, A, lda, B, ldb, beta, C, ldc, part);
  else if (ta) launch<T, BN2, true, false>(c, grid, M, N, K, kchunk, alpha, A, lda, B, ldb, beta, C, ldc, part);
  else if (tb) launch<T, BN2, false, true>(c, grid, M, N, K, kchunk, alpha, A, lda, B, ldb, beta, C, ldc, part);
  else launch<T, BN2, false, false>(c, grid, M, N, K, kchunk, alpha, A, lda, B, ldb, beta, C, ldc, part);
}

void dispatch_any(Ctx &c, int bn2, bool ta, bool tb, dim3 grid, int M, int N, int K, int kchunk,
                  double alpha, const double *A, int lda, const double *B, int ldb, double beta,
                  double *C, int ldc, double *part) {
  if (c.fp32) {
    if (bn2 == 128) dispatch<float, 128>(c, ta, tb, grid, M, N, K, kchunk, alpha, A, lda, B, ldb, beta, C, ldc, part);
    else dispatch<float, 64>(c, ta, tb, grid, M, N, K, kchunk, alpha, A, lda, B, ldb, beta, C, ldc, part);
  } else {
    if (bn2 == 128) dispatch<double, 128>(c, ta, tb, grid, M, N, K, kchunk, alpha, A, lda, B, ldb, beta, C, ldc, part);
    else dispatch<double, 64>(c, ta, tb, grid, M, N, K, kchunk, alpha, A, lda, B, ldb, beta, C, ldc, part);
  }
}

}  // namespace

void gemm(Ctx &c, bool transA, int M, int N, int K, double alpha, const double *A, int lda,
          const double *B, int ldb, double beta, double *C, int ldc) {
  gemm2(c, transA, false, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
}

namespace {

// Tile shape of one call: output tile width (64 or 128) and the shortest K chunk a split may
// cut (0: no split).  Default: 128-wide tiles when N fills them (each row panel of A is then
// read once) and chunks of at least 512.
struct TileChoice {
  int bn2, min_chunk;
};

TileChoice default_tiles(int N) { return {N > 64 ? 128 : 64, 512}; }

// Autotuner: the first call of a shape class (transposes, precision, M and K rounded up to
// powers of two, N) times every candidate tile shape on the caller's stream (writing C, so
// only calls with beta = 0 are tuned) and keeps the fastest for the process.  Off by default; while on, the choice can differ from run to run, and with
// it the split-K summation order (results then differ in their last bits between runs).
std::atomic<bool> g_tune{false};
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int, int, int>, TileChoice> g_tuned;

int ceil_log2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

void run_tiles(Ctx &c, TileChoice t, bool transA, bool transB, int M, int N, int K,
               double alpha, const double *A, int lda, const double *B, int ldb, double beta,
               double *C, int ldc) {
  const int tm = (M + BM - 1) / BM, tn = (N + t.bn2 - 1) / t.bn2;
  const int tiles = tm * tn;
  int S = 1;
  if (t.min_chunk > 0 && tiles < 256 && K >= t.min_chunk) {
    S = std::min((512 + tiles - 1) / tiles, K / t.min_chunk);
    S = std::max(S, 1);
  }
  int kchunk = (K + S - 1) / S;
  kchunk = ((kchunk + BK - 1) / BK) * BK;
  S = (K + kchunk - 1) / kchunk;
  if (S == 1) {
    dispatch_any(c, t.bn2, transA, transB, dim3(tm, tn, 1), M, N, K, kchunk, alpha, A, lda, B,
                 ldb, beta, C, ldc, nullptr);
    return;
  }
  Scope sc(c.arena);
  double *part = c.arena.dalloc((size_t)S * M * N);
  dispatch_any(c, t.bn2, transA, transB, dim3(tm, tn, S), M, N, K, kchunk, alpha, A, lda, B,
               ldb, beta, C, ldc, part);
}

TileChoice tuned_tiles(Ctx &c, bool transA, bool transB, int M, int N, int K, double alpha,
                       const double *A, int lda, const double *B, int ldb, double *C,
                       int ldc) {
  const auto key = std::make_tuple((int)transA, (int)transB, (int)c.fp32, ceil_log2(M), N,
                                   ceil_log2(K));
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) return it->second;
  }
  // under graph capture nothing can be timed: a class not tuned yet takes the fixed rule
  if (c.capturing) return default_tiles(N);
  std::vector<TileChoice> cand;
  for (int bn2 : {64, 128}) {
    if (bn2 == 128 && N <= 64) continue;
    for (int mc : {256, 512, 1024, 0}) cand.push_back({bn2, mc});
  }
  struct Events {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Events() {
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
    }
  } ev;
  HIP_CHECK(hipEventCreate(&ev.e0));
  HIP_CHECK(hipEventCreate(&ev.e1));
  hipEvent_t e0 = ev.e0, e1 = ev.e1;
  TileChoice best = default_tiles(N);
  float best_ms = 1e30f;
  for (const TileChoice &t : cand) {
    float ms = 0.f;
    for (int rep = 0; rep < 2; ++rep) {      // the second run is timed (warm caches)
      HIP_CHECK(hipEventRecord(e0, c.stream));
      run_tiles(c, t, transA, transB, M, N, K, alpha, A, lda, B, ldb, 0.0, C, ldc);
      HIP_CHECK(hipEventRecord(e1, c.stream));
      HIP_CHECK(hipEventSynchronize(e1));
      HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
    }
    if (ms < best_ms) {
      best_ms = ms;
      best = t;
    }
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  return g_tuned.emplace(key, best).first->second;   // a concurrent tuner may have won
}

}  // namespace

size_t gemm_arena_bytes(int M, int N, int K) {
  if (M <= 0 || N <= 0 || K <= 0) return 0;
  const TileChoice t = default_tiles(N);
  const int tiles = ((M + BM - 1) / BM) * ((N + t.bn2 - 1) / t.bn2);
  if (tiles >= 256 || K < t.min_chunk) return 0;
  int S = std::max(1, std::min((512 + tiles - 1) / tiles, K / t.min_chunk));
  int kchunk = (K + S - 1) / S;
  kchunk = ((kchunk + BK - 1) / BK) * BK;
  S = (K + kchunk - 1) / kchunk;
  return S == 1 ? 0 : (size_t)S * M * N * sizeof(double) + 256;
}

void gemm_autotune(bool on) { g_tune = on; }
bool gemm_autotune_on() { return g_tune; }

int gemm_tuned_classes() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  return (int)g_tuned.size();
}

void gemm2(Ctx &c, bool transA, bool transB, int M, int N, int K, double alpha, const double *A,
           int lda, const double *B, int ldb, double beta, double *C, int ldc) {
  if (M <= 0 || N <= 0) return;
  if (K <= 0) {  // C = beta * C
    copy_scale(c, C, ldc, C, ldc, M, N, beta);
    return;
  }
  const double fl = 2.0 * M * N * K;
  const double by = 8.0 * ((double)M * K + (double)K * N + (double)M * N);
  c.cnt.flops += fl;
  c.cnt.bytes += by;
  TileChoice t = default_tiles(N);
  if (g_tune && beta == 0.0 && !c.no_alloc)
    t = tuned_tiles(c, transA, transB, M, N, K, alpha, A, lda, B, ldb, C, ldc);
  TimedLaunch tl(c, "gemm", fl, by);
  run_tiles(c, t, transA, transB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
}

}  // namespace ttfv
