// Learned pivot proposer for the cross (an addition to the paper's method, which uses
// alternating maxvol sweeps, Section 3.3).
//
// A multilayer perceptron 16 -> 256 -> 256 -> 1 (ReLU) scores every column index of a
// cross from 16 features of the cross's starting TT and the previous pivots; the top-K
// indices become the column set of a single refinement sweep.  Weights and activations are
// BF16 with FP32 accumulation on the matrix cores (16x16x16 BF16 MFMA); FP32 master weights
// are trained with Adam on (features, final maxvol pivots) pairs logged from plain crosses.
//
// Features of index j (n2 indices, B0 = second core of the starting TT, n2 x r):
//   0 previous pivot flag, 1 exp(-d/2) with d the distance to the nearest previous pivot,
//   2..6 log(1 + lev(j+o)), 7..11 log(1 + jump(j+o)) for o = -2..2 (clamped), with
//   lev(j) = n2 |B0[j]|^2 / |B0|_F^2 and jump(j) = n2 |B0[j+1] - B0[j]|^2 / |B0|_F^2,
//   12 j/n2, 13 sin(2 pi j/n2), 14 cos(2 pi j/n2), 15 one.
#include "common.h"
#include "wave.h"

#include <algorithm>
#include <cmath>

namespace ttfv {
namespace {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int F = PM_F, HID = PM_H;
constexpr int GT = 64, GK = 16;        // bf16 GEMM tile (64 x 64) and K slice

__device__ __forceinline__ bf16_t f2bf(float x) {   // round to nearest even (finite inputs)
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (bf16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(bf16_t h) { return __uint_as_float((uint32_t)h << 16); }

// C (f32, row-major, ld ldc) = A B with A(i, k) = A[i sai + k sak], B(k, j) = B[k sbk + j sbj]
// (bf16).  Four waves each own a 32 x 32 sub-tile of 16x16 MFMA blocks; lane l supplies
// A(l % 16, 4 (l / 16) + q) and B(4 (l / 16) + q, l % 16), q = 0..3, and receives
// D(4 (l / 16) + v, l % 16).  Split-K partials (part != null) are summed by k_sum_parts.
__global__ __launch_bounds__(256) void k_gemm_bf16(int M, int N, int K, int kchunk,
                                                   const bf16_t *__restrict__ A, long sai,
                                                   long sak, const bf16_t *__restrict__ B,
                                                   long sbk, long sbj, float *__restrict__ C,
                                                   int ldc, float *__restrict__ part) {
  __shared__ bf16_t As[GT][GK + 4];   // As[i][k]
  __shared__ bf16_t Bs[GT][GK + 4];   // Bs[j][k]
  const int bm = blockIdx.x * GT, bn = blockIdx.y * GT;
  const int k0 = blockIdx.z * kchunk, k1 = min(K, k0 + kchunk);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  f4 acc[2][2];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) acc[u][v] = f4{0.f, 0.f, 0.f, 0.f};
  for (int kk = k0; kk < k1; kk += GK) {
#pragma unroll
    for (int t = tid; t < GT * GK; t += 256) {
      int i, k;
      if (sak == 1) { k = t % GK; i = t / GK; } else { i = t % GT; k = t / GT; }
      const int gi = bm + i, gk = kk + k;
      As[i][k] = (gi < M && gk < k1) ? A[gi * sai + gk * sak] : (bf16_t)0;
    }
#pragma unroll
    for (int t = tid; t < GT * GK; t += 256) {
      int j, k;
      if (sbk == 1) { k = t % GK; j = t / GK; } else { j = t % GT; k = t / GT; }
      const int gj = bn + j, gk = kk + k;
      Bs[j][k] = (gj < N && gk < k1) ? B[gk * sbk + gj * sbj] : (bf16_t)0;
    }
    __syncthreads();
    s4 a[2], b[2];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q) a[u][q] = (short)As[wr + 16 * u + li][4 * lk + q];
#pragma unroll
    for (int v = 0; v < 2; ++v)
#pragma unroll
      for (int q = 0; q < 4; ++q) b[v][q] = (short)Bs[wc + 16 * v + li][4 * lk + q];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int v = 0; v < 2; ++v)
        acc[u][v] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[u], b[v], acc[u][v], 0, 0, 0);
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const int gj = bn + wc + 16 * v + li;
      if (gj >= N) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gi = bm + wr + 16 * u + 4 * lk + e;
        if (gi >= M) continue;
        if (part) part[((size_t)blockIdx.z * M + gi) * N + gj] = acc[u][v][e];
        else C[(size_t)gi * ldc + gj] = acc[u][v][e];
      }
    }
}

__global__ void k_sum_parts(int M, int N, int S, const float *__restrict__ part,
                            float *__restrict__ C, int ldc) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= M * N) return;
  const int i = idx / N, j = idx % N;
  float s = 0.f;
  for (int z = 0; z < S; ++z) s += part[((size_t)z * M + i) * N + j];
  C[(size_t)i * ldc + j] = s;
}

// H = bf16(relu(Z + b)) row-major N x HID
__global__ void k_bias_relu(int N, const float *__restrict__ Z, const float *__restrict__ b,
                            bf16_t *__restrict__ H) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= N * HID) return;
  H[idx] = f2bf(fmaxf(Z[idx] + b[idx % HID], 0.f));
}

// s_i = H2[i] . w3 + b3 (one wave per row)
__global__ void k_head(int N, const bf16_t *__restrict__ H2, const bf16_t *__restrict__ w3,
                       const float *__restrict__ b3, float *__restrict__ s) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (row >= N) return;
  float acc = 0.f;
  for (int c = lane; c < HID; c += 64) acc += bf2f(H2[(size_t)row * HID + c]) * bf2f(w3[c]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) s[row] = acc + b3[0];
}

__global__ void k_to_bf16(int n, const float *__restrict__ x, bf16_t *__restrict__ y) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < n) y[idx] = f2bf(x[idx]);
}

// ds_i = w_i (sigmoid(s_i) - y_i) / Ntot ; loss partial sums per block
__global__ void k_loss_grad(int N, const float *__restrict__ s, const float *__restrict__ y,
                            float pos_weight, float inv_total, float *__restrict__ ds,
                            float *__restrict__ loss_part) {
  __shared__ float red[4];
  const int i = blockIdx.x * 256 + threadIdx.x;
  float l = 0.f;
  if (i < N) {
    const float si = s[i], yi = y[i];
    const float w = yi > 0.5f ? pos_weight : 1.f;
    const float sig = 1.f / (1.f + expf(-si));
    ds[i] = w * (sig - yi) * inv_total;
    const float sp = fmaxf(si, 0.f) + log1pf(expf(-fabsf(si)));
    l = w * (sp - yi * si) * inv_total;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) l += __shfl_xor(l, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = l;
  __syncthreads();
  if (threadIdx.x == 0) loss_part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// dH2 = bf16(ds_i w3[c] [H2 > 0])
__global__ void k_back_head(int N, const float *__restrict__ ds, const bf16_t *__restrict__ w3,
                            const bf16_t *__restrict__ H2, bf16_t *__restrict__ dH2) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= N * HID) return;
  const int i = idx / HID, c = idx % HID;
  const float g = bf2f(H2[idx]) > 0.f ? ds[i] * bf2f(w3[c]) : 0.f;
  dH2[idx] = f2bf(g);
}

// dH1 = bf16(G [H1 > 0])
__global__ void k_relu_mask(int N, const float *__restrict__ G, const bf16_t *__restrict__ H1,
                            bf16_t *__restrict__ dH1) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= N * HID) return;
  dH1[idx] = f2bf(bf2f(H1[idx]) > 0.f ? G[idx] : 0.f);
}

// out[c] = sum_i X(i, c) (w_i if w) over a chunk of rows; partials per block (row chunk)
__global__ void k_colsum_bf16(int N, int C, const bf16_t *__restrict__ X,
                              const float *__restrict__ w, int rows_per_block,
                              float *__restrict__ part) {
  const int c = threadIdx.x + blockIdx.y * blockDim.x;
  if (c >= C) return;
  const int r0 = blockIdx.x * rows_per_block, r1 = min(N, r0 + rows_per_block);
  float s = 0.f;
  for (int i = r0; i < r1; ++i) s += bf2f(X[(size_t)i * C + c]) * (w ? w[i] : 1.f);
  part[(size_t)blockIdx.x * C + c] = s;
}

__global__ void k_sum_rows(int S, int C, const float *__restrict__ part, float *__restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  float s = 0.f;
  for (int z = 0; z < S; ++z) s += part[(size_t)z * C + c];
  out[c] = s;
}

__global__ void k_sum_vec(int n, const float *__restrict__ x, float *__restrict__ out) {
  __shared__ float red[4];
  float s = 0.f;
  for (int i = threadIdx.x; i < n; i += 256) s += x[i];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void k_adam(int n, float *__restrict__ p, const float *__restrict__ g,
                       float *__restrict__ m, float *__restrict__ v, float lr, float c1,
                       float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = 0.9f * m[i] + 0.1f * gi;
  const float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

// ---- features -----------------------------------------------------------------------
__global__ void k_feat_rows(const double *__restrict__ B0, int n2, int r, int ldb,
                            double *__restrict__ lev, double *__restrict__ jump) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n2) return;
  const int jn = min(j + 1, n2 - 1);
  double a = 0.0, d = 0.0;
  for (int c = 0; c < r; ++c) {
    const double x = B0[j + (size_t)c * ldb];
    const double y = B0[jn + (size_t)c * ldb] - x;
    a += x * x;
    d += y * y;
  }
  lev[j] = a;
  jump[j] = d;
}

__global__ void k_sum_d(int n, const double *__restrict__ x, double *__restrict__ out) {
  __shared__ double red[16];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) s += x[i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < 16; ++w) t += red[w];
    out[0] = t;
  }
}

__global__ void k_features(int n2, const double *__restrict__ lev, const double *__restrict__ jump,
                           const double *__restrict__ nrm2p, const int *__restrict__ J, int nJ,
                           float *__restrict__ Xf, bf16_t *__restrict__ Xb) {
  __shared__ int Js[128];
  for (int t = threadIdx.x; t < nJ && t < 128; t += blockDim.x) Js[t] = J[t];
  __syncthreads();
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n2) return;
  double nrm2 = nrm2p[0];
  if (!(nrm2 > 0.0)) nrm2 = 1.0;
  const double sc = (double)n2 / nrm2;
  float f[F];
  int dmin = n2;
  bool in = false;
  for (int t = 0; t < min(nJ, 128); ++t) {
    const int d = abs(j - Js[t]);
    dmin = min(dmin, d);
    in = in || d == 0;
  }
  f[0] = in ? 1.f : 0.f;
  f[1] = (float)exp(-0.5 * dmin);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const int jj = min(max(j + k - 2, 0), n2 - 1);
    f[2 + k] = (float)log1p(sc * lev[jj]);
    f[7 + k] = (float)log1p(sc * jump[jj]);
  }
  const double x = (double)j / n2;
  f[12] = (float)x;
  f[13] = (float)sin(2.0 * M_PI * x);
  f[14] = (float)cos(2.0 * M_PI * x);
  f[15] = 1.f;
#pragma unroll
  for (int k = 0; k < F; ++k) {
    if (Xf) Xf[(size_t)j * F + k] = f[k];
    if (Xb) Xb[(size_t)j * F + k] = f2bf(f[k]);
  }
}

// ---- top-K: radix select on order-preserving keys, ties to the smaller index -----------
__device__ __forceinline__ uint32_t fkey(float x) {
  const uint32_t u = __float_as_uint(x);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

constexpr int TKT = 1024;

// exclusive prefix over threads (in thread order) of v; returns this thread's offset
__device__ int block_excl_scan(int v, int *buf) {
  buf[threadIdx.x] = v;
  __syncthreads();
  for (int off = 1; off < TKT; off <<= 1) {
    const int add = threadIdx.x >= off ? buf[threadIdx.x - off] : 0;
    __syncthreads();
    buf[threadIdx.x] += add;
    __syncthreads();
  }
  const int incl = buf[threadIdx.x];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(TKT) void k_topk(const float *__restrict__ s, int n, int K,
                                               int *__restrict__ out) {
  __shared__ int hist[256];
  __shared__ int buf[TKT];
  __shared__ uint32_t sh_prefix;
  __shared__ int sh_need;
  const int per = (n + TKT - 1) / TKT;
  const int lo = threadIdx.x * per, hi = min(n, lo + per);
  // radix select of the K-th largest key, 8 bits at a time from the top
  uint32_t prefix = 0, mask = 0;
  int need = K;
  for (int shift = 24; shift >= 0; shift -= 8) {
    for (int b = threadIdx.x; b < 256; b += TKT) hist[b] = 0;
    __syncthreads();
    for (int i = lo; i < hi; ++i) {
      const uint32_t k = fkey(s[i]);
      if ((k & mask) == prefix) atomicAdd(&hist[(k >> shift) & 255u], 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int cum = 0, b = 255;
      for (; b > 0; --b) {
        if (cum + hist[b] >= need) break;
        cum += hist[b];
      }
      sh_prefix = prefix | ((uint32_t)b << shift);
      sh_need = need - cum;
    }
    __syncthreads();
    prefix = sh_prefix;
    need = sh_need;
    mask |= 255u << shift;
    __syncthreads();
  }
  // prefix is the K-th largest key; take every key above it and the first `need` equal ones
  int eq = 0;
  for (int i = lo; i < hi; ++i) eq += fkey(s[i]) == prefix;
  const int eq_before = block_excl_scan(eq, buf);
  int sel = 0;
  {
    int e = eq_before;
    for (int i = lo; i < hi; ++i) {
      const uint32_t k = fkey(s[i]);
      if (k > prefix) ++sel;
      else if (k == prefix) sel += (e++ < need);
    }
  }
  int pos = block_excl_scan(sel, buf);
  {
    int e = eq_before;
    for (int i = lo; i < hi; ++i) {
      const uint32_t k = fkey(s[i]);
      bool take = k > prefix;
      if (k == prefix) take = (e++ < need);
      if (take) out[pos++] = i;
    }
  }
}

void gemm_bf16(Ctx &c, int M, int N, int K, const bf16_t *A, long sai, long sak,
               const bf16_t *B, long sbk, long sbj, float *C, int ldc) {
  const int tm = (M + GT - 1) / GT, tn = (N + GT - 1) / GT;
  int S = 1;
  if (tm * tn < 128 && K >= 1024) S = std::min(64, std::max(1, K / 512));
  int kchunk = (K + S - 1) / S;
  kchunk = (kchunk + GK - 1) / GK * GK;
  S = (K + kchunk - 1) / kchunk;
  c.cnt.flops += 2.0 * M * N * K;
  if (S == 1) {
    hipLaunchKernelGGL(k_gemm_bf16, dim3(tm, tn, 1), dim3(256), 0, c.stream, M, N, K, kchunk, A,
                       sai, sak, B, sbk, sbj, C, ldc, nullptr);
    return;
  }
  Scope sc(c.arena);
  float *part = static_cast<float *>(c.arena.alloc((size_t)S * M * N * sizeof(float)));
  hipLaunchKernelGGL(k_gemm_bf16, dim3(tm, tn, S), dim3(256), 0, c.stream, M, N, K, kchunk, A,
                     sai, sak, B, sbk, sbj, C, ldc, part);
  hipLaunchKernelGGL(k_sum_parts, dim3((M * N + 255) / 256), dim3(256), 0, c.stream, M, N, S,
                     part, C, ldc);
}

void colsum_bf16(Ctx &c, int N, int C, const bf16_t *X, const float *w, float *out) {
  Scope sc(c.arena);
  const int rpb = 256;
  const int S = (N + rpb - 1) / rpb;
  float *part = static_cast<float *>(c.arena.alloc((size_t)S * C * sizeof(float)));
  hipLaunchKernelGGL(k_colsum_bf16, dim3(S, (C + 255) / 256), dim3(256), 0, c.stream, N, C, X, w,
                     rpb, part);
  hipLaunchKernelGGL(k_sum_rows, dim3((C + 255) / 256), dim3(256), 0, c.stream, S, C, part, out);
}

inline dim3 grid1(size_t n) { return dim3((unsigned)((n + 255) / 256)); }

uint64_t sm64(uint64_t &s) {
  s += 0x9E3779B97F4A7C15ull;
  uint64_t z = s;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace

// ---- model ------------------------------------------------------------------------------

PivotModel::PivotModel(size_t max_rows, uint64_t seed) : cap(max_rows) {
  HIP_CHECK(hipMalloc(&p, PM_NPARAM * sizeof(float)));
  HIP_CHECK(hipMalloc(&g, PM_NPARAM * sizeof(float)));
  HIP_CHECK(hipMalloc(&m, PM_NPARAM * sizeof(float)));
  HIP_CHECK(hipMalloc(&v, PM_NPARAM * sizeof(float)));
  HIP_CHECK(hipMalloc(&wb, (PM_W1_N + PM_W2_N + PM_W3_N) * sizeof(bf16_t)));
  if (cap) {
    HIP_CHECK(hipMalloc(&Xd, cap * F * sizeof(bf16_t)));
    HIP_CHECK(hipMalloc(&Yd, cap * sizeof(float)));
  }
  HIP_CHECK(hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking));
  c.arena.init((size_t)1 << 30);
  c.prepare();
  // He-normal weights from a SplitMix64 stream (Box-Muller), zero biases
  std::vector<float> h(PM_NPARAM, 0.f);
  uint64_t st = seed;
  auto normal = [&]() {
    const double u1 = ((sm64(st) >> 11) + 1.0) * (1.0 / 9007199254740993.0);
    const double u2 = (sm64(st) >> 11) * (1.0 / 9007199254740992.0);
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * M_PI * u2);
  };
  for (size_t i = 0; i < PM_W1_N; ++i) h[PM_W1 + i] = (float)(normal() * std::sqrt(2.0 / F));
  for (size_t i = 0; i < PM_W2_N; ++i) h[PM_W2 + i] = (float)(normal() * std::sqrt(2.0 / HID));
  for (size_t i = 0; i < PM_W3_N; ++i) h[PM_W3 + i] = (float)(normal() * std::sqrt(1.0 / HID));
  set_weights(h.data());
}

PivotModel::~PivotModel() {
  (void)hipStreamSynchronize(c.stream);
  for (void *q : {(void *)p, (void *)g, (void *)m, (void *)v, (void *)wb, (void *)Xd, (void *)Yd})
    if (q) (void)hipFree(q);
  if (c.stream) (void)hipStreamDestroy(c.stream);
}

void PivotModel::set_weights(const float *host) {
  std::lock_guard<std::mutex> lk(mu);
  HIP_CHECK(hipMemcpyAsync(p, host, PM_NPARAM * sizeof(float), hipMemcpyHostToDevice, c.stream));
  HIP_CHECK(hipMemsetAsync(m, 0, PM_NPARAM * sizeof(float), c.stream));
  HIP_CHECK(hipMemsetAsync(v, 0, PM_NPARAM * sizeof(float), c.stream));
  t = 0;
  refresh_bf16();
  c.sync();
}

void PivotModel::get_weights(float *host) {
  std::lock_guard<std::mutex> lk(mu);
  HIP_CHECK(hipMemcpyAsync(host, p, PM_NPARAM * sizeof(float), hipMemcpyDeviceToHost, c.stream));
  c.sync();
}

void PivotModel::refresh_bf16() {
  hipLaunchKernelGGL(k_to_bf16, grid1(PM_W1_N), dim3(256), 0, c.stream, (int)PM_W1_N, p + PM_W1,
                     wb);
  hipLaunchKernelGGL(k_to_bf16, grid1(PM_W2_N), dim3(256), 0, c.stream, (int)PM_W2_N, p + PM_W2,
                     wb + PM_W1_N);
  hipLaunchKernelGGL(k_to_bf16, grid1(PM_W3_N), dim3(256), 0, c.stream, (int)PM_W3_N, p + PM_W3,
                     wb + PM_W1_N + PM_W2_N);
}

// scores s (N) of bf16 features Xb (N x F); activations go to the caller's arena
void PivotModel::forward(Ctx &w, const bf16_t *Xb, int N, float *s, bf16_t **H1_out,
                         bf16_t **H2_out) {
  const bf16_t *W1 = wb, *W2 = wb + PM_W1_N, *w3 = wb + PM_W1_N + PM_W2_N;
  float *Z = static_cast<float *>(w.arena.alloc((size_t)N * HID * sizeof(float)));
  bf16_t *H1 = static_cast<bf16_t *>(w.arena.alloc((size_t)N * HID * sizeof(bf16_t)));
  bf16_t *H2 = static_cast<bf16_t *>(w.arena.alloc((size_t)N * HID * sizeof(bf16_t)));
  gemm_bf16(w, N, HID, F, Xb, F, 1, W1, HID, 1, Z, HID);
  hipLaunchKernelGGL(k_bias_relu, grid1((size_t)N * HID), dim3(256), 0, w.stream, N, Z,
                     p + PM_B1, H1);
  gemm_bf16(w, N, HID, HID, H1, HID, 1, W2, HID, 1, Z, HID);
  hipLaunchKernelGGL(k_bias_relu, grid1((size_t)N * HID), dim3(256), 0, w.stream, N, Z,
                     p + PM_B2, H2);
  hipLaunchKernelGGL(k_head, dim3((N + 3) / 4), dim3(256), 0, w.stream, N, H2, w3, p + PM_B3, s);
  if (H1_out) *H1_out = H1;
  if (H2_out) *H2_out = H2;
}

// loss and gradients (into g) of a batch; returns the loss (synchronises)
double PivotModel::grad(Ctx &w, const bf16_t *Xb, const float *y, int N, double pos_weight) {
  Scope sc(w.arena);
  float *s = static_cast<float *>(w.arena.alloc((size_t)N * sizeof(float)));
  bf16_t *H1 = nullptr, *H2 = nullptr;
  forward(w, Xb, N, s, &H1, &H2);
  const bf16_t *W2 = wb + PM_W1_N, *w3 = wb + PM_W1_N + PM_W2_N;
  float *ds = static_cast<float *>(w.arena.alloc((size_t)N * sizeof(float)));
  const int nb = (N + 255) / 256;
  float *lp = static_cast<float *>(w.arena.alloc((size_t)nb * sizeof(float)));
  hipLaunchKernelGGL(k_loss_grad, dim3(nb), dim3(256), 0, w.stream, N, s, y, (float)pos_weight,
                     1.f / N, ds, lp);
  float *lsum = static_cast<float *>(w.arena.alloc(sizeof(float)));
  hipLaunchKernelGGL(k_sum_vec, dim3(1), dim3(256), 0, w.stream, nb, lp, lsum);
  // head: gw3 = H2^T ds, gb3 = sum ds
  colsum_bf16(w, N, HID, H2, ds, g + PM_W3);
  hipLaunchKernelGGL(k_sum_vec, dim3(1), dim3(256), 0, w.stream, N, ds, g + PM_B3);
  bf16_t *dH = static_cast<bf16_t *>(w.arena.alloc((size_t)N * HID * sizeof(bf16_t)));
  hipLaunchKernelGGL(k_back_head, grid1((size_t)N * HID), dim3(256), 0, w.stream, N, ds, w3, H2,
                     dH);
  // layer 2: gW2 = H1^T dH2, gb2 = colsum dH2, G = dH2 W2^T
  gemm_bf16(w, HID, HID, N, H1, 1, HID, dH, HID, 1, g + PM_W2, HID);
  colsum_bf16(w, N, HID, dH, nullptr, g + PM_B2);
  float *G = static_cast<float *>(w.arena.alloc((size_t)N * HID * sizeof(float)));
  gemm_bf16(w, N, HID, HID, dH, HID, 1, W2, 1, HID, G, HID);
  hipLaunchKernelGGL(k_relu_mask, grid1((size_t)N * HID), dim3(256), 0, w.stream, N, G, H1, dH);
  // layer 1: gW1 = X^T dH1, gb1 = colsum dH1
  gemm_bf16(w, F, HID, N, Xb, 1, F, dH, HID, 1, g + PM_W1, HID);
  colsum_bf16(w, N, HID, dH, nullptr, g + PM_B1);
  float lh = 0.f;
  HIP_CHECK(hipMemcpyAsync(&lh, lsum, sizeof(float), hipMemcpyDeviceToHost, w.stream));
  w.sync();
  return lh;
}

void PivotModel::adam(Ctx &w, double lr) {
  ++t;
  const float c1 = 1.f - std::pow(0.9f, (float)t), c2 = 1.f - std::pow(0.999f, (float)t);
  hipLaunchKernelGGL(k_adam, grid1(PM_NPARAM), dim3(256), 0, w.stream, (int)PM_NPARAM, p, g, m, v,
                     (float)lr, c1, c2);
}

void PivotModel::append(Ctx &w, const bf16_t *Xb, const int *J_dev, int nJ, int n2) {
  std::lock_guard<std::mutex> lk(mu);
  if (rows + (size_t)n2 > cap) return;                 // dataset full: drop further samples
  HIP_CHECK(hipMemcpyAsync(Xd + rows * F, Xb, (size_t)n2 * F * sizeof(bf16_t),
                           hipMemcpyDeviceToDevice, w.stream));
  std::vector<float> y(n2, 0.f);
  std::vector<int> J(nJ);
  HIP_CHECK(hipMemcpyAsync(J.data(), J_dev, nJ * sizeof(int), hipMemcpyDeviceToHost, w.stream));
  w.sync();
  for (int j : J)
    if (j >= 0 && j < n2) y[j] = 1.f;
  HIP_CHECK(hipMemcpyAsync(Yd + rows, y.data(), n2 * sizeof(float), hipMemcpyHostToDevice,
                           w.stream));
  w.sync();
  rows += n2;
  positives += nJ;
}

double PivotModel::train(int epochs, int batch, double lr) {
  std::lock_guard<std::mutex> lk(mu);
  TT_REQUIRE(rows > 0, "pivot model: no logged samples to train on");
  TT_REQUIRE(epochs >= 1 && batch >= 64, "pivot model: bad epochs / batch");
  const double pw = positives > 0 ? (double)(rows - positives) / positives : 1.0;
  // batches are contiguous slices in a seeded shuffled order of slice starts
  const int nb = (int)((rows + batch - 1) / batch);
  std::vector<int> order(nb);
  uint64_t st = 0x5EEDull + t;
  double last = 0.0;
  for (int e = 0; e < epochs; ++e) {
    for (int b = 0; b < nb; ++b) order[b] = b;
    for (int b = nb - 1; b > 0; --b) std::swap(order[b], order[sm64(st) % (uint64_t)(b + 1)]);
    double sum = 0.0;
    for (int b : order) {
      const size_t r0 = (size_t)b * batch;
      const int N = (int)std::min<size_t>(batch, rows - r0);
      sum += grad(c, Xd + r0 * F, Yd + r0, N, pw);
      adam(c, lr);
      refresh_bf16();
    }
    last = sum / nb;
  }
  c.sync();
  return last;
}

// features of all n2 column indices (f32 and/or bf16 outputs)
void pivot_features(Ctx &c, const double *B0, int n2, int r, int ldb, const int *J_dev, int nJ,
                    float *Xf, bf16_t *Xb) {
  TT_REQUIRE(nJ <= 128, "pivot features: more than 128 previous pivots");
  Scope sc(c.arena);
  double *lev = c.arena.dalloc(n2), *jump = c.arena.dalloc(n2), *nrm = c.arena.dalloc(1);
  hipLaunchKernelGGL(k_feat_rows, grid1(n2), dim3(256), 0, c.stream, B0, n2, r, ldb, lev, jump);
  hipLaunchKernelGGL(k_sum_d, dim3(1), dim3(1024), 0, c.stream, n2, lev, nrm);
  hipLaunchKernelGGL(k_features, grid1(n2), dim3(256), 0, c.stream, n2, lev, jump, nrm, J_dev,
                     nJ, Xf, Xb);
}

void to_bf16(Ctx &c, const float *x, size_t n, bf16_t *y) {
  hipLaunchKernelGGL(k_to_bf16, grid1(n), dim3(256), 0, c.stream, (int)n, x, y);
}

void topk_indices(Ctx &c, const float *s, int n, int K, int *out) {
  TT_REQUIRE(K >= 1 && K <= n, "top-k: need 1 <= K <= n");
  hipLaunchKernelGGL(k_topk, dim3(1), dim3(TKT), 0, c.stream, s, n, K, out);
}

}  // namespace ttfv
