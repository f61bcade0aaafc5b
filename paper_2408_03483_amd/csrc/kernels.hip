// Bandwidth-bound core kernels: stencil reconstruction on TT cores (Section 4.3.1),
// face-splitting (Hadamard) products of cores, concatenation/scaling, the Gauss-Legendre
// sum and the (T - 1) face difference (Section 4.1), column sums and helpers.
//
// Layout: every core is column-major (one rank column of n rows is contiguous), so a
// stencil along the mode index reads and writes contiguous memory; launches put the row
// index on threadIdx.x (coalesced) and the rank column on blockIdx.y.
#include "common.h"

namespace ttfv {

namespace {

constexpr int TPB = 256;

// row of cell q (in [-3, n + 3)) in a core column under a ghost rule, and the factor the
// rule applies: wrap; mirror times sign; zero (the value comes from separate boundary
// columns); or an explicitly extended column of n + 6 rows (cell q at row q + 3)
__device__ __forceinline__ int ghost_map(int q, int n, Ghost rule, double sign, double &s) {
  if (rule == Ghost::Explicit) { s = 1.0; return q + 3; }
  if (q >= 0 && q < n) { s = 1.0; return q; }
  if (rule == Ghost::Periodic) { s = 1.0; int m = q % n; return m < 0 ? m + n : m; }
  if (rule == Ghost::Zero) { s = 0.0; return 0; }
  s = sign;                                   // mirror about the wall: ghost k <-> cell k
  return q < 0 ? (-1 - q) : (2 * n - 1 - q);
}

__host__ __device__ __forceinline__ int core_ld(int n, Ghost rule) {
  return rule == Ghost::Explicit ? n + 6 : n;
}

__global__ void k_recon_face(const double *__restrict__ A, int n, Ghost rule, double sign,
                             StencilSet st, double *__restrict__ Am, double *__restrict__ Ap,
                             int nf) {
  int f = blockIdx.x * TPB + threadIdx.x;
  int c = blockIdx.y;
  if (f >= nf) return;
  const double *col = A + (size_t)c * core_ld(n, rule);
  double m = 0.0, p = 0.0;
  const int k = st.k;
  for (int o = -k; o <= k; ++o) {
    double s1, s2;
    int i1 = ghost_map(f - 1 + o, n, rule, sign, s1);   // right face of cell f-1
    int i2 = ghost_map(f - o, n, rule, sign, s2);       // left face of cell f (mirrored)
    double w = st.face[o + k];
    m += w * s1 * col[i1];
    p += w * s2 * col[i2];
  }
  Am[(size_t)c * nf + f] = m;
  Ap[(size_t)c * nf + f] = p;
}

__global__ void k_recon_quad(const double *__restrict__ B, int n, Ghost rule, double sign,
                             StencilSet st, double *__restrict__ Bq) {
  int j = blockIdx.x * TPB + threadIdx.x;
  int c = blockIdx.y;
  if (j >= n) return;
  const double *col = B + (size_t)c * core_ld(n, rule);
  const int k = st.k;
  double v[5];
  for (int o = -k; o <= k; ++o) {
    double s;
    int i = ghost_map(j + o, n, rule, sign, s);
    v[o + k] = s * col[i];
  }
  double *out = Bq + (size_t)c * n * st.nq + (size_t)j * st.nq;
  for (int m = 0; m < st.nq; ++m) {
    double acc = 0.0;
    for (int o = 0; o <= 2 * k; ++o) acc += st.quad[m][o] * v[o];
    out[m] = acc;
  }
}

__global__ void k_quad_sum(const double *__restrict__ Bq, int n, StencilSet st,
                           double *__restrict__ Bo) {
  int j = blockIdx.x * TPB + threadIdx.x;
  int c = blockIdx.y;
  if (j >= n) return;
  const double *in = Bq + (size_t)c * n * st.nq + (size_t)j * st.nq;
  double acc = 0.0;
  for (int m = 0; m < st.nq; ++m) acc += st.gw[m] * in[m];
  Bo[(size_t)c * n + j] = acc;
}

__global__ void k_face_diff(const double *__restrict__ A, int nf, int n, bool periodic,
                            double scale, double *__restrict__ Ao, int ldo) {
  int i = blockIdx.x * TPB + threadIdx.x;
  int c = blockIdx.y;
  if (i >= n) return;
  const double *col = A + (size_t)c * nf;
  int ip = periodic ? (i + 1 == nf ? 0 : i + 1) : i + 1;
  Ao[(size_t)c * ldo + i] = scale * (col[ip] - col[i]);
}

__global__ void k_ghost_extend(const double *__restrict__ A, int n, Ghost rule, double sign,
                               double *__restrict__ E) {
  int q = blockIdx.x * TPB + threadIdx.x;     // 0 .. n+5
  int c = blockIdx.y;
  if (q >= n + 6) return;
  double s;
  int i = ghost_map(q - 3, n, rule, sign, s);
  E[(size_t)c * (n + 6) + q] = s * A[(size_t)c * core_ld(n, rule) + i];
}

__global__ void k_khatri_rao(double *__restrict__ out, int n, const double *__restrict__ X,
                             int rx, const double *__restrict__ Y, int ry) {
  int i = blockIdx.x * TPB + threadIdx.x;
  int col = blockIdx.y;                       // a * ry + b
  if (i >= n) return;
  int a = col / ry, b = col - a * ry;
  out[(size_t)col * n + i] = X[(size_t)a * n + i] * Y[(size_t)b * n + i];
}

__global__ void k_copy_scale(double *__restrict__ dst, int ldd, const double *__restrict__ src,
                             int lds, int rows, double alpha) {
  int i = blockIdx.x * TPB + threadIdx.x;
  int c = blockIdx.y;
  if (i >= rows) return;
  dst[(size_t)c * ldd + i] = alpha * src[(size_t)c * lds + i];
}

__global__ void k_axpby(double *__restrict__ dst, int ldd, const double *__restrict__ x, int ldx,
                        double a, const double *__restrict__ y, int ldy, double b, int rows) {
  int i = blockIdx.x * TPB + threadIdx.x;
  int c = blockIdx.y;
  if (i >= rows) return;
  dst[(size_t)c * ldd + i] = a * x[(size_t)c * ldx + i] + b * y[(size_t)c * ldy + i];
}

__global__ void k_fill(double *__restrict__ dst, int ld, int rows, double v) {
  int i = blockIdx.x * TPB + threadIdx.x;
  int c = blockIdx.y;
  if (i >= rows) return;
  dst[(size_t)c * ld + i] = v;
}

__global__ void k_gather_rows(double *__restrict__ dst, int ldd, const double *__restrict__ src,
                              int lds, const int *__restrict__ rows, int nrows) {
  int t = blockIdx.x * TPB + threadIdx.x;
  int c = blockIdx.y;
  if (t >= nrows) return;
  dst[(size_t)c * ldd + t] = src[(size_t)c * lds + rows[t]];
}

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Gaussian test matrix for the randomized range finder: Box-Muller on hashed counters
__global__ void k_fill_gauss(double *__restrict__ O, int rows, int ld, uint64_t seed) {
  int i = blockIdx.x * TPB + threadIdx.x;
  int c = blockIdx.y;
  if (i >= rows) return;
  uint64_t idx = (uint64_t)c * (uint64_t)rows + (uint64_t)i;
  uint64_t h1 = mix64(seed ^ (idx * 2 + 1) * 0x9E3779B97F4A7C15ull);
  uint64_t h2 = mix64(h1 + 0x632BE59BD9B4E019ull);
  double u1 = ((h1 >> 11) + 1.0) * (1.0 / 9007199254740993.0);   // (0, 1]
  double u2 = (h2 >> 11) * (1.0 / 9007199254740992.0);
  O[(size_t)c * ld + i] = sqrt(-2.0 * log(u1)) * cospi(2.0 * u2);
}

// column sums: one block per column, fixed-order tree reduction (deterministic)
__global__ void k_colsum(const double *__restrict__ A, int n, int ld, double *__restrict__ out) {
  __shared__ double red[TPB];
  int c = blockIdx.x;
  const double *col = A + (size_t)c * ld;
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += TPB) acc += col[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = TPB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = red[0];
}

__global__ void k_colsumsq(const double *__restrict__ A, int n, int ld,
                           double *__restrict__ out) {
  __shared__ double red[TPB];
  int c = blockIdx.x;
  const double *col = A + (size_t)c * ld;
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += TPB) acc += col[i] * col[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = TPB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = red[0];
}

__global__ void k_transpose(double *__restrict__ dst, int ldd, const double *__restrict__ src,
                            int lds, int rows, int cols) {
  __shared__ double tile[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8 threads
  for (int k = ty; k < 32; k += 8) {
    const int i = bx + tx, j = by + k;
    tile[k][tx] = (i < rows && j < cols) ? src[i + (size_t)j * lds] : 0.0;
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int j = by + tx, i = bx + k;     // dst(j, i) = src(i, j)
    if (i < rows && j < cols) dst[j + (size_t)i * ldd] = tile[tx][k];
  }
}

inline dim3 grid2(int rows, int cols) { return dim3((rows + TPB - 1) / TPB, cols); }

}  // namespace

void recon_face(Ctx &c, const double *A, int n, int r, Ghost rule, double sign,
                const StencilSet &st, double *Am, double *Ap, int nf) {
  if (r <= 0 || nf <= 0) return;
  hipLaunchKernelGGL(k_recon_face, grid2(nf, r), dim3(TPB), 0, c.stream, A, n, rule, sign,
                     st, Am, Ap, nf);
  c.cnt.flops += 4.0 * (2 * st.k + 1) * nf * r;
  c.cnt.bytes += 8.0 * r * (n + 2.0 * nf);
}

void recon_quad(Ctx &c, const double *B, int n, int r, Ghost rule, double sign,
                const StencilSet &st, double *Bq) {
  if (r <= 0) return;
  hipLaunchKernelGGL(k_recon_quad, grid2(n, r), dim3(TPB), 0, c.stream, B, n, rule, sign, st,
                     Bq);
  c.cnt.flops += 2.0 * (2 * st.k + 1) * st.nq * n * r;
  c.cnt.bytes += 8.0 * r * n * (1.0 + st.nq);
}

void quad_sum(Ctx &c, const double *Bq, int n, int nq, int r, const StencilSet &st, double *Bo) {
  if (r <= 0) return;
  hipLaunchKernelGGL(k_quad_sum, grid2(n, r), dim3(TPB), 0, c.stream, Bq, n, st, Bo);
  c.cnt.flops += 2.0 * nq * n * r;
  c.cnt.bytes += 8.0 * r * n * (1.0 + nq);
}

void face_diff(Ctx &c, const double *A, int nf, int n, int r, bool periodic, double scale,
               double *Ao, int ldo) {
  if (r <= 0) return;
  hipLaunchKernelGGL(k_face_diff, grid2(n, r), dim3(TPB), 0, c.stream, A, nf, n, periodic, scale,
                     Ao, ldo);
  c.cnt.bytes += 8.0 * r * (nf + n);
}

void ghost_extend(Ctx &c, const double *A, int n, int r, Ghost rule, double sign, double *E) {
  if (r <= 0) return;
  hipLaunchKernelGGL(k_ghost_extend, grid2(n + 6, r), dim3(TPB), 0, c.stream, A, n, rule,
                     sign, E);
}

void khatri_rao(Ctx &c, double *out, int n, const double *X, int rx, const double *Y, int ry) {
  if (rx * ry <= 0) return;
  hipLaunchKernelGGL(k_khatri_rao, grid2(n, rx * ry), dim3(TPB), 0, c.stream, out, n, X, rx, Y,
                     ry);
  c.cnt.flops += 1.0 * n * rx * ry;
  c.cnt.bytes += 8.0 * n * (rx + ry + (double)rx * ry);
}

void copy_scale(Ctx &c, double *dst, int ldd, const double *src, int lds, int rows, int cols,
                double alpha) {
  if (rows <= 0 || cols <= 0) return;
  hipLaunchKernelGGL(k_copy_scale, grid2(rows, cols), dim3(TPB), 0, c.stream, dst, ldd, src, lds,
                     rows, alpha);
}

void axpby(Ctx &c, double *dst, int ldd, const double *x, int ldx, double a, const double *y,
           int ldy, double b, int rows, int cols) {
  if (rows <= 0 || cols <= 0) return;
  hipLaunchKernelGGL(k_axpby, grid2(rows, cols), dim3(TPB), 0, c.stream, dst, ldd, x, ldx, a, y,
                     ldy, b, rows);
}

void fill_value(Ctx &c, double *dst, int ld, int rows, int cols, double v) {
  if (rows <= 0 || cols <= 0) return;
  hipLaunchKernelGGL(k_fill, grid2(rows, cols), dim3(TPB), 0, c.stream, dst, ld, rows, v);
}

void gather_rows(Ctx &c, double *dst, int ldd, const double *src, int lds, const int *rows_dev,
                 int nrows, int cols) {
  if (nrows <= 0 || cols <= 0) return;
  hipLaunchKernelGGL(k_gather_rows, grid2(nrows, cols), dim3(TPB), 0, c.stream, dst, ldd, src,
                     lds, rows_dev, nrows);
}

void transpose(Ctx &c, double *dst, int ldd, const double *src, int lds, int rows, int cols) {
  if (rows <= 0 || cols <= 0) return;
  hipLaunchKernelGGL(k_transpose, dim3((rows + 31) / 32, (cols + 31) / 32), dim3(256), 0, c.stream,
                     dst, ldd, src, lds, rows, cols);
}

void fill_gauss(Ctx &c, double *O, int rows, int cols, int ld, uint64_t seed) {
  if (rows <= 0 || cols <= 0) return;
  hipLaunchKernelGGL(k_fill_gauss, grid2(rows, cols), dim3(TPB), 0, c.stream, O, rows, ld, seed);
}

void colsum(Ctx &c, const double *A, int n, int r, int ld, double *out) {
  if (r <= 0) return;
  hipLaunchKernelGGL(k_colsum, dim3(r), dim3(TPB), 0, c.stream, A, n, ld, out);
}

void colsumsq(Ctx &c, const double *A, int n, int r, int ld, double *out) {
  if (r <= 0) return;
  hipLaunchKernelGGL(k_colsumsq, dim3(r), dim3(TPB), 0, c.stream, A, n, ld, out);
  c.cnt.bytes += 8.0 * n * r;
}

}  // namespace ttfv
