// Cross interpolation kernels (Section 3.3): maxvol row selection and fiber evaluation.
//
// maxvol (Goreinov et al., cited in Section 3.3) on an orthonormal basis Q (n x r):
//   start: greedy rows -- repeatedly the row of largest residual norm, whose direction is
//          then projected out of every row (a pivoted QR of Q^T); for an orthonormal basis
//          this start does not depend on which basis of the column space is given.  One
//          launch per chosen row spreads the n x r residual over all CUs;
//   swaps: B = Q Q[I]^-1; while max |B_ij| > tau, row i replaces the j-th chosen row and B
//          gets the rank-one correction B -= B(:,j) (B(i,:) - e_j) / B_ij.
//   Ties in every argmax go to the smallest row, then the smallest column.
// Fibers: the entries of the matrix being interpolated are pointwise functions of one or
// more TTs, evaluated as rank-r dot products of core rows (with ghost-extended cores for
// the shifted WENO stencils), so a column or row fiber never materialises a full field.
#include "common.h"
#include "weno.h"

#include <algorithm>

namespace ttfv {
namespace {

constexpr int NT = 1024;

struct Best {
  double v;
  int i, j;
};

__device__ __forceinline__ bool better(const Best &a, const Best &b) {
  if (a.v != b.v) return a.v > b.v;
  if (a.i != b.i) return a.i < b.i;
  return a.j < b.j;
}

__device__ __forceinline__ Best wave_best(Best b) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    Best o;
    o.v = __shfl_xor(b.v, off, 64);
    o.i = __shfl_xor(b.i, off, 64);
    o.j = __shfl_xor(b.j, off, 64);
    if (better(o, b)) b = o;
  }
  return b;
}

// argmax over the block under the total order `better` (so the result is unique)
__device__ Best block_best(Best b, Best *red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  b = wave_best(b);
  if (lane == 0) red[wave] = b;
  __syncthreads();
  if (wave == 0) {
    Best x = lane < NT / 64 ? red[lane] : Best{-1.0, 0x7fffffff, 0x7fffffff};
    x = wave_best(x);
    if (lane == 0) red[NT / 64] = x;
  }
  __syncthreads();
  Best r = red[NT / 64];
  __syncthreads();
  return r;
}

// Greedy start, one launch per chosen row over all CUs: each block owns GB rows of R (the
// residual of Q, updated in place) and publishes its best row (squared residual norm,
// index, and the row itself) into a double-buffered candidate table.  The next launch picks
// the winner among the block candidates (largest norm, then smallest row), normalises its
// row to v, projects v out of every owned row and publishes new candidates.  Every row
// update and norm is summed in the same order as a single-block sweep would.
constexpr int GB = 256;

__device__ Best block_best_gb(Best b, Best *red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  b = wave_best(b);
  if (lane == 0) red[wave] = b;
  __syncthreads();
  if (wave == 0) {
    Best x = lane < GB / 64 ? red[lane] : Best{-1.0, 0x7fffffff, 0x7fffffff};
    x = wave_best(x);
    if (lane == 0) red[GB / 64] = x;
  }
  __syncthreads();
  return red[GB / 64];
}

__global__ __launch_bounds__(GB) void k_greedy_init(const double *__restrict__ R, int n, int r,
                                                    int ldr, double *__restrict__ cval,
                                                    int *__restrict__ cidx,
                                                    double *__restrict__ cvec) {
  __shared__ Best red[GB / 64 + 1];
  const int i = blockIdx.x * GB + threadIdx.x;
  Best b{-1.0, n, 0};
  if (i < n) {
    double s = 0.0;
    for (int c = 0; c < r; ++c) {
      const double x = R[i + (size_t)c * ldr];
      s += x * x;
    }
    b = Best{s, i, 0};
  }
  const Best w = block_best_gb(b, red);
  if (threadIdx.x == 0) {
    cval[blockIdx.x] = w.v;
    cidx[blockIdx.x] = w.i;
  }
  for (int c = threadIdx.x; c < r; c += GB) cvec[(size_t)blockIdx.x * r + c] = R[w.i + (size_t)c * ldr];
}

template <int MAXR>
__global__ __launch_bounds__(GB) void k_greedy_step(double *__restrict__ R, int n, int r, int ldr,
                                                    int nblk, int t,
                                                    const double *__restrict__ cval_in,
                                                    const int *__restrict__ cidx_in,
                                                    const double *__restrict__ cvec_in,
                                                    double *__restrict__ cval_out,
                                                    int *__restrict__ cidx_out,
                                                    double *__restrict__ cvec_out,
                                                    int *__restrict__ rows_dev) {
  __shared__ Best red[GB / 64 + 1];
  __shared__ double v[128];
  __shared__ Best win;
  if (threadIdx.x < 64) {
    Best b{-1.0, 0x7fffffff, 0x7fffffff};
    for (int k = threadIdx.x; k < nblk; k += 64) {
      const Best cand{cval_in[k], cidx_in[k], k};
      if (better(cand, b)) b = cand;
    }
    b = wave_best(b);
    if (threadIdx.x == 0) win = b;
  }
  __syncthreads();
  const Best w = win;
  const double inv = w.v > 0.0 ? 1.0 / sqrt(w.v) : 0.0;
  for (int c = threadIdx.x; c < r; c += GB) v[c] = cvec_in[(size_t)w.j * r + c] * inv;
  if (blockIdx.x == 0 && threadIdx.x == 0) rows_dev[t] = w.i;
  __syncthreads();
  const int i = blockIdx.x * GB + threadIdx.x;
  Best b{-1.0, n, 0};
  if (i < n) {
    double x[MAXR];                          // the row stays in registers between the passes
#pragma unroll
    for (int c = 0; c < MAXR; ++c) x[c] = c < r ? R[i + (size_t)c * ldr] : 0.0;
    double d = 0.0;
#pragma unroll
    for (int c = 0; c < MAXR; ++c)
      if (c < r) d += x[c] * v[c];
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < MAXR; ++c) {
      if (c >= r) continue;
      x[c] = x[c] - d * v[c];
      R[i + (size_t)c * ldr] = x[c];
      s += x[c] * x[c];
    }
    b = Best{s, i, 0};
  }
  const Best bb = block_best_gb(b, red);   // its barrier also publishes the row updates
  if (threadIdx.x == 0) {
    cval_out[blockIdx.x] = bb.v;
    cidx_out[blockIdx.x] = bb.i;
  }
  for (int c = threadIdx.x; c < r; c += GB)
    cvec_out[(size_t)blockIdx.x * r + c] = R[bb.i + (size_t)c * ldr];
}

// swap iterations on B = Q Q[I]^-1 (n x r, ld n)
__global__ __launch_bounds__(NT) void k_maxvol_swaps(double *__restrict__ B, int n, int r,
                                                     double tau, int maxit,
                                                     int *__restrict__ rows_dev) {
  __shared__ Best red[NT / 64 + 1];
  __shared__ double bi[128];
  for (int it = 0; it < maxit; ++it) {
    Best b{-1.0, n, r};
    for (int i = threadIdx.x; i < n; i += NT)
      for (int c = 0; c < r; ++c) {
        Best cand{fabs(B[i + (size_t)c * n]), i, c};
        if (better(cand, b)) b = cand;
      }
    Best w = block_best(b, red);
    if (w.v <= tau) break;
    const int is = w.i, js = w.j;
    const double piv = B[is + (size_t)js * n];
    for (int c = threadIdx.x; c < r; c += NT)
      bi[c] = (B[is + (size_t)c * n] - (c == js ? 1.0 : 0.0)) / piv;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += NT) {
      const double bj = B[i + (size_t)js * n];
      for (int c = 0; c < r; ++c) B[i + (size_t)c * n] -= bj * bi[c];
    }
    if (threadIdx.x == 0) rows_dev[js] = is;
    __syncthreads();
  }
}

// --- pointwise functions -----------------------------------------------------------------

__device__ __forceinline__ double dotrow(const double *A, int lda, int ia, const double *B,
                                         int ldb, int ib, int r) {
  double s = 0.0;
  for (int a = 0; a < r; ++a) s += A[ia + (size_t)a * lda] * B[ib + (size_t)a * ldb];
  return s;
}

struct FibArgs {
  int fn, n_in;
  FiberInput in[6];
  double g;
  int nq, ncol;
};

__device__ double fiber_entry(const FibArgs &f, const WenoArgs &w, int i, int j) {
  switch (f.fn) {
    case TT_FN_IDENTITY:
      return dotrow(f.in[0].A, f.in[0].lda, i, f.in[0].B, f.in[0].ldb, j, f.in[0].r);
    case TT_FN_RECIP:
      return 1.0 / dotrow(f.in[0].A, f.in[0].lda, i, f.in[0].B, f.in[0].ldb, j, f.in[0].r);
    case TT_FN_LLF_LAMBDA: {
      double x[4];
      for (int t = 0; t < 4; ++t)
        x[t] = dotrow(f.in[t].A, f.in[t].lda, i, f.in[t].B, f.in[t].ldb, j, f.in[t].r);
      const double lm = fabs(x[1] / x[0]) + sqrt(f.g * x[0]);
      const double lp = fabs(x[3] / x[2]) + sqrt(f.g * x[2]);
      return fmax(lm, lp);
    }
    case TT_FN_LLF_FLUX: {
      // column j = component * ncol + quadrature column; states (h, m, t) minus then plus
      const int comp = j / f.ncol, jj = j - comp * f.ncol;
      double x[6];
      for (int t = 0; t < 6; ++t)
        x[t] = dotrow(f.in[t].A, f.in[t].lda, i, f.in[t].B, f.in[t].ldb, jj, f.in[t].r);
      const double hm = x[0], mm = x[1], tm = x[2], hp = x[3], mp = x[4], tp = x[5];
      const double lam = fmax(fabs(mm / hm) + sqrt(f.g * hm), fabs(mp / hp) + sqrt(f.g * hp));
      double fm, fp, um, up;
      if (comp == 0) {
        fm = mm; fp = mp; um = hm; up = hp;
      } else if (comp == 1) {
        fm = mm * mm / hm + 0.5 * f.g * hm * hm;
        fp = mp * mp / hp + 0.5 * f.g * hp * hp;
        um = mm; up = mp;
      } else {
        fm = mm * tm / hm; fp = mp * tp / hp; um = tm; up = tp;
      }
      return 0.5 * (fm + fp) - 0.5 * lam * (up - um);
    }
    case TT_FN_WENO_FACE_M:
    case TT_FN_WENO_FACE_P: {
      // first core ghost-extended by 3 rows: cell q is row q + 3
      double v[5];
      for (int o = -2; o <= 2; ++o) {
        const int cell = (f.fn == TT_FN_WENO_FACE_M) ? (i - 1 + o) : (i - o);
        v[o + 2] = dotrow(f.in[0].A, f.in[0].lda, cell + 3, f.in[0].B, f.in[0].ldb, j, f.in[0].r);
      }
      return weno_face(w, v);
    }
    case TT_FN_WENO_QUAD: {
      // second core ghost-extended by 3 rows; column j = cell * nq + point
      const int cell = j / f.nq, m = j - cell * f.nq;
      double v[5];
      for (int o = -2; o <= 2; ++o)
        v[o + 2] = dotrow(f.in[0].A, f.in[0].lda, i, f.in[0].B, f.in[0].ldb, cell + o + 3,
                          f.in[0].r);
      return weno_quad(w, v, m);
    }
  }
  return 0.0;
}

__global__ void k_fiber_cols(FibArgs f, WenoArgs w, int n1, const int *__restrict__ J, int nj,
                             double *__restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int t = blockIdx.y;
  if (i >= n1 || t >= nj) return;
  out[i + (size_t)t * n1] = fiber_entry(f, w, i, J[t]);
}

__global__ void k_fiber_rows(FibArgs f, WenoArgs w, int n2, const int *__restrict__ I, int ni,
                             double *__restrict__ outT) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int t = blockIdx.y;
  if (j >= n2 || t >= ni) return;
  outT[j + (size_t)t * n2] = fiber_entry(f, w, I[t], j);
}

FibArgs make_args(const FiberSpec &fs) {
  FibArgs a{};
  a.fn = fs.fn;
  a.n_in = fs.n_in;
  for (int t = 0; t < 6; ++t) a.in[t] = fs.in[t];
  a.g = fs.g;
  a.nq = fs.nq;
  a.ncol = fs.ncol;
  return a;
}

WenoArgs make_weno(const FiberSpec &fs) {
  WenoArgs w{};
  if (fs.wt) w.t = *fs.wt;
  w.eps = fs.eps_w;
  return w;
}

double fiber_cost(const FiberSpec &fs) {
  double r = 0;
  for (int t = 0; t < fs.n_in; ++t) r += fs.in[t].r;
  if (fs.fn == TT_FN_WENO_FACE_M || fs.fn == TT_FN_WENO_FACE_P || fs.fn == TT_FN_WENO_QUAD)
    return 2.0 * 5 * r + 70.0;
  return 2.0 * r + 10.0;
}

}  // namespace

void maxvol_dev(Ctx &c, const double *Q, int n, int r, int ldq, double tau, int maxit,
                int *rows_dev, const int *k_dev) {
  TT_REQUIRE(r >= 1 && r <= 96 && n >= r, "maxvol: need n >= r, 1 <= r <= 96");
  Scope sc(c.arena);
  double *R = c.arena.dalloc((size_t)n * r);
  copy_scale(c, R, n, Q, ldq, n, r, 1.0);
  {
    const int nblk = (n + GB - 1) / GB;
    double *cval = c.arena.dalloc(2 * (size_t)nblk);
    int *cidx = c.arena.ialloc(2 * (size_t)nblk);
    double *cvec = c.arena.dalloc(2 * (size_t)nblk * r);
    hipLaunchKernelGGL(k_greedy_init, dim3(nblk), dim3(GB), 0, c.stream, R, n, r, n, cval, cidx,
                       cvec);
    auto step = r <= 32 ? k_greedy_step<32> : r <= 64 ? k_greedy_step<64> : k_greedy_step<96>;
    for (int t = 0; t < r; ++t) {
      const int pi = t & 1, po = pi ^ 1;
      hipLaunchKernelGGL(step, dim3(nblk), dim3(GB), 0, c.stream, R, n, r, n, nblk, t,
                         cval + pi * nblk, cidx + pi * nblk, cvec + (size_t)pi * nblk * r,
                         cval + po * nblk, cidx + po * nblk, cvec + (size_t)po * nblk * r,
                         rows_dev);
    }
  }
  // B = Q Q[I]^-1
  double *QI = c.arena.dalloc((size_t)r * r);
  double *QIinv = c.arena.dalloc((size_t)r * r);
  double *B = c.arena.dalloc((size_t)n * r);
  gather_rows(c, QI, r, Q, ldq, rows_dev, r, r);
  // with zero columns from *k_dev on, Q[I] is completed by the identity outside its leading
  // block: B keeps those columns zero, so the swaps never touch them
  if (k_dev) qi_pad(c, QI, r, k_dev);
  small_inverse(c, QI, r, r, QIinv);
  gemm(c, false, n, r, r, 1.0, Q, ldq, QIinv, r, 0.0, B, n);
  hipLaunchKernelGGL(k_maxvol_swaps, dim3(1), dim3(NT), 0, c.stream, B, n, r, tau, maxit,
                     rows_dev);
  c.cnt.flops += 3.0 * n * r * r;
}

void fiber_cols(Ctx &c, const FiberSpec &fs, int n1, const int *J_dev, int nj, double *out) {
  if (nj <= 0) return;
  hipLaunchKernelGGL(k_fiber_cols, dim3((n1 + 255) / 256, nj), dim3(256), 0, c.stream,
                     make_args(fs), make_weno(fs), n1, J_dev, nj, out);
  c.cnt.flops += fiber_cost(fs) * n1 * nj;
  c.cnt.bytes += 8.0 * n1 * nj;
}

void fiber_rows(Ctx &c, const FiberSpec &fs, int n2, const int *I_dev, int ni, double *outT) {
  if (ni <= 0) return;
  hipLaunchKernelGGL(k_fiber_rows, dim3((n2 + 255) / 256, ni), dim3(256), 0, c.stream,
                     make_args(fs), make_weno(fs), n2, I_dev, ni, outT);
  c.cnt.flops += fiber_cost(fs) * n2 * ni;
  c.cnt.bytes += 8.0 * n2 * ni;
}

}  // namespace ttfv
