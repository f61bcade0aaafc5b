// Tall-skinny Householder QR (TSQR) with an explicit orthonormal factor.
//
// Used by TT rounding (Section 3.2 orthogonalises the cores by QR) and by the cross
// (orthonormal column/row bases for maxvol).  The n x m panel (m <= 96) is cut into row
// blocks that fit one workgroup's LDS; each block is factorised by Householder reflections
// in LDS (LAPACK-style reflectors, R on and above the diagonal, v below it, v_0 = 1).  The
// m x m triangles are then combined `arity` at a time in a reduction tree, again by
// Householder in LDS.  The explicit Q is formed top-down: the root starts from the first m
// columns of the identity, every node applies its reflectors to its slab, and each leaf
// applies its reflectors to produce its rows of Q.  In the apply kernels each wavefront
// keeps one column of the slab in registers and runs through all reflectors (no barriers).
//
// Row blocks hold between m and 2m..bmax rows (blocks are balanced), so every block has at
// least m real rows and no padding rows enter the factorisation.
#include "common.h"
#include "wave.h"

#include <algorithm>

namespace ttfv {
namespace {

constexpr int NT = 1024;     // 16 wavefronts = 64 groups of 16 lanes (one DPP row each)
constexpr int NG = NT / 16;
constexpr int MAXROWS = 256; // rows of a block held in registers (16 lanes x RS slots)

// Layout of an (rows x m) panel in registers: column c lives in group c % 64, slot c / 64;
// row i lives in lane i % 16 of that group, slot i / 16.  A group's reductions over rows
// are 16-lane DPP all-reduces; only reflector vectors travel through LDS.

// Householder QR of the register panel x (LAPACK-style reflectors: R on and above the
// diagonal, v below it, v_j(j) = 1).  vbuf: 2 * 16 * RS doubles of LDS, taus: m doubles.
template <int RS, int CS>
__device__ void qr_regs(double (&x)[CS][RS], int rows, int m, double *vbuf, double *taus) {
  const int gid = threadIdx.x >> 4, gl = threadIdx.x & 15;
  for (int j = 0; j < m; ++j) {
    double *vb = vbuf + (j & 1) * (16 * RS);
    const int og = j % NG, os = j / NG;
    if (gid == og) {
#pragma unroll
      for (int s = 0; s < CS; ++s) {
        if (s != os) continue;
        double red[2] = {0.0, 0.0};
#pragma unroll
        for (int r = 0; r < RS; ++r) {
          const int i = gl + 16 * r;
          const double v = x[s][r];
          if (i > j && i < rows) red[0] += v * v;
          if (i == j) red[1] += v;
        }
        row16_sum_n<2>(red);
        const double ss = red[0], alpha = red[1];
        double t = 0.0, scal = 0.0, beta = alpha;
        if (ss > 0.0) {
          const double nrm = sqrt(alpha * alpha + ss);
          beta = alpha >= 0.0 ? -nrm : nrm;
          t = (beta - alpha) / beta;
          scal = 1.0 / (alpha - beta);
        }
#pragma unroll
        for (int r = 0; r < RS; ++r) {
          const int i = gl + 16 * r;
          double v = x[s][r];
          if (i > j && i < rows) v *= scal;
          if (i == j) v = beta;
          x[s][r] = v;
          vb[i] = (i > j && i < rows) ? v : (i == j ? 1.0 : 0.0);
        }
        if (gl == 0) taus[j] = t;
      }
    }
    __syncthreads();
    const double t = taus[j];
    if (t != 0.0) {
      double v[RS];
#pragma unroll
      for (int r = 0; r < RS; ++r) v[r] = vb[gl + 16 * r];
      double d[CS];
#pragma unroll
      for (int s = 0; s < CS; ++s) {
        double acc = 0.0;
#pragma unroll
        for (int r = 0; r < RS; ++r) acc += v[r] * x[s][r];
        d[s] = acc;
      }
      row16_sum_n<CS>(d);
#pragma unroll
      for (int s = 0; s < CS; ++s) {
        const int c = gid + NG * s;
        if (c <= j || c >= m) continue;
        const double du = t * d[s];
#pragma unroll
        for (int r = 0; r < RS; ++r) x[s][r] -= du * v[r];
      }
    }
  }
  __syncthreads();
}

// Apply H_0 ... H_{m-1} (V in LDS, rows x m, ld rows; taus) to the register panel x;
// reflectors run m-1 .. 0.  No barriers: V is read-only here.
template <int RS, int CS>
__device__ void apply_regs(const double *V, const double *taus, int rows, int m,
                           double (&x)[CS][RS]) {
  const int gl = threadIdx.x & 15;
  for (int j = m - 1; j >= 0; --j) {
    const double t = taus[j];
    if (t == 0.0) continue;
    const double *vj = V + (size_t)j * rows;
    double v[RS];
#pragma unroll
    for (int r = 0; r < RS; ++r) {
      const int i = gl + 16 * r;
      v[r] = (i < rows && i >= j) ? (i == j ? 1.0 : vj[i]) : 0.0;
    }
    double d[CS];
#pragma unroll
    for (int s = 0; s < CS; ++s) {
      double acc = 0.0;
#pragma unroll
      for (int r = 0; r < RS; ++r) acc += v[r] * x[s][r];
      d[s] = acc;
    }
    row16_sum_n<CS>(d);
#pragma unroll
    for (int s = 0; s < CS; ++s) {
      const double du = t * d[s];
#pragma unroll
      for (int r = 0; r < RS; ++r) x[s][r] -= du * v[r];
    }
  }
}

__device__ __forceinline__ void leaf_range(int L, int n, int nleaf, int &start, int &rows) {
  start = (int)(((long long)L * n) / nleaf);
  const int end = (int)(((long long)(L + 1) * n) / nleaf);
  rows = end - start;
}

template <int RS, int CS>
__global__ __launch_bounds__(NT) void k_leaf_qr(const double *__restrict__ Y, int n, int m,
                                                int ldy, int nleaf, int bmax,
                                                double *__restrict__ V, double *__restrict__ tau,
                                                double *__restrict__ R) {
  __shared__ double vbuf[2 * 16 * RS];
  __shared__ double taus[128];
  const int L = blockIdx.x;
  int start, rows;
  leaf_range(L, n, nleaf, start, rows);
  const int gid = threadIdx.x >> 4, gl = threadIdx.x & 15;
  double x[CS][RS];
#pragma unroll
  for (int s = 0; s < CS; ++s)
#pragma unroll
    for (int r = 0; r < RS; ++r) {
      const int c = gid + NG * s, i = gl + 16 * r;
      x[s][r] = (c < m && i < rows) ? Y[(size_t)(start + i) + (size_t)c * ldy] : 0.0;
    }
  qr_regs<RS, CS>(x, rows, m, vbuf, taus);
  double *VL = V + (size_t)L * bmax * m;
  double *RL = R + (size_t)L * m * m;
#pragma unroll
  for (int s = 0; s < CS; ++s)
#pragma unroll
    for (int r = 0; r < RS; ++r) {
      const int c = gid + NG * s, i = gl + 16 * r;
      if (c >= m) continue;
      if (i < rows) VL[i + (size_t)c * bmax] = x[s][r];
      if (i < m) RL[i + (size_t)c * m] = (i <= c) ? x[s][r] : 0.0;
    }
  for (int c = threadIdx.x; c < m; c += NT) tau[(size_t)L * m + c] = taus[c];
}

// Combine up to `arity` child triangles (m x m each) of the level below.
template <int RS, int CS>
__global__ __launch_bounds__(NT) void k_node_qr(const double *__restrict__ Rin, int cnt_in, int m,
                                                int arity, double *__restrict__ V,
                                                double *__restrict__ tau,
                                                double *__restrict__ Rout) {
  __shared__ double vbuf[2 * 16 * RS];
  __shared__ double taus[128];
  const int k = blockIdx.x;
  const int c0 = k * arity;
  const int nch = min(arity, cnt_in - c0);
  const int rows = nch * m;
  double *Ro = Rout + (size_t)k * m * m;
  if (nch == 1) {
    for (int idx = threadIdx.x; idx < m * m; idx += NT) Ro[idx] = Rin[(size_t)c0 * m * m + idx];
    return;
  }
  const int gid = threadIdx.x >> 4, gl = threadIdx.x & 15;
  double x[CS][RS];
#pragma unroll
  for (int s = 0; s < CS; ++s)
#pragma unroll
    for (int r = 0; r < RS; ++r) {
      const int c = gid + NG * s, i = gl + 16 * r;
      double v = 0.0;
      if (c < m && i < rows) {
        const int ch = i / m, ii = i - ch * m;
        v = Rin[(size_t)(c0 + ch) * m * m + ii + (size_t)c * m];
      }
      x[s][r] = v;
    }
  qr_regs<RS, CS>(x, rows, m, vbuf, taus);
  const int ldv = arity * m;
  double *Vk = V + (size_t)k * ldv * m;
#pragma unroll
  for (int s = 0; s < CS; ++s)
#pragma unroll
    for (int r = 0; r < RS; ++r) {
      const int c = gid + NG * s, i = gl + 16 * r;
      if (c >= m) continue;
      if (i < rows) Vk[i + (size_t)c * ldv] = x[s][r];
      if (i < m) Ro[i + (size_t)c * m] = (i <= c) ? x[s][r] : 0.0;
    }
  for (int c = threadIdx.x; c < m; c += NT) tau[(size_t)k * m + c] = taus[c];
}

// Top-down: slab Zin[k] (m x m) of node k -> slabs Zout[c0 .. c0+nch-1] of its children.
// Zin == nullptr means the identity slab (root).
template <int RS, int CS>
__global__ __launch_bounds__(NT) void k_node_apply(const double *__restrict__ V,
                                                   const double *__restrict__ tau, int cnt_in,
                                                   int m, int arity,
                                                   const double *__restrict__ Zin,
                                                   double *__restrict__ Zout) {
  extern __shared__ double sm[];
  const int k = blockIdx.x;
  const int c0 = k * arity;
  const int nch = min(arity, cnt_in - c0);
  const int rows = nch * m;
  if (nch == 1) {
    for (int idx = threadIdx.x; idx < m * m; idx += NT) {
      const int i = idx % m, c = idx / m;
      Zout[(size_t)c0 * m * m + idx] = Zin ? Zin[(size_t)k * m * m + idx] : (i == c ? 1.0 : 0.0);
    }
    return;
  }
  const int ldv = arity * m;
  double *Vs = sm;
  double *ts = sm + (size_t)rows * m;
  const double *Vk = V + (size_t)k * ldv * m;
  for (int idx = threadIdx.x; idx < rows * m; idx += NT) {
    const int i = idx % rows, c = idx / rows;
    Vs[i + (size_t)c * rows] = Vk[i + (size_t)c * ldv];
  }
  for (int c = threadIdx.x; c < m; c += NT) ts[c] = tau[(size_t)k * m + c];
  const int gid = threadIdx.x >> 4, gl = threadIdx.x & 15;
  double x[CS][RS];
#pragma unroll
  for (int s = 0; s < CS; ++s)
#pragma unroll
    for (int r = 0; r < RS; ++r) {
      const int c = gid + NG * s, i = gl + 16 * r;
      double v = 0.0;
      if (c < m && i < m) v = Zin ? Zin[(size_t)k * m * m + i + (size_t)c * m] : (i == c ? 1.0 : 0.0);
      x[s][r] = v;
    }
  __syncthreads();
  apply_regs<RS, CS>(Vs, ts, rows, m, x);
#pragma unroll
  for (int s = 0; s < CS; ++s)
#pragma unroll
    for (int r = 0; r < RS; ++r) {
      const int c = gid + NG * s, i = gl + 16 * r;
      if (c >= m || i >= rows) continue;
      const int ch = i / m, ii = i - ch * m;
      Zout[(size_t)(c0 + ch) * m * m + ii + (size_t)c * m] = x[s][r];
    }
}

template <int RS, int CS>
__global__ __launch_bounds__(NT) void k_leaf_apply(const double *__restrict__ V,
                                                   const double *__restrict__ tau, int n, int m,
                                                   int nleaf, int bmax,
                                                   const double *__restrict__ Z,
                                                   double *__restrict__ Q, int ldq) {
  extern __shared__ double sm[];
  const int L = blockIdx.x;
  int start, rows;
  leaf_range(L, n, nleaf, start, rows);
  double *Vs = sm;
  double *ts = sm + (size_t)rows * m;
  const double *VL = V + (size_t)L * bmax * m;
  for (int idx = threadIdx.x; idx < rows * m; idx += NT) {
    const int i = idx % rows, c = idx / rows;
    Vs[i + (size_t)c * rows] = VL[i + (size_t)c * bmax];
  }
  for (int c = threadIdx.x; c < m; c += NT) ts[c] = tau[(size_t)L * m + c];
  const int gid = threadIdx.x >> 4, gl = threadIdx.x & 15;
  double x[CS][RS];
#pragma unroll
  for (int s = 0; s < CS; ++s)
#pragma unroll
    for (int r = 0; r < RS; ++r) {
      const int c = gid + NG * s, i = gl + 16 * r;
      double v = 0.0;
      if (c < m && i < m) v = Z ? Z[(size_t)L * m * m + i + (size_t)c * m] : (i == c ? 1.0 : 0.0);
      x[s][r] = v;
    }
  __syncthreads();
  apply_regs<RS, CS>(Vs, ts, rows, m, x);
#pragma unroll
  for (int s = 0; s < CS; ++s)
#pragma unroll
    for (int r = 0; r < RS; ++r) {
      const int c = gid + NG * s, i = gl + 16 * r;
      if (c < m && i < rows) Q[(size_t)(start + i) + (size_t)c * ldq] = x[s][r];
    }
}

int g_lds_doubles = 0;

int lds_doubles() {
  if (g_lds_doubles == 0) {
    int dev = 0, v = 0;
    HIP_CHECK(hipGetDevice(&dev));
    HIP_CHECK(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    g_lds_doubles = v / 8;
  }
  return g_lds_doubles;
}

template <typename K>
void set_lds(K kern, size_t bytes) {
  HIP_CHECK(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)bytes));
}

struct Plan {
  int n, m, nleaf, bmax, arity;
  std::vector<int> cnt;
};

template <int RS, int CS>
void run_tsqr(Ctx &c, const double *Y, int ldy, const Plan &pl, double *Q, int ldq, double *R,
              int ldr) {
  const int n = pl.n, m = pl.m, nleaf = pl.nleaf, bmax = pl.bmax, arity = pl.arity;
  Scope sc(c.arena);
  double *Vleaf = c.arena.dalloc((size_t)nleaf * bmax * m);
  double *tleaf = c.arena.dalloc((size_t)nleaf * m);
  double *Rleaf = c.arena.dalloc((size_t)nleaf * m * m);
  const double mm3 = (double)m * m * m;
  {
    TimedLaunch tl(c, "tsqr_leaf_qr", 2.0 * n * m * m - 2.0 / 3.0 * mm3 * nleaf,
                   8.0 * (2.0 * n * m + (double)nleaf * m * m));
    hipLaunchKernelGGL((k_leaf_qr<RS, CS>), dim3(nleaf), dim3(NT), 0, c.stream, Y, n, m, ldy,
                       nleaf, bmax, Vleaf, tleaf, Rleaf);
  }
  const int levels = (int)pl.cnt.size() - 1;
  std::vector<double *> Vl(levels + 1, nullptr), tl(levels + 1, nullptr), Rl(levels + 1, nullptr);
  Rl[0] = Rleaf;
  for (int l = 1; l <= levels; ++l) {
    const int cout = pl.cnt[l];
    Vl[l] = c.arena.dalloc((size_t)cout * arity * m * m);
    tl[l] = c.arena.dalloc((size_t)cout * m);
    Rl[l] = c.arena.dalloc((size_t)cout * m * m);
    const double rows_l = (double)pl.cnt[l - 1] * m;
    TimedLaunch tq(c, "tsqr_node_qr", 2.0 * rows_l * m * m - 2.0 / 3.0 * mm3 * cout,
                   8.0 * (2.0 * rows_l * m + (double)cout * m * m));
    hipLaunchKernelGGL((k_node_qr<RS, CS>), dim3(cout), dim3(NT), 0, c.stream, Rl[l - 1],
                       pl.cnt[l - 1], m, arity, Vl[l], tl[l], Rl[l]);
  }
  copy_scale(c, R, ldr, Rl[levels], m, m, m, 1.0);
  size_t zmax = 0;
  for (int v : pl.cnt) zmax = std::max(zmax, (size_t)v);
  double *Z[2] = {c.arena.dalloc(zmax * m * m), c.arena.dalloc(zmax * m * m)};
  const double *Zin = nullptr;
  int which = 0;
  for (int l = levels; l >= 1; --l) {
    const size_t lds = ((size_t)arity * m * m + m) * sizeof(double);
    set_lds(k_node_apply<RS, CS>, lds);
    const double rows_l = (double)pl.cnt[l - 1] * m;
    TimedLaunch ta(c, "tsqr_node_apply", 2.0 * rows_l * m * m - 2.0 / 3.0 * mm3 * pl.cnt[l],
                   8.0 * (2.0 * rows_l * m + (double)pl.cnt[l] * m * m));
    hipLaunchKernelGGL((k_node_apply<RS, CS>), dim3(pl.cnt[l]), dim3(NT), lds, c.stream, Vl[l],
                       tl[l], pl.cnt[l - 1], m, arity, Zin, Z[which]);
    Zin = Z[which];
    which ^= 1;
  }
  const size_t lds = ((size_t)bmax * m + m) * sizeof(double);
  set_lds(k_leaf_apply<RS, CS>, lds);
  TimedLaunch tl2(c, "tsqr_leaf_apply", 2.0 * n * m * m - 2.0 / 3.0 * mm3 * nleaf,
                  8.0 * (2.0 * n * m + (double)nleaf * m * m));
  hipLaunchKernelGGL((k_leaf_apply<RS, CS>), dim3(nleaf), dim3(NT), lds, c.stream, Vleaf, tleaf,
                     n, m, nleaf, bmax, Zin, Q, ldq);
}

}  // namespace

int qr_max_cols() { return QR_MAXM; }

void tsqr(Ctx &c, const double *Y, int n, int m, int ldy, double *Q, int ldq, double *R,
          int ldr) {
  TT_REQUIRE(m >= 1 && n >= m, "tsqr: need n >= m >= 1");
  TT_REQUIRE(m <= QR_MAXM, "tsqr: more than 96 columns");
  const int d = lds_doubles();
  Plan pl;
  pl.n = n;
  pl.m = m;
  // rows per leaf: registers hold <= 256 rows; the apply kernel keeps V (rows x m) in LDS
  pl.bmax = std::min(MAXROWS, (d - 2 * m) / m);
  TT_REQUIRE(pl.bmax >= 2 * m || n <= pl.bmax, "tsqr: LDS too small for this width");
  pl.nleaf = std::max(1, (n + pl.bmax - 1) / pl.bmax);
  pl.arity = std::max(2, std::min(16, std::min(MAXROWS / m, (d - m) / (m * m))));
  pl.cnt = {pl.nleaf};
  while (pl.cnt.back() > 1) pl.cnt.push_back((pl.cnt.back() + pl.arity - 1) / pl.arity);
  const int rowsmax = std::max(std::min(pl.bmax, n), pl.nleaf > 1 ? pl.arity * m : 0);
  TT_REQUIRE(rowsmax <= MAXROWS, "tsqr: block too tall");
  const int rs = (rowsmax + 15) / 16;
  const int cs = (m + NG - 1) / NG;
  if (cs == 1) {
    if (rs <= 2) run_tsqr<2, 1>(c, Y, ldy, pl, Q, ldq, R, ldr);
    else if (rs <= 4) run_tsqr<4, 1>(c, Y, ldy, pl, Q, ldq, R, ldr);
    else if (rs <= 8) run_tsqr<8, 1>(c, Y, ldy, pl, Q, ldq, R, ldr);
    else run_tsqr<16, 1>(c, Y, ldy, pl, Q, ldq, R, ldr);
  } else {
    if (rs <= 8) run_tsqr<8, 2>(c, Y, ldy, pl, Q, ldq, R, ldr);
    else run_tsqr<16, 2>(c, Y, ldy, pl, Q, ldq, R, ldr);
  }
  c.cnt.flops += 4.0 * n * m * m;
  c.cnt.bytes += 8.0 * 3.0 * n * m;
}

}  // namespace ttfv
