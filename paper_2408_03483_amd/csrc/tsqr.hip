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
template <typename T, int RS, int CS>
__device__ void qr_regs(T (&x)[CS][RS], int rows, int m, T *vbuf, T *taus) {
  const int gid = threadIdx.x >> 4, gl = threadIdx.x & 15;
  for (int j = 0; j < m; ++j) {
    T *vb = vbuf + (j & 1) * (16 * RS);
    const int og = j % NG, os = j / NG;
    if (gid == og) {
#pragma unroll
      for (int s = 0; s < CS; ++s) {
        if (s != os) continue;
        T red[2] = {T(0), T(0)};
#pragma unroll
        for (int r = 0; r < RS; ++r) {
          const int i = gl + 16 * r;
          const T v = x[s][r];
          if (i > j && i < rows) red[0] += v * v;
          if (i == j) red[1] += v;
        }
        row16_sum_n<2>(red);
        const T ss = red[0], alpha = red[1];
        T t = T(0), scal = T(0), beta = alpha;
        if (ss > T(0)) {
          const T nrm = sqrt(alpha * alpha + ss);
          beta = alpha >= T(0) ? -nrm : nrm;
          t = (beta - alpha) / beta;
          scal = T(1) / (alpha - beta);
        }
#pragma unroll
        for (int r = 0; r < RS; ++r) {
          const int i = gl + 16 * r;
          T v = x[s][r];
          if (i > j && i < rows) v *= scal;
          if (i == j) v = beta;
          x[s][r] = v;
          vb[i] = (i > j && i < rows) ? v : (i == j ? T(1) : T(0));
        }
        if (gl == 0) taus[j] = t;
      }
    }
    __syncthreads();
    const T t = taus[j];
    // groups holding no column right of j have nothing to update
    bool active = false;
#pragma unroll
    for (int s = 0; s < CS; ++s) {
      const int c = gid + NG * s;
      active = active || (c > j && c < m);
    }
    if (t != T(0) && active) {
      T v[RS];
#pragma unroll
      for (int r = 0; r < RS; ++r) v[r] = vb[gl + 16 * r];
      T d[CS];
#pragma unroll
      for (int s = 0; s < CS; ++s) {
        T acc = T(0);
#pragma unroll
        for (int r = 0; r < RS; ++r) acc += v[r] * x[s][r];
        d[s] = acc;
      }
      row16_sum_n<CS>(d);
#pragma unroll
      for (int s = 0; s < CS; ++s) {
        const int c = gid + NG * s;
        if (c <= j || c >= m) continue;
        const T du = t * d[s];
#pragma unroll
        for (int r = 0; r < RS; ++r) x[s][r] -= du * v[r];
      }
    }
  }
  __syncthreads();
}

// Apply H_0 ... H_{m-1} (V in LDS, rows x m, ld rows; taus) to the register panel x;
// reflectors run m-1 .. 0.  No barriers: V is read-only here.
template <typename T, int RS, int CS>
__device__ void apply_regs(const T *V, const T *taus, int rows, int m, T (&x)[CS][RS]) {
  const int gl = threadIdx.x & 15;
  for (int j = m - 1; j >= 0; --j) {
    const T t = taus[j];
    if (t == T(0)) continue;
    const T *vj = V + (size_t)j * rows;
    T v[RS];
#pragma unroll
    for (int r = 0; r < RS; ++r) {
      const int i = gl + 16 * r;
      v[r] = (i < rows && i >= j) ? (i == j ? T(1) : vj[i]) : T(0);
    }
    T d[CS];
#pragma unroll
    for (int s = 0; s < CS; ++s) {
      T acc = T(0);
#pragma unroll
      for (int r = 0; r < RS; ++r) acc += v[r] * x[s][r];
      d[s] = acc;
    }
    row16_sum_n<CS>(d);
#pragma unroll
    for (int s = 0; s < CS; ++s) {
      const T du = t * d[s];
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

template <typename T, int RS, int CS>
__global__ __launch_bounds__(NT) void k_leaf_qr(const double *__restrict__ Y, int n, int m,
                                                int ldy, int nleaf, int bmax,
                                                T *__restrict__ V, T *__restrict__ tau,
                                                T *__restrict__ R, double *__restrict__ Rfin,
                                                int ldr) {
  __shared__ T vbuf[2 * 16 * RS];
  __shared__ T taus[128];
  const int L = blockIdx.x;
  int start, rows;
  leaf_range(L, n, nleaf, start, rows);
  const int gid = threadIdx.x >> 4, gl = threadIdx.x & 15;
  T x[CS][RS];
#pragma unroll
  for (int s = 0; s < CS; ++s)
#pragma unroll
    for (int r = 0; r < RS; ++r) {
      const int c = gid + NG * s, i = gl + 16 * r;
      x[s][r] = (c < m && i < rows) ? T(Y[(size_t)(start + i) + (size_t)c * ldy]) : T(0);
    }
  qr_regs<T, RS, CS>(x, rows, m, vbuf, taus);
  T *VL = V + (size_t)L * bmax * m;
  T *RL = R + (size_t)L * m * m;
#pragma unroll
  for (int s = 0; s < CS; ++s)
#pragma unroll
    for (int r = 0; r < RS; ++r) {
      const int c = gid + NG * s, i = gl + 16 * r;
      if (c >= m) continue;
      if (i < rows) VL[i + (size_t)c * bmax] = x[s][r];
      if (i < m) RL[i + (size_t)c * m] = (i <= c) ? x[s][r] : T(0);
      if (Rfin && i < m) Rfin[i + (size_t)c * ldr] = (i <= c) ? (double)x[s][r] : 0.0;
    }
  for (int c = threadIdx.x; c < m; c += NT) tau[(size_t)L * m + c] = taus[c];
}

// Combine up to `arity` child triangles (m x m each) of the level below.
template <typename T, int RS, int CS>
__global__ __launch_bounds__(NT) void k_node_qr(const T *__restrict__ Rin, int cnt_in, int m,
                                                int arity, T *__restrict__ V,
                                                T *__restrict__ tau, T *__restrict__ Rout,
                                                double *__restrict__ Rfin, int ldr) {
  __shared__ T vbuf[2 * 16 * RS];
  __shared__ T taus[128];
  const int k = blockIdx.x;
  const int c0 = k * arity;
  const int nch = min(arity, cnt_in - c0);
  const int rows = nch * m;
  T *Ro = Rout + (size_t)k * m * m;
  if (nch == 1) {
    for (int idx = threadIdx.x; idx < m * m; idx += NT) {
      const T v = Rin[(size_t)c0 * m * m + idx];
      Ro[idx] = v;
      if (Rfin) Rfin[(idx % m) + (size_t)(idx / m) * ldr] = (double)v;
    }
    return;
  }
  const int gid = threadIdx.x >> 4, gl = threadIdx.x & 15;
  T x[CS][RS];
#pragma unroll
  for (int s = 0; s < CS; ++s)
#pragma unroll
    for (int r = 0; r < RS; ++r) {
      const int c = gid + NG * s, i = gl + 16 * r;
      T v = T(0);
      if (c < m && i < rows) {
        const int ch = i / m, ii = i - ch * m;
        v = Rin[(size_t)(c0 + ch) * m * m + ii + (size_t)c * m];
      }
      x[s][r] = v;
    }
  qr_regs<T, RS, CS>(x, rows, m, vbuf, taus);
  const int ldv = arity * m;
  T *Vk = V + (size_t)k * ldv * m;
#pragma unroll
  for (int s = 0; s < CS; ++s)
#pragma unroll
    for (int r = 0; r < RS; ++r) {
      const int c = gid + NG * s, i = gl + 16 * r;
      if (c >= m) continue;
      if (i < rows) Vk[i + (size_t)c * ldv] = x[s][r];
      if (i < m) Ro[i + (size_t)c * m] = (i <= c) ? x[s][r] : T(0);
      if (Rfin && i < m) Rfin[i + (size_t)c * ldr] = (i <= c) ? (double)x[s][r] : 0.0;
    }
  for (int c = threadIdx.x; c < m; c += NT) tau[(size_t)k * m + c] = taus[c];
}

// Top-down: slab Zin[k] (m x m) of node k -> slabs Zout[c0 .. c0+nch-1] of its children.
// Zin == nullptr means the identity slab (root).
template <typename T, int RS, int CS>
__global__ __launch_bounds__(NT) void k_node_apply(const T *__restrict__ V,
                                                   const T *__restrict__ tau, int cnt_in,
                                                   int m, int arity, const T *__restrict__ Zin,
                                                   T *__restrict__ Zout) {
  extern __shared__ __align__(8) unsigned char smraw[];
  T *sm = reinterpret_cast<T *>(smraw);
  const int k = blockIdx.x;
  const int c0 = k * arity;
  const int nch = min(arity, cnt_in - c0);
  const int rows = nch * m;
  if (nch == 1) {
    for (int idx = threadIdx.x; idx < m * m; idx += NT) {
      const int i = idx % m, c = idx / m;
      Zout[(size_t)c0 * m * m + idx] = Zin ? Zin[(size_t)k * m * m + idx] : T(i == c ? 1 : 0);
    }
    return;
  }
  const int ldv = arity * m;
  T *Vs = sm;
  T *ts = sm + (size_t)rows * m;
  const T *Vk = V + (size_t)k * ldv * m;
  for (int idx = threadIdx.x; idx < rows * m; idx += NT) {
    const int i = idx % rows, c = idx / rows;
    Vs[i + (size_t)c * rows] = Vk[i + (size_t)c * ldv];
  }
  for (int c = threadIdx.x; c < m; c += NT) ts[c] = tau[(size_t)k * m + c];
  const int gid = threadIdx.x >> 4, gl = threadIdx.x & 15;
  T x[CS][RS];
#pragma unroll
  for (int s = 0; s < CS; ++s)
#pragma unroll
    for (int r = 0; r < RS; ++r) {
      const int c = gid + NG * s, i = gl + 16 * r;
      T v = T(0);
      if (c < m && i < m) v = Zin ? Zin[(size_t)k * m * m + i + (size_t)c * m] : T(i == c ? 1 : 0);
      x[s][r] = v;
    }
  __syncthreads();
  apply_regs<T, RS, CS>(Vs, ts, rows, m, x);
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

template <typename T, int RS, int CS>
__global__ __launch_bounds__(NT) void k_leaf_apply(const T *__restrict__ V,
                                                   const T *__restrict__ tau, int n, int m,
                                                   int nleaf, int bmax, const T *__restrict__ Z,
                                                   double *__restrict__ Q, int ldq) {
  extern __shared__ __align__(8) unsigned char smraw[];
  T *sm = reinterpret_cast<T *>(smraw);
  const int L = blockIdx.x;
  int start, rows;
  leaf_range(L, n, nleaf, start, rows);
  T *Vs = sm;
  T *ts = sm + (size_t)rows * m;
  const T *VL = V + (size_t)L * bmax * m;
  for (int idx = threadIdx.x; idx < rows * m; idx += NT) {
    const int i = idx % rows, c = idx / rows;
    Vs[i + (size_t)c * rows] = VL[i + (size_t)c * bmax];
  }
  for (int c = threadIdx.x; c < m; c += NT) ts[c] = tau[(size_t)L * m + c];
  const int gid = threadIdx.x >> 4, gl = threadIdx.x & 15;
  T x[CS][RS];
#pragma unroll
  for (int s = 0; s < CS; ++s)
#pragma unroll
    for (int r = 0; r < RS; ++r) {
      const int c = gid + NG * s, i = gl + 16 * r;
      T v = T(0);
      if (c < m && i < m) v = Z ? Z[(size_t)L * m * m + i + (size_t)c * m] : T(i == c ? 1 : 0);
      x[s][r] = v;
    }
  __syncthreads();
  apply_regs<T, RS, CS>(Vs, ts, rows, m, x);
#pragma unroll
  for (int s = 0; s < CS; ++s)
#pragma unroll
    for (int r = 0; r < RS; ++r) {
      const int c = gid + NG * s, i = gl + 16 * r;
      if (c < m && i < rows) Q[(size_t)(start + i) + (size_t)c * ldq] = double(x[s][r]);
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

template <typename T, int RS, int CS>
void run_tsqr(Ctx &c, const double *Y, int ldy, const Plan &pl, double *Q, int ldq, double *R,
              int ldr) {
  const int n = pl.n, m = pl.m, nleaf = pl.nleaf, bmax = pl.bmax, arity = pl.arity;
  Scope sc(c.arena);
  auto talloc = [&](size_t k) { return reinterpret_cast<T *>(c.arena.alloc(k * sizeof(T))); };
  T *Vleaf = talloc((size_t)nleaf * bmax * m);
  T *tleaf = talloc((size_t)nleaf * m);
  T *Rleaf = talloc((size_t)nleaf * m * m);
  const double mm3 = (double)m * m * m;
  {
    TimedLaunch tl(c, "tsqr_leaf_qr", 2.0 * n * m * m - 2.0 / 3.0 * mm3 * nleaf,
                   8.0 * (2.0 * n * m + (double)nleaf * m * m));
    hipLaunchKernelGGL((k_leaf_qr<T, RS, CS>), dim3(nleaf), dim3(NT), 0, c.stream, Y, n, m, ldy,
                       nleaf, bmax, Vleaf, tleaf, Rleaf, nleaf == 1 ? R : nullptr, ldr);
  }
  const int levels = (int)pl.cnt.size() - 1;
  std::vector<T *> Vl(levels + 1, nullptr), tl(levels + 1, nullptr), Rl(levels + 1, nullptr);
  Rl[0] = Rleaf;
  for (int l = 1; l <= levels; ++l) {
    const int cout = pl.cnt[l];
    Vl[l] = talloc((size_t)cout * arity * m * m);
    tl[l] = talloc((size_t)cout * m);
    Rl[l] = talloc((size_t)cout * m * m);
    const double rows_l = (double)pl.cnt[l - 1] * m;
    TimedLaunch tq(c, "tsqr_node_qr", 2.0 * rows_l * m * m - 2.0 / 3.0 * mm3 * cout,
                   8.0 * (2.0 * rows_l * m + (double)cout * m * m));
    hipLaunchKernelGGL((k_node_qr<T, RS, CS>), dim3(cout), dim3(NT), 0, c.stream, Rl[l - 1],
                       pl.cnt[l - 1], m, arity, Vl[l], tl[l], Rl[l], l == levels ? R : nullptr,
                       ldr);
  }
  if (!Q) return;                      // R only: no top-down pass
  size_t zmax = 0;
  for (int v : pl.cnt) zmax = std::max(zmax, (size_t)v);
  T *Z[2] = {talloc(zmax * m * m), talloc(zmax * m * m)};
  const T *Zin = nullptr;
  int which = 0;
  for (int l = levels; l >= 1; --l) {
    const size_t lds = ((size_t)arity * m * m + m) * sizeof(T);
    set_lds(k_node_apply<T, RS, CS>, lds);
    const double rows_l = (double)pl.cnt[l - 1] * m;
    TimedLaunch ta(c, "tsqr_node_apply", 2.0 * rows_l * m * m - 2.0 / 3.0 * mm3 * pl.cnt[l],
                   8.0 * (2.0 * rows_l * m + (double)pl.cnt[l] * m * m));
    hipLaunchKernelGGL((k_node_apply<T, RS, CS>), dim3(pl.cnt[l]), dim3(NT), lds, c.stream, Vl[l],
                       tl[l], pl.cnt[l - 1], m, arity, Zin, Z[which]);
    Zin = Z[which];
    which ^= 1;
  }
  const size_t lds = ((size_t)bmax * m + m) * sizeof(T);
  set_lds(k_leaf_apply<T, RS, CS>, lds);
  TimedLaunch tl2(c, "tsqr_leaf_apply", 2.0 * n * m * m - 2.0 / 3.0 * mm3 * nleaf,
                  8.0 * (2.0 * n * m + (double)nleaf * m * m));
  hipLaunchKernelGGL((k_leaf_apply<T, RS, CS>), dim3(nleaf), dim3(NT), lds, c.stream, Vleaf,
                     tleaf, n, m, nleaf, bmax, Zin, Q, ldq);
}

template <typename T>
void dispatch_tsqr(Ctx &c, const double *Y, int ldy, const Plan &pl, int rs, int cs, double *Q,
                   int ldq, double *R, int ldr) {
  if (cs == 1) {
    if (rs <= 2) run_tsqr<T, 2, 1>(c, Y, ldy, pl, Q, ldq, R, ldr);
    else if (rs <= 4) run_tsqr<T, 4, 1>(c, Y, ldy, pl, Q, ldq, R, ldr);
    else if (rs <= 8) run_tsqr<T, 8, 1>(c, Y, ldy, pl, Q, ldq, R, ldr);
    else run_tsqr<T, 16, 1>(c, Y, ldy, pl, Q, ldq, R, ldr);
  } else {
    if (rs <= 8) run_tsqr<T, 8, 2>(c, Y, ldy, pl, Q, ldq, R, ldr);
    else if (rs <= 12) run_tsqr<T, 12, 2>(c, Y, ldy, pl, Q, ldq, R, ldr);
    else run_tsqr<T, 16, 2>(c, Y, ldy, pl, Q, ldq, R, ldr);
  }
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
  // two columns per lane group above 64 columns: 192-row blocks keep the panel in registers
  if (m > NG) pl.bmax = std::min(pl.bmax, 192);
  TT_REQUIRE(pl.bmax >= 2 * m || n <= pl.bmax, "tsqr: LDS too small for this width");
  pl.nleaf = std::max(1, (n + pl.bmax - 1) / pl.bmax);
  pl.arity = std::max(2, std::min(16, std::min(MAXROWS / m, (d - m) / (m * m))));
  pl.cnt = {pl.nleaf};
  while (pl.cnt.back() > 1) pl.cnt.push_back((pl.cnt.back() + pl.arity - 1) / pl.arity);
  const int rowsmax = std::max(std::min(pl.bmax, n), pl.nleaf > 1 ? pl.arity * m : 0);
  TT_REQUIRE(rowsmax <= MAXROWS, "tsqr: block too tall");
  const int rs = (rowsmax + 15) / 16;
  const int cs = (m + NG - 1) / NG;
  if (c.fp32)
    dispatch_tsqr<float>(c, Y, ldy, pl, rs, cs, Q, ldq, R, ldr);
  else
    dispatch_tsqr<double>(c, Y, ldy, pl, rs, cs, Q, ldq, R, ldr);
  c.cnt.flops += 4.0 * n * m * m;
  c.cnt.bytes += 8.0 * 3.0 * n * m;
}

}  // namespace ttfv
