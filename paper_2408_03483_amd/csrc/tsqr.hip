// Tall-skinny Householder QR (TSQR) with an explicit orthonormal factor.
//
// Used by TT rounding (Section 3.2 orthogonalises the cores by QR) and by the cross
// (orthonormal column/row bases for maxvol).  The n x m panel (m <= 96) is cut into row
// blocks of at most 256 rows; each block is factorised by Householder reflections held in
// registers (LAPACK-style reflectors, R on and above the diagonal, v below it, v_0 = 1).
// The m x m triangles are then combined `arity` at a time in a reduction tree, again by
// Householder.  The explicit Q is formed top-down: the root starts from the first m columns
// of the identity, every node applies its reflectors to its slab, and each leaf applies its
// reflectors to produce its rows of Q; these applications use the compact WY form of the
// block's reflectors on the matrix cores (k_apply_wy).
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

// ---------------------------------------------------------------------------------------
// Top-down pass in compact WY form.  The reflectors of a block (leaf or node) multiply to
// H_0 ... H_{m-1} = I - V T V^T with T upper triangular and T^{-1} = diag(1 / tau) +
// strictly-upper(V^T V) (the unit-diagonal V of the stored reflectors).  The block's slab
// of Q is then  [Z; 0] - V W2  with  W1 = V_top^T Z  (V_top: its first m rows) and W2 the
// solution of T^{-1} W2 = W1 by back substitution, where a reflector with tau = 0 (H = I)
// gives a zero row of W2.  The three products run on the matrix cores (16x16x4 MFMA); the
// back substitution takes the rows four at a time from the bottom (m / 4 dependent steps),
// with a quad of lanes per column of W1.

// exchange with the neighbouring lane of the quad (quad_perm [1,0,3,2]) and with the other
// pair (quad_perm [2,3,0,1])
template <typename T>
__device__ __forceinline__ T quad_swap1(T v) { return dpp_shift<0xB1>(v); }
template <typename T>
__device__ __forceinline__ T quad_swap2(T v) { return dpp_shift<0x4E>(v); }

template <typename T>
struct Mf;
template <>
struct Mf<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // lane l supplies A(l % 16, l / 16) and B(l / 16, l % 16); result v is D(row, l % 16)
  static __device__ __forceinline__ int row(int lk, int v) { return lk + 4 * v; }
};
template <>
struct Mf<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int v) { return 4 * lk + v; }
};

constexpr int WY_KC = 32;        // rows of V (and Z) staged per step of the S / W1 products
constexpr int NTW = 512;         // 8 wavefronts: up to 256 VGPRs each

template <typename T, bool LEAF>
__global__ __launch_bounds__(NTW) void k_apply_wy(const T *__restrict__ V,
                                                 const T *__restrict__ tau, int cnt_in, int m,
                                                 int arity, int n, int nleaf, int bmax,
                                                 const T *__restrict__ Zin,
                                                 T *__restrict__ Zout, double *__restrict__ Q,
                                                 int ldq) {
  extern __shared__ __align__(8) unsigned char smraw[];
  using V4 = typename Mf<T>::v4;
  constexpr int NBMAX = QR_MAXM / 16;              // 16-column tiles of the widest slab
  const int mp = (m + 15) & ~15, nb = mp >> 4, ld = mp + 1;
  T *Ss = reinterpret_cast<T *>(smraw);          // V^T V, row-major (ld)
  T *W = Ss + (size_t)mp * ld;                   // W1, then W2 in place, row-major (ld)
  T *ts = W + (size_t)mp * ld;                   // tau (mp, zero padded)
  T *Vst = ts + mp;                              // staging of WY_KC rows of V and of Z;
  T *Zst = Vst + (size_t)WY_KC * ld;             // (overlaid on Ss / W when they fit)
  if ((size_t)2 * WY_KC * ld <= (size_t)2 * mp * ld) {
    Vst = Ss;
    Zst = Ss + (size_t)WY_KC * ld;
  }
  int rows, ldv, start = 0, c0 = 0;
  const T *Vb, *Zb, *tb;
  if (LEAF) {
    const int L = blockIdx.x;
    leaf_range(L, n, nleaf, start, rows);
    Vb = V + (size_t)L * bmax * m;
    ldv = bmax;
    tb = tau + (size_t)L * m;
    Zb = Zin ? Zin + (size_t)L * m * m : nullptr;
  } else {
    const int k = blockIdx.x;
    c0 = k * arity;
    const int nch = min(arity, cnt_in - c0);
    if (nch == 1) {
      for (int idx = threadIdx.x; idx < m * m; idx += NTW) {
        const int i = idx % m, c = idx / m;
        Zout[(size_t)c0 * m * m + idx] =
            Zin ? Zin[(size_t)k * m * m + idx] : T(i == c ? 1 : 0);
      }
      return;
    }
    rows = nch * m;
    ldv = arity * m;
    Vb = V + (size_t)k * ldv * m;
    tb = tau + (size_t)k * m;
    Zb = Zin ? Zin + (size_t)k * m * m : nullptr;
  }
  // unit lower-trapezoidal V and the slab Z (identity at the root), zero outside; the loads
  // are unconditional (clamped to a valid address) so that unrolled loops can batch them
  auto vfull = [&](int i, int c) -> T {
    const bool in = c < m && i < rows && i > c;
    const T v = Vb[in ? i + c * ldv : 0];         // 32-bit offsets: a block holds < 2^31
    return in ? v : T(i == c && c < m ? 1 : 0);
  };
  auto zfull = [&](int i, int c) -> T {
    const bool in = i < m && c < m;
    if (!Zb) return T(in && i == c ? 1 : 0);
    const T v = Zb[in ? i + c * m : 0];
    return in ? v : T(0);
  };
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
  for (int i = threadIdx.x; i < mp; i += NTW) ts[i] = i < m ? tb[i] : T(0);

  // S = V^T V on the block-upper tiles (ti <= tj) and W1 = V_top^T Z on all tiles; wave w
  // owns tiles w, w + 16, ...; V and Z rows are staged through LDS with coalesced loads
  const int ns = nb * (nb + 1) / 2, ntile = ns + nb * nb;
  auto decode = [&](int q, int &ti, int &tj) {
    if (q < ns) {
      int r = q;
      ti = 0;
      while (r >= nb - ti) {
        r -= nb - ti;
        ++ti;
      }
      tj = ti + r;
    } else {
      ti = (q - ns) / nb;
      tj = (q - ns) - ti * nb;
    }
  };
  constexpr int TPW = 8;                           // tiles per wave (57 at most)
  V4 acc[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) acc[t] = V4{0, 0, 0, 0};
  // the next chunk is fetched into registers while the current one is multiplied
  constexpr int PF = WY_KC * QR_MAXM / NTW;          // staged values per thread (6)
  T pv[PF], pz[PF];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int e = 0; e < PF; ++e) {
      const int idx = threadIdx.x + NTW * e;
      const int kk = idx % WY_KC, cc = idx / WY_KC;
      pv[e] = vfull(k0 + kk, cc);                    // zero for cc >= m
      pz[e] = k0 < mp ? zfull(k0 + kk, cc) : T(0);
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < rows; k0 += WY_KC) {
    const bool withZ = k0 < mp;
#pragma unroll
    for (int e = 0; e < PF; ++e) {
      const int idx = threadIdx.x + NTW * e;
      const int kk = idx % WY_KC, cc = idx / WY_KC;
      if (cc < mp) {
        Vst[(size_t)kk * ld + cc] = pv[e];
        if (withZ) Zst[(size_t)kk * ld + cc] = pz[e];
      }
    }
    __syncthreads();
    if (k0 + WY_KC < rows) fetch(k0 + WY_KC);
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int q = wave + (NTW / 64) * t;
      if (q >= ntile || (q >= ns && !withZ)) continue;
      int ti, tj;
      decode(q, ti, tj);
      const T *Ap = Vst + (size_t)lk * ld + 16 * ti + li;
      const T *Bp = (q < ns ? Vst : Zst) + (size_t)lk * ld + 16 * tj + li;
#pragma unroll
      for (int u = 0; u < WY_KC / 4; ++u)
        acc[t] = Mf<T>::op(Ap[(size_t)4 * u * ld], Bp[(size_t)4 * u * ld], acc[t]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int q = wave + (NTW / 64) * t;
    if (q >= ntile) continue;
    int ti, tj;
    decode(q, ti, tj);
    T *D = q < ns ? Ss : W;
#pragma unroll
    for (int v = 0; v < 4; ++v)
      D[(size_t)(16 * ti + Mf<T>::row(lk, v)) * ld + 16 * tj + li] = acc[t][v];
  }
  __syncthreads();

  // back substitution W2(i, c) = tau_i (W1(i, c) - sum_{l > i} S(i, l) W2(l, c)), i from
  // the bottom, four rows at a time: a quad of lanes per column c, lane p summing the terms
  // l = p (mod 4) below the block (quad sums are symmetric, so the four lanes agree
  // bitwise), then the 4 x 4 triangle in every lane of the quad
  if (threadIdx.x < 4 * mp) {
    const int c = threadIdx.x >> 2, p = threadIdx.x & 3;
    for (int i0 = mp - 4; i0 >= 0; i0 -= 4) {
      const T *S0 = Ss + (size_t)i0 * ld;
      T s0 = T(0), s1 = T(0), s2 = T(0), s3 = T(0);
      // rows l = i0 + 4 + p + 4 e below the block, 4 per lane at a time so that the loads of
      // a pass are in flight together (rows >= mp read row mp - 1 and count zero)
      for (int l0 = i0 + 4 + p; l0 < mp; l0 += 16) {
        T w[4], a0[4], a1[4], a2[4], a3[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int l = l0 + 4 * e, lc = min(l, mp - 1);
          const T wv = W[(size_t)lc * ld + c];
          w[e] = l < mp ? wv : T(0);
          a0[e] = S0[lc];
          a1[e] = S0[ld + lc];
          a2[e] = S0[2 * ld + lc];
          a3[e] = S0[3 * ld + lc];
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          s0 += a0[e] * w[e];
          s1 += a1[e] * w[e];
          s2 += a2[e] * w[e];
          s3 += a3[e] * w[e];
        }
      }
      s0 += quad_swap1(s0);
      s1 += quad_swap1(s1);
      s2 += quad_swap1(s2);
      s3 += quad_swap1(s3);
      s0 += quad_swap2(s0);
      s1 += quad_swap2(s1);
      s2 += quad_swap2(s2);
      s3 += quad_swap2(s3);
      const T y0 = W[(size_t)i0 * ld + c], y1 = W[(size_t)(i0 + 1) * ld + c];
      const T y2 = W[(size_t)(i0 + 2) * ld + c], y3 = W[(size_t)(i0 + 3) * ld + c];
      const T w3 = ts[i0 + 3] * (y3 - s3);
      const T w2 = ts[i0 + 2] * (y2 - s2 - S0[2 * ld + i0 + 3] * w3);
      const T w1 = ts[i0 + 1] * (y1 - s1 - S0[ld + i0 + 2] * w2 - S0[ld + i0 + 3] * w3);
      const T w0 = ts[i0] * (y0 - s0 - S0[i0 + 1] * w1 - S0[i0 + 2] * w2 - S0[i0 + 3] * w3);
      const T wp = p == 0 ? w0 : p == 1 ? w1 : p == 2 ? w2 : w3;
      W[(size_t)(i0 + p) * ld + c] = wp;
    }
  }
  __syncthreads();

  // output slab [Z; 0] - V W2, formed transposed so that lanes run along rows: tile
  // (columns 16 tc.., rows 16 st..) = W2^T V^T
  const int nstrip = (rows + 15) >> 4;
  constexpr int NH = NBMAX;                          // column tiles per pass
  for (int job = wave; job < nstrip; job += NTW / 64) {
    const int st = job, tc0 = 0;
    V4 o[NH];
#pragma unroll
    for (int tc = 0; tc < NH; ++tc) o[tc] = V4{0, 0, 0, 0};
    const int kend = min(mp, 16 * st + 16);          // V(i, k) = 0 for k > i
#pragma unroll 1
    for (int k0 = 0; k0 < kend; k0 += 32) {        // 32 columns of V per group of loads
      T b[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) b[u] = vfull(16 * st + li, k0 + 4 * u + lk);
      const int ucnt = min(8, (kend - k0) >> 2);
      for (int u = 0; u < ucnt; ++u) {
        const T *Wk = W + (size_t)(k0 + 4 * u + lk) * ld + 16 * tc0 + li;
        T bu = b[0];
#pragma unroll
        for (int uu = 1; uu < 8; ++uu) bu = u == uu ? b[uu] : bu;
#pragma unroll
        for (int tc = 0; tc < NH; ++tc)
          if (tc0 + tc < nb) o[tc] = Mf<T>::op(Wk[16 * tc], bu, o[tc]);
      }
    }
    const int i = 16 * st + li;
    if (i >= rows) continue;
    // destination of row i: Q row start + i (leaf) or row ii of child ch (node)
    const int ch = LEAF ? 0 : i / m, ii = LEAF ? 0 : i - ch * m;
    double *qrow = LEAF ? Q + (start + i) : nullptr;
    T *zrow = LEAF ? nullptr : Zout + (size_t)(c0 + ch) * m * m + ii;
    const int ldo = LEAF ? ldq : m;
#pragma unroll
    for (int tc = 0; tc < NH; ++tc) {
      if (tc0 + tc >= nb) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int c = 16 * (tc0 + tc) + Mf<T>::row(lk, v);
        if (c >= m) continue;
        const T val = (i < m ? zfull(i, c) : T(0)) - o[tc][v];
        if (LEAF)
          qrow[c * ldo] = double(val);
        else
          zrow[c * ldo] = val;
      }
    }
  }
}

size_t apply_wy_lds(int m, size_t elem) {
  const size_t mp = (size_t)((m + 15) & ~15), ld = mp + 1;
  const size_t stage = 2 * (size_t)WY_KC * ld;
  return (2 * mp * ld + mp + (stage <= 2 * mp * ld ? 0 : stage)) * elem;
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
    TimedLaunch tl(c, "tsqr_qr_leaf", 2.0 * n * m * m - 2.0 / 3.0 * mm3 * nleaf,
                   8.0 * (2.0 * n * m + (double)nleaf * m * m));
    TT_LAUNCH(c, (k_leaf_qr<T, RS, CS>), dim3(nleaf), dim3(NT), 0, Y, n, m, ldy, nleaf, bmax,
              Vleaf, tleaf, Rleaf, nleaf == 1 ? R : (double *)nullptr, ldr);
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
    TimedLaunch tq(c, "tsqr_qr_node", 2.0 * rows_l * m * m - 2.0 / 3.0 * mm3 * cout,
                   8.0 * (2.0 * rows_l * m + (double)cout * m * m));
    TT_LAUNCH(c, (k_node_qr<T, RS, CS>), dim3(cout), dim3(NT), 0, (const T *)Rl[l - 1],
              pl.cnt[l - 1], m, arity, Vl[l], tl[l], Rl[l], l == levels ? R : (double *)nullptr,
              ldr);
  }
  if (!Q) return;                      // R only: no top-down pass
  size_t zmax = 0;
  for (int v : pl.cnt) zmax = std::max(zmax, (size_t)v);
  T *Z[2] = {talloc(zmax * m * m), talloc(zmax * m * m)};
  const T *Zin = nullptr;
  int which = 0;
  const size_t wy_lds = apply_wy_lds(m, sizeof(T));
  for (int l = levels; l >= 1; --l) {
    set_lds(k_apply_wy<T, false>, wy_lds);
    const double rows_l = (double)pl.cnt[l - 1] * m;
    TimedLaunch ta(c, "tsqr_wy_node", 2.0 * rows_l * m * m - 2.0 / 3.0 * mm3 * pl.cnt[l],
                   8.0 * (2.0 * rows_l * m + (double)pl.cnt[l] * m * m));
    TT_LAUNCH(c, (k_apply_wy<T, false>), dim3(pl.cnt[l]), dim3(NTW), wy_lds,
              (const T *)Vl[l], (const T *)tl[l], pl.cnt[l - 1], m, arity, 0, 0, 0, Zin, Z[which],
              (double *)nullptr, 0);
    Zin = Z[which];
    which ^= 1;
  }
  set_lds(k_apply_wy<T, true>, wy_lds);
  TimedLaunch tl2(c, "tsqr_wy_leaf", 2.0 * n * m * m - 2.0 / 3.0 * mm3 * nleaf,
                  8.0 * (2.0 * n * m + (double)nleaf * m * m));
  TT_LAUNCH(c, (k_apply_wy<T, true>), dim3(nleaf), dim3(NTW), wy_lds, (const T *)Vleaf,
            (const T *)tleaf, 0, m, 0, n, nleaf, bmax, Zin, (T *)nullptr, Q, ldq);
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

// the arena draws of run_tsqr<double> for the plan tsqr() makes (each rounded up to the
// arena's 256-byte alignment)
size_t tsqr_arena_bytes(int n, int m) {
  if (m < 1 || n < m) return 0;
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t e = sizeof(double);
  const int bmax = m > NG ? 192 : MAXROWS;
  const int nleaf = std::max(1, (n + bmax - 1) / bmax);
  const int arity = std::max(2, std::min(16, MAXROWS / m));
  std::vector<int> cnt{nleaf};
  while (cnt.back() > 1) cnt.push_back((cnt.back() + arity - 1) / arity);
  const size_t mm = (size_t)m * m;
  size_t b = al((size_t)nleaf * bmax * m * e) + al((size_t)nleaf * m * e) + al(nleaf * mm * e);
  size_t zmax = 0;
  for (size_t l = 1; l < cnt.size(); ++l)
    b += al((size_t)cnt[l] * arity * mm * e) + al((size_t)cnt[l] * m * e) + al(cnt[l] * mm * e);
  for (int v : cnt) zmax = std::max(zmax, (size_t)v);
  return std::max(b + 2 * al(zmax * mm * e), cholqr_arena_bytes(n, m, false));
}

int qr_max_cols() { return QR_MAXM; }

void tsqr(Ctx &c, const double *Y, int n, int m, int ldy, double *Q, int ldq, double *R,
          int ldr) {
  TT_REQUIRE(m >= 1 && n >= m, "tsqr: need n >= m >= 1");
  TT_REQUIRE(m <= QR_MAXM, "tsqr: more than 96 columns");
  const bool chol = c.qr == TT_QR_CHOLESKY || (c.qr == TT_QR_AUTO && m > 64);
  if (chol && !c.householder) {
    cholqr(c, Y, n, m, ldy, Q, ldq, R, ldr);
    return;
  }
  const int d = lds_doubles();
  Plan pl;
  pl.n = n;
  pl.m = m;
  // rows per leaf: registers hold <= 256 rows; two columns per lane group above 64
  // columns: 192-row blocks keep the panel in registers
  pl.bmax = m > NG ? 192 : MAXROWS;
  TT_REQUIRE(apply_wy_lds(m, sizeof(double)) <= (size_t)d * sizeof(double),
             "tsqr: LDS too small for this width");
  pl.nleaf = std::max(1, (n + pl.bmax - 1) / pl.bmax);
  pl.arity = std::max(2, std::min(16, MAXROWS / m));
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
