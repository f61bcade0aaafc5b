// Full-grid finite-volume comparator: the scheme of Sections 2.2-2.4 and 4.4 on n x n arrays
// of cell averages, without tensor-train compression (the "full-tensor" form the paper times
// its TT solver against, Section 4.1's equation SWE-system-no-loop).
//
// One kernel per SSP-RK3 stage computes L(U) for a tile of TI x TJ cells and writes the stage
// combination; the tile and a halo of k + 1 cells of the three variables sit in LDS:
//   1. Step 1 in x: minus/plus values at the TI + 1 x-faces of the tile, for the TJ + 2k rows
//      that Step 2 needs (Upwind: the combined linear face stencil; WENO5: Jiang-Shu weights);
//   2. Step 2 in y at the Gauss points of every face segment, the LLF flux at each point and
//      the Gauss-Legendre sum: the face flux Fhat (TI + 1 faces x TJ rows);
//   3-4. the same for the y-faces;
//   5. per cell L = -((Fhat_r - Fhat_l) + (Ghat_t - Ghat_b)) / dx + Coriolis source, then the
//      stage: U1 = U + dt L; U2 = 3/4 U0 + 1/4 (U1 + dt L); U' = U0/3 + 2/3 (U2 + dt L).
// Boundaries per axis: periodic, reflective walls (ghost cells mirrored, normal momentum
// negated), or exact (ghost cells from separable terms amp cos(omega t + phase) X Y at the
// stage time; corners follow the other axis's rule).  Separable forcing terms are added to L.
//
// Layout in HBM: U[v][i][j] (variable, x cell, y cell; y contiguous), FP64.  Bound: the
// reconstruction arithmetic (about 1.5 kflop per cell and stage for Upwind5) against
// 9 x 8 bytes of HBM traffic per cell and stage (read U and U0, write the stage).
#include "common.h"
#include "weno.h"

#include <cmath>

namespace ttfv {

namespace {

constexpr int TI = 8, TJ = 32, NT = 256;   // tile: 8 x-cells by 32 y-cells, one thread per cell
static_assert(TI * TJ == NT, "one thread per cell in the last phase");

constexpr int BC_PERIODIC = 0, BC_WALL = 1, BC_EXACT = 2;
constexpr int MAX_TERMS = 256;

struct GridTerm {
  int var, where;
  double amp, omega, phase;
  const double *X, *Y;
};

struct GridArgs {
  int n, bc[2];
  double g, H, f, dx, dt;
  StencilSet st;
  WenoArgs w;
  const GridTerm *terms;   // device, nterms entries
  int nterms;
};

template <int K>
struct Dims {
  static constexpr int H = K + 1;                 // halo
  static constexpr int LI = TI + 2 * H, LJ = TJ + 2 * H;
  static constexpr int XF_ROWS = TJ + 2 * K;      // rows of x-face values Step 2 reads
  static constexpr int YF_COLS = TI + 2 * K;
  static constexpr int XF = (TI + 1) * XF_ROWS;   // x-face values per variable and side
  static constexpr int YF = (TJ + 1) * YF_COLS;
  static constexpr int FACES = XF > YF ? XF : YF;
};

// global index of a (possibly ghost) cell and the sign the mirror applies
__device__ __forceinline__ int map_cell(int gi, int n, bool periodic, bool &flip) {
  flip = false;
  if (periodic) {
    gi %= n;
    return gi < 0 ? gi + n : gi;
  }
  if (gi < 0) {
    gi = -1 - gi;
    flip = true;
  } else if (gi >= n) {
    gi = 2 * n - 1 - gi;
    flip = true;
  }
  // cells far outside (a tile wider than the domain) are never read by a valid output
  return gi < 0 ? 0 : (gi >= n ? n - 1 : gi);
}

template <int SCH>
__device__ __forceinline__ double face_value(const GridArgs &a, const double *v) {
  // v[0..2K] = cells c-K .. c+K; value at the right face of cell c
  if constexpr (SCH == 55) {
    return weno_face(a.w, v);
  } else {
    constexpr int K = SCH == 3 ? 1 : 2;
    double s = 0.0;
    for (int o = 0; o <= 2 * K; ++o) s += a.st.face[o] * v[o];
    return s;
  }
}

template <int SCH>
__device__ __forceinline__ void quad_values(const GridArgs &a, const double *v, double *out) {
  // v[0..2K] = cells j-K .. j+K; values at the Gauss points of cell j
  if constexpr (SCH == 55) {
    double beta[3];
    smoothness(v, beta);
    const WenoTables &t = a.w.t;
    out[0] = weno_combine(t.quad_C[0], t.quad_g[0], beta, v, a.w.eps);
    out[1] = t.sp * weno_combine(t.quad_C[1], t.gp, beta, v, a.w.eps) -
             t.sm * weno_combine(t.quad_C[1], t.gm, beta, v, a.w.eps);
    out[2] = weno_combine(t.quad_C[2], t.quad_g[2], beta, v, a.w.eps);
  } else {
    constexpr int K = SCH == 3 ? 1 : 2, NQ = SCH == 3 ? 2 : 3;
    for (int m = 0; m < NQ; ++m) {
      double s = 0.0;
      for (int o = 0; o <= 2 * K; ++o) s += a.st.quad[m][o] * v[o];
      out[m] = s;
    }
  }
}

// LLF flux (Section 2.2) through a face with normal direction d (0: x, 1: y)
template <bool NL>
__device__ __forceinline__ void llf(const GridArgs &a, int d, const double *um, const double *up,
                                    double *F) {
  double fm[3], fp[3], lam;
  if constexpr (NL) {
    const int mom = 1 + d;
    const double hm = um[0], hp = up[0];
    if (d == 0) {
      fm[0] = um[1];
      fm[1] = um[1] * um[1] / hm + 0.5 * a.g * hm * hm;
      fm[2] = um[1] * um[2] / hm;
      fp[0] = up[1];
      fp[1] = up[1] * up[1] / hp + 0.5 * a.g * hp * hp;
      fp[2] = up[1] * up[2] / hp;
    } else {
      fm[0] = um[2];
      fm[1] = um[1] * um[2] / hm;
      fm[2] = um[2] * um[2] / hm + 0.5 * a.g * hm * hm;
      fp[0] = up[2];
      fp[1] = up[1] * up[2] / hp;
      fp[2] = up[2] * up[2] / hp + 0.5 * a.g * hp * hp;
    }
    const double lm = fabs(um[mom] / hm) + sqrt(a.g * hm);
    const double lp = fabs(up[mom] / hp) + sqrt(a.g * hp);
    lam = fmax(lm, lp);
  } else {
    if (d == 0) {
      fm[0] = a.H * um[1];
      fm[1] = a.g * um[0];
      fm[2] = 0.0;
      fp[0] = a.H * up[1];
      fp[1] = a.g * up[0];
      fp[2] = 0.0;
    } else {
      fm[0] = a.H * um[2];
      fm[1] = 0.0;
      fm[2] = a.g * um[0];
      fp[0] = a.H * up[2];
      fp[1] = 0.0;
      fp[2] = a.g * up[0];
    }
    lam = sqrt(a.g * a.H);
  }
  for (int v = 0; v < 3; ++v) F[v] = 0.5 * (fm[v] + fp[v]) - 0.5 * lam * (up[v] - um[v]);
}

// sum of the ghost terms of variable v on one side at ghost cell g (0..2) and cell c of the
// other axis (x sides: X[g] Y[c]; y sides: X[c] Y[g])
__device__ __forceinline__ double ghost_sum(const GridArgs &a, const double *tf, int v,
                                            int where, int g, int c) {
  double s = 0.0;
  const bool xs = where == TT_TERM_X_LO || where == TT_TERM_X_HI;
  for (int k = 0; k < a.nterms; ++k) {
    const GridTerm &tm = a.terms[k];
    if (tm.var != v || tm.where != where) continue;
    s += tf[k] * (xs ? tm.X[g] * tm.Y[c] : tm.X[c] * tm.Y[g]);
  }
  return s;
}

// U0 and out are the same array in the last stage (each thread reads its own cells of U0
// before writing them; halos come from U), so neither is declared restrict
template <int SCH, bool NL>
__global__ __launch_bounds__(NT) void k_grid_stage(GridArgs a, const double *__restrict__ U,
                                                   const double *U0, double *out, int stage,
                                                   double tstage) {
  constexpr int K = SCH == 3 ? 1 : 2, NQ = SCH == 3 ? 2 : 3;
  using D = Dims<K>;
  __shared__ double sU[3][D::LI][D::LJ];
  __shared__ double sFm[3][D::FACES], sFp[3][D::FACES];
  __shared__ double sX[3][TI + 1][TJ];    // x-face fluxes
  __shared__ double sY[3][TJ + 1][TI];    // y-face fluxes
  __shared__ double sTf[MAX_TERMS];       // time factors of the terms at this stage
  const int n = a.n;
  const bool per[2] = {a.bc[0] == BC_PERIODIC, a.bc[1] == BC_PERIODIC};
  const int i0 = blockIdx.y * TI, j0 = blockIdx.x * TJ;
  const size_t nn = (size_t)n * n;
  const int tid = threadIdx.x;
  for (int k = tid; k < a.nterms; k += NT)
    sTf[k] = a.terms[k].amp * cos(a.terms[k].omega * tstage + a.terms[k].phase);
  __syncthreads();

  // tile with halo; ghost cells by periodic wrap, mirror (normal momentum negated) or, on an
  // exact axis, the ghost terms (at the other axis's mapped cell)
  for (int e = tid; e < D::LI * D::LJ; e += NT) {
    const int ii = e / D::LJ, jj = e - ii * D::LJ;
    const int ci = i0 - D::H + ii, cj = j0 - D::H + jj;
    bool fx, fy;
    if ((ci < 0 || ci >= n) && a.bc[0] == BC_EXACT) {
      const int gj = map_cell(cj, n, per[1], fy);
      const int where = ci < 0 ? TT_TERM_X_LO : TT_TERM_X_HI;
      const int g = min(max(ci < 0 ? ci + 3 : ci - n, 0), 2);
      for (int v = 0; v < 3; ++v) {
        const double x = ghost_sum(a, sTf, v, where, g, gj);
        sU[v][ii][jj] = (v == 2 && fy) ? -x : x;
      }
      continue;
    }
    if ((cj < 0 || cj >= n) && a.bc[1] == BC_EXACT) {
      const int gi = map_cell(ci, n, per[0], fx);
      const int where = cj < 0 ? TT_TERM_Y_LO : TT_TERM_Y_HI;
      const int g = min(max(cj < 0 ? cj + 3 : cj - n, 0), 2);
      for (int v = 0; v < 3; ++v) {
        const double x = ghost_sum(a, sTf, v, where, g, gi);
        sU[v][ii][jj] = (v == 1 && fx) ? -x : x;
      }
      continue;
    }
    const int gi = map_cell(ci, n, per[0], fx);
    const int gj = map_cell(cj, n, per[1], fy);
    const size_t off = (size_t)gi * n + gj;
    sU[0][ii][jj] = U[off];
    sU[1][ii][jj] = fx ? -U[nn + off] : U[nn + off];
    sU[2][ii][jj] = fy ? -U[2 * nn + off] : U[2 * nn + off];
  }
  __syncthreads();

  // 1. Step 1 along x: face fl (between local cells fl-1 and fl), row jl in [-K, TJ+K);
  //    tile column index of cell il is H + il, of row jl is H + jl
  for (int e = tid; e < D::XF; e += NT) {
    const int fl = e / D::XF_ROWS, r = e - fl * D::XF_ROWS;
    const int jj = D::H - K + r;
    for (int v = 0; v < 3; ++v) {
      double vm[2 * K + 1], vp[2 * K + 1];
      for (int o = -K; o <= K; ++o) {
        vm[o + K] = sU[v][D::H + fl - 1 + o][jj];   // cells fl-1+o: right face of fl-1
        vp[o + K] = sU[v][D::H + fl - o][jj];       // mirrored about cell fl: its left face
      }
      sFm[v][e] = face_value<SCH>(a, vm);
      sFp[v][e] = face_value<SCH>(a, vp);
    }
  }
  __syncthreads();

  // 2. Step 2 along y at the Gauss points of face fl, cell row jl; LLF; Gauss sum
  for (int e = tid; e < (TI + 1) * TJ; e += NT) {
    const int fl = e / TJ, jl = e - fl * TJ;
    double qm[3][NQ], qp[3][NQ];
    for (int v = 0; v < 3; ++v) {
      double vm[2 * K + 1], vp[2 * K + 1];
      for (int o = 0; o <= 2 * K; ++o) {
        vm[o] = sFm[v][fl * D::XF_ROWS + jl + o];
        vp[o] = sFp[v][fl * D::XF_ROWS + jl + o];
      }
      quad_values<SCH>(a, vm, qm[v]);
      quad_values<SCH>(a, vp, qp[v]);
    }
    double acc[3] = {0.0, 0.0, 0.0};
    for (int m = 0; m < NQ; ++m) {
      const double um[3] = {qm[0][m], qm[1][m], qm[2][m]};
      const double up[3] = {qp[0][m], qp[1][m], qp[2][m]};
      double F[3];
      llf<NL>(a, 0, um, up, F);
      for (int v = 0; v < 3; ++v) acc[v] += a.st.gw[m] * F[v];
    }
    for (int v = 0; v < 3; ++v) sX[v][fl][jl] = acc[v];
  }
  __syncthreads();

  // 3. Step 1 along y: face gl (between local rows gl-1 and gl), column il in [-K, TI+K)
  for (int e = tid; e < D::YF; e += NT) {
    const int gl = e / D::YF_COLS, c = e - gl * D::YF_COLS;
    const int ii = D::H - K + c;
    for (int v = 0; v < 3; ++v) {
      double vm[2 * K + 1], vp[2 * K + 1];
      for (int o = -K; o <= K; ++o) {
        vm[o + K] = sU[v][ii][D::H + gl - 1 + o];
        vp[o + K] = sU[v][ii][D::H + gl - o];
      }
      sFm[v][e] = face_value<SCH>(a, vm);
      sFp[v][e] = face_value<SCH>(a, vp);
    }
  }
  __syncthreads();

  // 4. Step 2 along x at the Gauss points of face gl, cell column il; LLF; Gauss sum
  for (int e = tid; e < (TJ + 1) * TI; e += NT) {
    const int gl = e / TI, il = e - gl * TI;
    double qm[3][NQ], qp[3][NQ];
    for (int v = 0; v < 3; ++v) {
      double vm[2 * K + 1], vp[2 * K + 1];
      for (int o = 0; o <= 2 * K; ++o) {
        vm[o] = sFm[v][gl * D::YF_COLS + il + o];
        vp[o] = sFp[v][gl * D::YF_COLS + il + o];
      }
      quad_values<SCH>(a, vm, qm[v]);
      quad_values<SCH>(a, vp, qp[v]);
    }
    double acc[3] = {0.0, 0.0, 0.0};
    for (int m = 0; m < NQ; ++m) {
      const double um[3] = {qm[0][m], qm[1][m], qm[2][m]};
      const double up[3] = {qp[0][m], qp[1][m], qp[2][m]};
      double F[3];
      llf<NL>(a, 1, um, up, F);
      for (int v = 0; v < 3; ++v) acc[v] += a.st.gw[m] * F[v];
    }
    for (int v = 0; v < 3; ++v) sY[v][gl][il] = acc[v];
  }
  __syncthreads();

  // 5. L and the stage combination for the cell of this thread
  const int il = tid / TJ, jl = tid - (tid / TJ) * TJ;
  const int gi = i0 + il, gj = j0 + jl;
  if (gi >= n || gj >= n) return;
  const size_t off = (size_t)gi * n + gj;
  double L[3];
  for (int v = 0; v < 3; ++v)
    L[v] = -((sX[v][il + 1][jl] - sX[v][il][jl]) + (sY[v][jl + 1][il] - sY[v][jl][il])) / a.dx;
  const double u1 = sU[1][D::H + il][D::H + jl], u2 = sU[2][D::H + il][D::H + jl];
  if (a.f != 0.0) {
    L[1] = L[1] + a.f * u2;
    L[2] = L[2] - a.f * u1;
  }
  for (int k = 0; k < a.nterms; ++k) {
    const GridTerm &tm = a.terms[k];
    if (tm.where == TT_TERM_FORCING) L[tm.var] += sTf[k] * tm.X[gi] * tm.Y[gj];
  }
  for (int v = 0; v < 3; ++v) {
    const double u = sU[v][D::H + il][D::H + jl];
    const double e = u + a.dt * L[v];
    double r;
    if (stage == 0) {
      r = e;
    } else if (stage == 1) {
      r = 0.75 * U0[v * nn + off] + 0.25 * e;
    } else {
      r = U0[v * nn + off] / 3.0 + 2.0 / 3.0 * e;
    }
    out[v * nn + off] = r;
  }
}

template <int SCH, bool NL>
void launch_stage(Ctx &c, const GridArgs &a, const double *U, const double *U0, double *out,
                  int stage, double tstage) {
  const dim3 grid((a.n + TJ - 1) / TJ, (a.n + TI - 1) / TI);
  TT_LAUNCH(c, (k_grid_stage<SCH, NL>), grid, dim3(NT), 0, a, U, U0, out, stage, tstage);
  HIP_CHECK(hipGetLastError());
}

}  // namespace

struct Grid {
  tt_fv_params p{};
  Ctx c;
  GridArgs a{};
  double *U1 = nullptr, *U2 = nullptr;
  double t = 0.0;                 // time at the start of the next step
  void *term_mem = nullptr;       // GridTerm array followed by the factor vectors
};

Grid *grid_create(const tt_fv_params *p, void *stream) {
  TT_REQUIRE(p, "tt_grid_init: null argument");
  TT_REQUIRE(p->n >= 6, "tt_grid_init: n must be >= 6");
  TT_REQUIRE(p->scheme == 3 || p->scheme == 5 || p->scheme == 55, "tt_grid_init: bad scheme");
  TT_REQUIRE(p->nonlinear || p->g * p->H0 > 0.0, "tt_grid_init: g H0 must be positive");
  TT_REQUIRE(p->bc_x >= 0 && p->bc_x <= TT_BC_EXACT && p->bc_y >= 0 && p->bc_y <= TT_BC_EXACT,
             "tt_grid_init: unknown boundary kind");
  TT_REQUIRE(!(p->bc_x == TT_BC_EXACT && p->bc_y == TT_BC_EXACT),
             "tt_grid_init: at most one axis can have exact boundaries");
  TT_REQUIRE(std::isfinite(p->t0), "tt_grid_init: t0 not finite");
  Grid *s = new Grid();
  try {
    s->p = *p;
    s->c.stream = (hipStream_t)stream;
    const size_t bytes = 3 * (size_t)p->n * p->n * sizeof(double);
    HIP_CHECK(hipMalloc((void **)&s->U1, bytes));
    HIP_CHECK(hipMalloc((void **)&s->U2, bytes));
    GridArgs &a = s->a;
    a.n = p->n;
    for (int ax = 0; ax < 2; ++ax) {
      const int kind = (ax == 0 ? p->bc_x : p->bc_y) ? (ax == 0 ? p->bc_x : p->bc_y)
                                                     : (p->periodic ? TT_BC_PERIODIC : TT_BC_WALL);
      a.bc[ax] = kind == TT_BC_PERIODIC ? BC_PERIODIC : kind == TT_BC_WALL ? BC_WALL : BC_EXACT;
    }
    a.terms = nullptr;
    a.nterms = 0;
    s->t = p->t0;
    a.g = p->g;
    a.H = p->H0;
    a.f = p->f;
    a.dx = 1.0 / p->n;
    a.st = derive_stencils(p->scheme == 3 ? 3 : 5);
    a.w.t = derive_weno_tables();
    a.w.eps = a.dx * a.dx;
  } catch (...) {
    if (s->U1) (void)hipFree(s->U1);
    if (s->U2) (void)hipFree(s->U2);
    delete s;
    throw;
  }
  return s;
}

void grid_destroy(Grid *s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->c.stream);
  (void)hipFree(s->U1);
  (void)hipFree(s->U2);
  if (s->term_mem) (void)hipFree(s->term_mem);
  delete s;
}

void grid_set_terms(Grid *s, const tt_fv_term *tv, int count) {
  TT_REQUIRE(count >= 0 && count <= MAX_TERMS && (count == 0 || tv),
             "tt_grid_set_terms: bad term list (at most 256 terms)");
  const int n = s->a.n;
  // device block: the GridTerm array, then every term's X and Y
  size_t doubles = 0;
  for (int k = 0; k < count; ++k) {
    const tt_fv_term &t = tv[k];
    TT_REQUIRE(t.var >= 0 && t.var < 3, "tt_grid_set_terms: var must be 0, 1 or 2");
    TT_REQUIRE(t.where >= TT_TERM_FORCING && t.where <= TT_TERM_Y_HI,
               "tt_grid_set_terms: unknown where");
    TT_REQUIRE(t.X && t.Y, "tt_grid_set_terms: null factor");
    const bool xs = t.where == TT_TERM_X_LO || t.where == TT_TERM_X_HI;
    const bool ys = t.where == TT_TERM_Y_LO || t.where == TT_TERM_Y_HI;
    TT_REQUIRE(!xs || s->a.bc[0] == BC_EXACT, "tt_grid_set_terms: x ghost terms need bc_x exact");
    TT_REQUIRE(!ys || s->a.bc[1] == BC_EXACT, "tt_grid_set_terms: y ghost terms need bc_y exact");
    doubles += (xs ? 3 : n) + (ys ? 3 : n);
  }
  const size_t head = ((size_t)count * sizeof(GridTerm) + 255) & ~(size_t)255;
  std::vector<unsigned char> host(head + doubles * sizeof(double));
  HIP_CHECK(hipStreamSynchronize(s->c.stream));
  if (s->term_mem) HIP_CHECK(hipFree(s->term_mem));
  s->term_mem = nullptr;
  s->a.terms = nullptr;
  s->a.nterms = 0;
  if (!count) return;
  HIP_CHECK(hipMalloc(&s->term_mem, host.size()));
  auto *dev = (unsigned char *)s->term_mem;
  auto *gt = (GridTerm *)host.data();
  double *vec = (double *)(host.data() + head);
  size_t off = 0;
  for (int k = 0; k < count; ++k) {
    const tt_fv_term &t = tv[k];
    const bool xs = t.where == TT_TERM_X_LO || t.where == TT_TERM_X_HI;
    const bool ys = t.where == TT_TERM_Y_LO || t.where == TT_TERM_Y_HI;
    const int nx = xs ? 3 : n, ny = ys ? 3 : n;
    std::copy(t.X, t.X + nx, vec + off);
    std::copy(t.Y, t.Y + ny, vec + off + nx);
    gt[k] = {t.var, t.where, t.amp, t.omega, t.phase,
             (const double *)(dev + head) + off, (const double *)(dev + head) + off + nx};
    off += nx + ny;
  }
  HIP_CHECK(hipMemcpy(s->term_mem, host.data(), host.size(), hipMemcpyHostToDevice));
  s->a.terms = (const GridTerm *)s->term_mem;
  s->a.nterms = count;
}

template <int SCH, bool NL>
void grid_steps(Grid *s, double *U, int nsteps) {
  const double dt = s->a.dt;
  for (int k = 0; k < nsteps; ++k) {
    // stage times of SSP-RK3: t, t + dt, t + dt/2
    launch_stage<SCH, NL>(s->c, s->a, U, U, s->U1, 0, s->t);
    launch_stage<SCH, NL>(s->c, s->a, s->U1, U, s->U2, 1, s->t + dt);
    launch_stage<SCH, NL>(s->c, s->a, s->U2, U, U, 2, s->t + 0.5 * dt);
    s->t += dt;
  }
}

void grid_step(Grid *s, double *U, double dt, int nsteps) {
  TT_REQUIRE(U, "tt_grid_step: null state");
  TT_REQUIRE(nsteps >= 0 && std::isfinite(dt), "tt_grid_step: bad dt or nsteps");
  s->a.dt = dt;
  const bool nl = s->p.nonlinear != 0;
  switch (s->p.scheme) {
    case 3: nl ? grid_steps<3, true>(s, U, nsteps) : grid_steps<3, false>(s, U, nsteps); break;
    case 5: nl ? grid_steps<5, true>(s, U, nsteps) : grid_steps<5, false>(s, U, nsteps); break;
    default: nl ? grid_steps<55, true>(s, U, nsteps) : grid_steps<55, false>(s, U, nsteps);
  }
}

}  // namespace ttfv
