// WENO5 point reconstruction (Section 2.3) on five neighbouring cell averages, shared by the
// cross fiber functions and the full-grid comparator.
//   smoothness: the Jiang-Shu indicators beta_0..beta_2 about the middle cell;
//   weno_combine: candidates sum_l C[r][l] v[2 - r + l], weights gam_r / (beta_r + eps)^2
//                 normalised;
//   weno_face: Step 1, the value at the right face of the middle cell;
//   weno_quad: Step 2, the value at Gauss point m; the middle point, whose linear weights
//              are not all positive, takes the positive/negative split (gamma+, gamma-,
//              sigma+, sigma-).
#pragma once
#include "common.h"

namespace ttfv {

struct WenoArgs {
  WenoTables t;
  double eps;
};

__device__ __forceinline__ void smoothness(const double *v, double *beta) {
  // v[0..4] = cells c-2 .. c+2
  const double a = v[2] - 2 * v[3] + v[4], b = 3 * v[2] - 4 * v[3] + v[4];
  const double c = v[1] - 2 * v[2] + v[3], d = v[1] - v[3];
  const double e = v[0] - 2 * v[1] + v[2], f = v[0] - 4 * v[1] + 3 * v[2];
  beta[0] = 13.0 / 12.0 * a * a + 0.25 * b * b;
  beta[1] = 13.0 / 12.0 * c * c + 0.25 * d * d;
  beta[2] = 13.0 / 12.0 * e * e + 0.25 * f * f;
}

__device__ __forceinline__ double weno_combine(const double (*C)[3], const double *gam,
                                               const double *beta, const double *v, double eps) {
  double cand[3], al[3], s = 0.0;
  for (int r = 0; r < 3; ++r) {
    double acc = 0.0;
    for (int l = 0; l < 3; ++l) acc += C[r][l] * v[2 - r + l];
    cand[r] = acc;
    const double be = beta[r] + eps;
    al[r] = gam[r] / (be * be);
    s += al[r];
  }
  return (al[0] * cand[0] + al[1] * cand[1] + al[2] * cand[2]) / s;
}

__device__ __forceinline__ double weno_face(const WenoArgs &w, const double *v) {
  double beta[3];
  smoothness(v, beta);
  return weno_combine(w.t.face_C, w.t.face_d, beta, v, w.eps);
}

__device__ __forceinline__ double weno_quad(const WenoArgs &w, const double *v, int m) {
  double beta[3];
  smoothness(v, beta);
  if (m == 1) {
    const double up = weno_combine(w.t.quad_C[1], w.t.gp, beta, v, w.eps);
    const double um = weno_combine(w.t.quad_C[1], w.t.gm, beta, v, w.eps);
    return w.t.sp * up - w.t.sm * um;
  }
  return weno_combine(w.t.quad_C[m], w.t.quad_g[m], beta, v, w.eps);
}

}  // namespace ttfv
