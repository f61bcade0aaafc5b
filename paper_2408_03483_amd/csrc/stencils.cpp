// Reconstruction constants of Section 2.3, derived at start-up from their definition:
// the value at a point x0 of cell j = [-1/2, 1/2] (cell units) of the polynomial whose
// averages over cells at integer offsets o_l equal the given averages.  The weights solve
//     sum_l c_l * avg_{[o_l - 1/2, o_l + 1/2]} y^p = x0^p,  p = 0 .. len - 1,
// here in long double by Gaussian elimination with partial pivoting.  Step 1 evaluates at
// the face x0 = 1/2, Step 2 at the Gauss-Legendre points (2 points -/+ 1/(2 sqrt 3) for
// third order, 3 points -sqrt(15)/10, 0, sqrt(15)/10 for fifth order, ascending).
#include <cmath>
#include <vector>

#include "common.h"

namespace ttfv {
namespace {

using LD = long double;

std::vector<LD> point_weights(const std::vector<int> &off, LD x0) {
  const int n = (int)off.size();
  std::vector<std::vector<LD>> A(n, std::vector<LD>(n + 1));
  LD xp = 1.0L;
  for (int p = 0; p < n; ++p) {
    for (int l = 0; l < n; ++l) {
      const LD lo = off[l] - 0.5L, hi = off[l] + 0.5L;
      A[p][l] = (std::pow(hi, p + 1) - std::pow(lo, p + 1)) / (LD)(p + 1);
    }
    A[p][n] = xp;
    xp *= x0;
  }
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r][c]) > std::fabs(A[piv][c])) piv = r;
    std::swap(A[c], A[piv]);
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const LD f = A[r][c] / A[c][c];
      for (int k = c; k <= n; ++k) A[r][k] -= f * A[c][k];
    }
  }
  std::vector<LD> w(n);
  for (int i = 0; i < n; ++i) w[i] = A[i][n] / A[i][i];
  return w;
}

std::vector<int> range(int a, int b) {
  std::vector<int> v;
  for (int i = a; i <= b; ++i) v.push_back(i);
  return v;
}

std::vector<LD> gauss_points(int nq) {
  if (nq == 2) {
    const LD d = 1.0L / (2.0L * std::sqrt(3.0L));
    return {-d, d};
  }
  const LD d = std::sqrt(15.0L) / 10.0L;
  return {-d, 0.0L, d};
}

std::vector<LD> gauss_weights(int nq) {
  if (nq == 2) return {0.5L, 0.5L};
  return {5.0L / 18.0L, 8.0L / 18.0L, 5.0L / 18.0L};
}

// candidate stencil r of order 2k+1 covers cells j-r .. j-r+k
std::vector<std::vector<LD>> candidates(int k, LD x0) {
  std::vector<std::vector<LD>> C;
  for (int r = 0; r <= k; ++r) C.push_back(point_weights(range(-r, -r + k), x0));
  return C;
}

// linear weights gamma with sum_r gamma_r C_r = full 5-cell stencil (k = 2)
std::vector<LD> linear_weights5(LD x0) {
  auto C = candidates(2, x0);
  auto F = point_weights(range(-2, 2), x0);
  const LD g0 = F[4] / C[0][2];   // offset +2 only in stencil 0
  const LD g2 = F[0] / C[2][0];   // offset -2 only in stencil 2
  return {g0, 1.0L - g0 - g2, g2};
}

}  // namespace

StencilSet derive_stencils(int scheme) {
  StencilSet s;
  s.k = (scheme == 3) ? 1 : 2;
  s.nq = (scheme == 3) ? 2 : 3;
  auto face = point_weights(range(-s.k, s.k), 0.5L);
  for (int o = 0; o <= 2 * s.k; ++o) s.face[o] = (double)face[o];
  auto pts = gauss_points(s.nq);
  auto gw = gauss_weights(s.nq);
  for (int m = 0; m < s.nq; ++m) {
    auto w = point_weights(range(-s.k, s.k), pts[m]);
    for (int o = 0; o <= 2 * s.k; ++o) s.quad[m][o] = (double)w[o];
    s.gw[m] = (double)gw[m];
  }
  return s;
}

WenoTables derive_weno_tables() {
  WenoTables t{};
  auto fc = candidates(2, 0.5L);
  auto fd = linear_weights5(0.5L);
  for (int r = 0; r < 3; ++r) {
    t.face_d[r] = (double)fd[r];
    for (int l = 0; l < 3; ++l) t.face_C[r][l] = (double)fc[r][l];
  }
  auto pts = gauss_points(3);
  for (int m = 0; m < 3; ++m) {
    auto C = candidates(2, pts[m]);
    auto g = linear_weights5(pts[m]);
    for (int r = 0; r < 3; ++r) {
      t.quad_g[m][r] = (double)g[r];
      for (int l = 0; l < 3; ++l) t.quad_C[m][r][l] = (double)C[r][l];
    }
    if (m == 1) {
      // negative linear weights at the middle point: split gamma = gamma+ - gamma- with
      // gamma+ = (gamma + 3|gamma|)/2, each part normalised by its sum sigma+-
      LD gp[3], gm[3], sp = 0, sm = 0;
      for (int r = 0; r < 3; ++r) {
        gp[r] = (g[r] + 3.0L * std::fabs(g[r])) / 2.0L;
        gm[r] = gp[r] - g[r];
        sp += gp[r];
        sm += gm[r];
      }
      for (int r = 0; r < 3; ++r) {
        t.gp[r] = (double)(gp[r] / sp);
        t.gm[r] = (double)(gm[r] / sm);
      }
      t.sp = (double)sp;
      t.sm = (double)sm;
    }
  }
  return t;
}

}  // namespace ttfv
