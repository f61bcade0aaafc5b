// Decision rules evaluated both on the host (the dynamic path, which reads singular values and
// pivots back) and on the device (fixed shapes, fixed.hip): one definition, taken in the same
// order on both sides, so that a fixed-shape step makes the dynamic step's decisions.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace ttfv {

// Kept rank of a truncation: the fewest leading singular values (s descending, m of them)
// whose discarded tail is within eps of the total, at most rmax, and never a direction at or
// below the SVD's norm floor max(1e-17, floor_rel) ||s||: the Jacobi SVD does not rotate such
// columns, so they are not orthogonal to the others and keeping one would turn the projection
// Q U_k U_k^T into a non-projection.  A tolerance below that floor (below round-off) therefore
// keeps every direction above it.  tail: m + 1 doubles of scratch.  capped (optional): the rank
// cap, not eps or the floor, set k.
__host__ __device__ inline int rule_trunc_rank(const double *s, int m, double eps, int rmax,
                                               double floor_rel, double *tail, bool *capped) {
  tail[m] = 0.0;
  for (int i = m - 1; i >= 0; --i) tail[i] = tail[i + 1] + s[i] * s[i];
  const double thr = eps * eps * tail[0];
  int k = m;
  for (int kk = 1; kk <= m; ++kk)
    if (tail[kk] <= thr) {
      k = kk;
      break;
    }
  const double fl = fmax(1e-17, floor_rel) * sqrt(tail[0]);
  int kf = 0;
  while (kf < m && s[kf] > fl) ++kf;
  if (kf < 1) kf = 1;
  if (k > kf) k = kf;
  const bool cap = k > rmax;
  if (k > rmax) k = rmax;
  if (k < 1) k = 1;
  if (capped) *capped = cap && (tail[k] > thr);
  return k;
}

// Directions an orthogonalisation keeps: the leading singular values above drop times the
// largest (none when the largest is zero).
__host__ __device__ inline int rule_kept_directions(const double *s, int m, double drop) {
  int k = 0;
  if (s[0] > 0.0)
    while (k < m && s[k] > drop * s[0]) ++k;
  return k;
}

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): the state advances by the golden-ratio
// increment and the output is its finalising mix.
__host__ __device__ inline uint64_t rule_splitmix64(uint64_t &state) {
  state += 0x9E3779B97F4A7C15ull;
  uint64_t z = state;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Seeded fresh columns of a cross sweep: J[0 .. have) holds distinct indices; up to `count`
// indices in [0, n) not yet in J are appended, drawn as SplitMix64 outputs mod n from `key`,
// at most 64 (count + 1) draws and never more than n indices in all.  Returns the number
// appended.
__host__ __device__ inline int rule_kicks(int *J, int have, int n, int count, uint64_t key) {
  uint64_t state = key;
  int out = 0, tries = 0;
  while (out < count && have + out < n && tries < 64 * (count + 1)) {
    const int idx = (int)(rule_splitmix64(state) % (uint64_t)n);
    ++tries;
    bool seen = false;
    for (int t = 0; t < have + out; ++t)
      if (J[t] == idx) {
        seen = true;
        break;
      }
    if (!seen) J[have + out++] = idx;
  }
  return out;
}

}  // namespace ttfv
