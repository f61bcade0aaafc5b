// Wavefront (64-lane) reductions of doubles without LDS traffic.
//
// Four DPP row_shr steps (1, 2, 4, 8; lanes shifted in from outside a row of 16 read 0)
// leave the sum of each row of 16 lanes in its lane 15; the four row sums are then read
// with v_readlane and added in a fixed order.  The result is the same in every lane and
// the summation order is fixed, so the reductions are deterministic.  wave_sum_n reduces
// N independent values with their DPP steps interleaved, which hides the DPP latency.
#pragma once
#include <hip/hip_runtime.h>

namespace ttfv {

template <int CTRL>
__device__ __forceinline__ double dpp_shift(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double lane_value(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

template <int N>
__device__ __forceinline__ void wave_sum_n(double (&v)[N]) {
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] += dpp_shift<0x111>(v[k]);   // row_shr:1
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] += dpp_shift<0x112>(v[k]);   // row_shr:2
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] += dpp_shift<0x114>(v[k]);   // row_shr:4
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] += dpp_shift<0x118>(v[k]);   // row_shr:8
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const double a = lane_value(v[k], 15), b = lane_value(v[k], 31);
    const double c = lane_value(v[k], 47), d = lane_value(v[k], 63);
    v[k] = (a + b) + (c + d);
  }
}

// Maximum over the wavefront with the same DPP pattern (lanes shifted in from outside a row
// read 0, so the inputs must not all be negative); NaNs are ignored.
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_shift<0x111>(v));
  v = fmax(v, dpp_shift<0x112>(v));
  v = fmax(v, dpp_shift<0x114>(v));
  v = fmax(v, dpp_shift<0x118>(v));
  const double a = lane_value(v, 15), b = lane_value(v, 31);
  const double c = lane_value(v, 47), d = lane_value(v, 63);
  return fmax(fmax(a, b), fmax(c, d));
}

__device__ __forceinline__ double wave_sum(double x) {
  double v[1] = {x};
  wave_sum_n<1>(v);
  return v[0];
}

}  // namespace ttfv

namespace ttfv {

// Sum over the 16 lanes of a DPP row, returned in every lane of the row: four row_ror
// steps (8, 4, 2, 1).  Every lane adds the same pairs in the same tree, so all 16 lanes
// hold bitwise-identical results.
template <int CTRL>
__device__ __forceinline__ float dpp_shift(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}

template <int N, typename T>
__device__ __forceinline__ void row16_sum_n(T (&v)[N]) {
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] += dpp_shift<0x128>(v[k]);   // row_ror:8
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] += dpp_shift<0x124>(v[k]);   // row_ror:4
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] += dpp_shift<0x122>(v[k]);   // row_ror:2
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] += dpp_shift<0x121>(v[k]);   // row_ror:1
}

}  // namespace ttfv

namespace ttfv {

// Sum over each group of 8 lanes (half a DPP row), returned in every lane of the group:
// quad_perm [1,0,3,2] and [2,3,0,1] add within quads, row_half_mirror adds the other quad.
// The pairs added are symmetric, so the 8 lanes hold bitwise-identical results.
template <int N>
__device__ __forceinline__ void group8_sum_n(double (&v)[N]) {
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] += dpp_shift<0xB1>(v[k]);    // quad_perm [1,0,3,2]
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] += dpp_shift<0x4E>(v[k]);    // quad_perm [2,3,0,1]
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] += dpp_shift<0x141>(v[k]);   // row_half_mirror
}

template <int LP, int N>
__device__ __forceinline__ void group_sum_n(double (&v)[N]) {
  static_assert(LP == 8 || LP == 16, "group of 8 or 16 lanes");
  if constexpr (LP == 8) group8_sum_n<N>(v);
  else row16_sum_n<N>(v);
}

}  // namespace ttfv

