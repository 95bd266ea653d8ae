// Wave-level FP64 sums on CDNA (wave64) with DPP lane moves instead of LDS
// permutes: within each row of 16 lanes, exchanges across lanes xor 1, xor 2
// (quad permutes), then the half-row and row mirrors leave every lane of the
// row holding the same row sum (each step adds two values in either order,
// which is exact-commutative); the rows are then combined from lanes 0, 16,
// 32, 48 with readlane in a fixed order.  Deterministic and identical on
// every lane that receives it.
#pragma once

#include <hip/hip_runtime.h>

namespace lobpcg {

template <int kCtrl>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), kCtrl, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), kCtrl, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double lane_value(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Every lane receives the sum over its row of 16 lanes.
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]: lane xor 1
  v += dpp_move<0x4E>(v);   // quad_perm [2,3,0,1]: lane xor 2
  v += dpp_move<0x141>(v);  // row_half_mirror: the two quads of a half row
  v += dpp_move<0x140>(v);  // row_mirror: the two half rows
  return v;
}

// Sum over the 64 lanes of the wave, on every lane.
__device__ __forceinline__ double wave64_sum(double v) {
  v = row16_sum(v);
  return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}

// Sum over each half wave (lanes 0-31, 32-63), on the lanes of that half.
__device__ __forceinline__ double half32_sum(double v) {
  v = row16_sum(v);
  const double s0 = lane_value(v, 0) + lane_value(v, 16);
  const double s1 = lane_value(v, 32) + lane_value(v, 48);
  return (threadIdx.x & 32) ? s1 : s0;
}

}  // namespace lobpcg
