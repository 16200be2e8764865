// Wavefront-wide operations shared by the device kernels (64-lane waves).
#pragma once

#include <hip/hip_runtime.h>

namespace peers {

// One DPP move of a double within rows of 16 lanes (quad_perm / row mirrors).
template <int CTRL>
__device__ __forceinline__ double dpp(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}

// A DPP move of a double into the rows enabled by ROWS; the other rows of the
// result are left undefined.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_rows(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, ROWS, 0xf, false);
  return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes, in a fixed order, without LDS traffic, left in lane
// 63 (other lanes hold partial or undefined values): butterflies inside each
// row of 16 (quad_perm [1,0,3,2], [2,3,0,1], row_half_mirror, row_mirror)
// leave row r's sum S_r in all its lanes; then row_bcast:15 adds S_2 (lane
// 47) into row 3 and S_0 into row 1, and row_bcast:31 adds row 1's lane 31
// into row 3, so lane 63 holds (S_3 + S_2) + (S_1 + S_0). Lane 63 only reads
// rows that every step wrote.
__device__ __forceinline__ double wave_sum_to_lane63(double v) {
  v += dpp<0xB1>(v);
  v += dpp<0x4E>(v);
  v += dpp<0x141>(v);
  v += dpp<0x140>(v);
  v += dpp_rows<0x142, 0xA>(v);
  v += dpp_rows<0x143, 0xC>(v);
  return v;
}

// The lane-63 sum above as a wave-uniform value.
__device__ __forceinline__ double wave_sum(double v) {
  v = wave_sum_to_lane63(v);
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 63),
                          __builtin_amdgcn_readlane(__double2loint(v), 63));
}

}  // namespace peers
