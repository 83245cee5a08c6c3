// Cross-lane reductions of a wave64 by DPP moves (and one swizzle), in fixed orders.
#pragma once

#include <hip/hip_runtime.h>

namespace spa {

// DPP moves of a double (two 32-bit moves) and of a float (lanes of rows outside ROWS read
// 0); ds_swizzle exchange of lanes i and i ^ 16 inside each group of 32 lanes; a double
// read from one lane.
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ double dpp_move_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b), CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), CTRL, ROWS, 0xf, false);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ float dpp_move_f32(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xf, false));
}
__device__ __forceinline__ double swizzle_xor16_f64(double v) {
  constexpr int kXor16 = 0x1f | (0x10 << 10);   // bit mode: and 0x1f, or 0, xor 0x10
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_swizzle(static_cast<int>(b), kXor16);
  const int hi = __builtin_amdgcn_ds_swizzle(static_cast<int>(b >> 32), kXor16);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
__device__ __forceinline__ double read_lane_f64(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(static_cast<int>(b), l);
  const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), l);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// Sum over groups of LP lanes (a particle's row), the same value in every lane of a group: a
// butterfly of pairwise sums (each step adds a lane's value to its partner's, so both
// hold the same sum: addition commutes) by DPP quad permutations (lanes i ^ 1, i ^ 2), the
// half-row and row mirrors (i ^ 7, i ^ 15 inside 8 and 16 lanes), a swizzle (i ^ 16) and,
// for 64 lanes, the two halves read from lanes 0 and 32.
template <int LP>
__device__ __forceinline__ double lane_group_sum(double v) {
  static_assert(LP == 8 || LP == 16 || LP == 32 || LP == 64, "groups of 8 to 64 lanes");
  v += dpp_move_f64<0xB1>(v);                         // quad_perm [1,0,3,2]
  v += dpp_move_f64<0x4E>(v);                         // quad_perm [2,3,0,1]
  v += dpp_move_f64<0x141>(v);                        // row_half_mirror
  if constexpr (LP >= 16) v += dpp_move_f64<0x140>(v);  // row_mirror
  if constexpr (LP >= 32) v += swizzle_xor16_f64(v);
  if constexpr (LP == 64) v = read_lane_f64(v, 0) + read_lane_f64(v, 32);
  return v;
}

// Sum over the 64 lanes of a wave in a fixed order, returned in every lane: butterflies
// inside each row of 16 lanes (quad permutations, half-row and row mirrors), the row totals
// chained by the row-15 and row-31 broadcasts, the total read from lane 63.  Six dependent
// DPP steps instead of six dependent cross-lane permutes through the LDS unit.
__device__ __forceinline__ double wave_total_f64(double v) {
  v += dpp_move_f64<0xB1>(v);        // quad_perm [1,0,3,2]
  v += dpp_move_f64<0x4E>(v);        // quad_perm [2,3,0,1]
  v += dpp_move_f64<0x141>(v);       // row_half_mirror
  v += dpp_move_f64<0x140>(v);       // row_mirror
  v += dpp_move_f64<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_move_f64<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
  return read_lane_f64(v, 63);
}
__device__ __forceinline__ float wave_total_f32(float v) {
  v += dpp_move_f32<0xB1>(v);
  v += dpp_move_f32<0x4E>(v);
  v += dpp_move_f32<0x141>(v);
  v += dpp_move_f32<0x140>(v);
  v += dpp_move_f32<0x142, 0xA>(v);
  v += dpp_move_f32<0x143, 0xC>(v);
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

}  // namespace spa
