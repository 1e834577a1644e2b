// Lane exchanges inside a DPP row of 16 lanes (pure VALU data movement: no
// trip through the LDS crossbar that __shfl_xor takes).
//   0xB1: quad_perm [1, 0, 3, 2]   (partner lane ^ 1)
//   0x4E: quad_perm [2, 3, 0, 1]   (partner lane ^ 2)
//   0x141: row_half_mirror         (lane 7 - i within each half row)
//   0x140: row_mirror              (lane 15 - i within the row)
#pragma once
#include <hip/hip_runtime.h>

namespace slar {

template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// Sum over aligned groups of N = 2, 4, 8 or 16 lanes; every lane of a group
// receives the group's total.  After the quad sums every lane of a quad
// holds the same value, so the mirrors pair whole quads and half rows.
template <int N, typename T>
__device__ __forceinline__ T group_sum(T v) {
  static_assert(N == 2 || N == 4 || N == 8 || N == 16, "group width");
  v += dpp_move<0xB1>(v);
  if (N >= 4) v += dpp_move<0x4E>(v);
  if (N >= 8) v += dpp_move<0x141>(v);
  if (N >= 16) v += dpp_move<0x140>(v);
  return v;
}

}  // namespace slar
