// Cross-lane moves by DPP (data-parallel primitives of the VALU): a lane takes
// the value of another lane of its group of four or of its 16-lane row in the
// same instruction stream, without an LDS round trip. Used where a cell's or a
// face's 4 x 4 grid of points fills one 16-lane row (point (a, b) in lane
// a + 4 b of the row), so that the 1D contractions across the grid read their
// operands from the neighbouring lanes.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dgi {

template <typename T, int CTRL>
__device__ __forceinline__ T dpp_move(T v) {
  if constexpr (sizeof(T) == 8) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(T, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
  } else {
    return __builtin_bit_cast(T, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
  }
}

// every lane gets the value of lane J of its group of four (quad_perm)
template <int J, typename T>
__device__ __forceinline__ T quad_bcast(T v) {
  return dpp_move<T, J | (J << 2) | (J << 4) | (J << 6)>(v);
}

// lane i gets the value of lane i - R (mod 16) of its 16-lane row (row_ror)
template <int R, typename T>
__device__ __forceinline__ T row_rot(T v) {
  if constexpr (R == 0)
    return v;
  else
    return dpp_move<T, 0x120 + R>(v);
}

// On a 4 x 4 grid in a 16-lane row (the lane's point (a, b)): the
// contractions sum_j M[a][j] v(j, b) and sum_j M[b][j] v(a, j) of the lanes'
// values v, M row-major in `m` (LDS or registers); row_rot<4k> brings the
// value of point (a, b - k mod 4).
template <typename T>
__device__ __forceinline__ void grid4_rows(const T* __restrict__ m, int a, int b, T v, T& va, T& vb) {
  va = fma(m[a * 4 + 0], quad_bcast<0>(v), T(0));
  va = fma(m[a * 4 + 1], quad_bcast<1>(v), va);
  va = fma(m[a * 4 + 2], quad_bcast<2>(v), va);
  va = fma(m[a * 4 + 3], quad_bcast<3>(v), va);
  vb = fma(m[b * 4 + b], v, T(0));
  vb = fma(m[b * 4 + ((b - 1) & 3)], row_rot<4>(v), vb);
  vb = fma(m[b * 4 + ((b - 2) & 3)], row_rot<8>(v), vb);
  vb = fma(m[b * 4 + ((b - 3) & 3)], row_rot<12>(v), vb);
}

}  // namespace dgi
