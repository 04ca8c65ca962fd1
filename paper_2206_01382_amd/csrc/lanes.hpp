// Butterfly lane exchange on a gfx950 wavefront without the LDS unit: lane x receives the value
// of lane x ^ X. Distances 1, 2, 4 and 8 stay inside a 16-lane row and map to DPP moves
// (quad permutations, half-row mirror, row rotation by 8); 16 and 32 use the gfx950 row-swap
// instructions (v_permlane16_swap / v_permlane32_swap) and a select.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fpp {

template <int X>
__device__ __forceinline__ uint32_t xor_lanes(uint32_t v) {
  static_assert(X == 1 || X == 2 || X == 4 || X == 8 || X == 16 || X == 32, "butterfly distance");
  const int s = (int)v;
  if constexpr (X == 1) {
    return (uint32_t)__builtin_amdgcn_mov_dpp(s, 0xB1, 0xF, 0xF, true);   // quad_perm 1,0,3,2
  } else if constexpr (X == 2) {
    return (uint32_t)__builtin_amdgcn_mov_dpp(s, 0x4E, 0xF, 0xF, true);   // quad_perm 2,3,0,1
  } else if constexpr (X == 4) {
    // mirror within 8 lanes (x -> 7 - x), then reverse each quad (x -> x ^ 3): x -> x ^ 4
    const int m = __builtin_amdgcn_mov_dpp(s, 0x141, 0xF, 0xF, true);      // row_half_mirror
    return (uint32_t)__builtin_amdgcn_mov_dpp(m, 0x1B, 0xF, 0xF, true);   // quad_perm 3,2,1,0
  } else if constexpr (X == 8) {
    return (uint32_t)__builtin_amdgcn_mov_dpp(s, 0x128, 0xF, 0xF, true);  // row_ror:8
  } else if constexpr (X == 16) {
    // after the swap, even rows of r[1] hold the odd rows' values and odd rows of r[0] the
    // even rows' values
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    return (__lane_id() & 16) ? r[0] : r[1];
  } else {
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return (__lane_id() & 32) ? r[0] : r[1];
  }
}

template <int X>
__device__ __forceinline__ float xor_lanes(float v) {
  return __uint_as_float(xor_lanes<X>(__float_as_uint(v)));
}

template <int X>
__device__ __forceinline__ int32_t xor_lanes(int32_t v) {
  return (int32_t)xor_lanes<X>((uint32_t)v);
}

template <int X>
__device__ __forceinline__ uint64_t xor_lanes(uint64_t v) {
  const uint32_t lo = xor_lanes<X>((uint32_t)v), hi = xor_lanes<X>((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// Lane x receives the value of lane x ^ M for M = 2^a - 1 (the mirror image inside aligned
// groups of M + 1 lanes): one DPP move up to M = 15 (quad reversal, half-row and row mirror),
// then the row swaps for the bits 16 and 32.
template <int M>
__device__ __forceinline__ uint32_t mirror_lanes(uint32_t v) {
  static_assert(M == 1 || M == 3 || M == 7 || M == 15 || M == 31 || M == 63, "mirror width");
  const int s = (int)v;
  if constexpr (M == 1) {
    return xor_lanes<1>(v);
  } else if constexpr (M == 3) {
    return (uint32_t)__builtin_amdgcn_mov_dpp(s, 0x1B, 0xF, 0xF, true);   // quad_perm 3,2,1,0
  } else if constexpr (M == 7) {
    return (uint32_t)__builtin_amdgcn_mov_dpp(s, 0x141, 0xF, 0xF, true);  // row_half_mirror
  } else {
    const uint32_t r = (uint32_t)__builtin_amdgcn_mov_dpp(s, 0x140, 0xF, 0xF, true);  // row_mirror
    if constexpr (M == 15) return r;
    else if constexpr (M == 31) return xor_lanes<16>(r);
    else return xor_lanes<32>(xor_lanes<16>(r));
  }
}

// Run-time distance (a compile-time constant after unrolling); distances >= 64 are invalid.
template <typename T>
__device__ __forceinline__ T xor_lanes_n(T v, int x) {
  switch (x) {
    case 1: return xor_lanes<1>(v);
    case 2: return xor_lanes<2>(v);
    case 4: return xor_lanes<4>(v);
    case 8: return xor_lanes<8>(v);
    case 16: return xor_lanes<16>(v);
    default: return xor_lanes<32>(v);
  }
}

}  // namespace fpp
