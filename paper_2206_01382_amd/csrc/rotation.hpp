// The structured rotation of the query-side hash kernels (Section 2.2 Eq. 1; Section 3.4: three
// rounds of "flip signs by a random +-1 diagonal, then unnormalised Walsh-Hadamard transform"),
// held in registers across the lanes of a wavefront.
//
// An item (vector, function) spans LPI = P / E lanes; lane x of the item holds the E consecutive
// elements j = x * E + e. Butterfly stages h < E pair register e with e ^ h inside the lane;
// stages h >= E pair lane x with x ^ (h / E) (the lower lane adds, the upper subtracts) through
// DPP / row-swap lane exchanges; stages run in the order h = 1, 2, ..., P/2, and every operation
// is one float32 rounding of a + b or a - b, so the results are those of that expression tree.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lanes.hpp"

namespace fpp {

__device__ __forceinline__ float flip(float v, uint32_t mask) {
  return __uint_as_float(__float_as_uint(v) ^ mask);
}

template <int P>
struct QLayout {
  static constexpr int E = P < 16 ? P : (P / 64 > 16 ? P / 64 : 16);  // elements per lane
  static constexpr int LPI = P / E;                                 // lanes per item
  static constexpr int IPW = 64 / LPI;                              // items per wavefront
};

// v + (v of lane ^ X) * mul. For X = 1, 2 and 8 the partner is a DPP operand of one v_fmac (quad
// permutes, and a rotation by 8 within a 16-lane row), for X = 4 after one DPP move; the s_nop
// gives the two wait states a DPP read needs after a VALU write of its source. Other distances go
// through xor_lanes.
template <int X>
__device__ __forceinline__ float fmac_xor(float v, float mul) {
  float src = v;
  if constexpr (X == 1) {
    asm volatile("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf" : "+v"(v) : "v"(src), "v"(mul));
  } else if constexpr (X == 2) {
    asm volatile("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf" : "+v"(v) : "v"(src), "v"(mul));
  } else if constexpr (X == 8) {
    asm volatile("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 row_ror:8 row_mask:0xf bank_mask:0xf" : "+v"(v) : "v"(src), "v"(mul));
  } else if constexpr (X == 4) {
    // x ^ 4 = (x ^ 7) ^ 3: a half-row mirror move, then the quad reversal as the DPP operand
    src = __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x141, 0xF, 0xF, true));
    asm volatile("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 quad_perm:[3,2,1,0] row_mask:0xf bank_mask:0xf" : "+v"(v) : "v"(src), "v"(mul));
  } else {
    v = __builtin_fmaf(xor_lanes<X>(v), mul, v);
  }
  return v;
}
__device__ __forceinline__ float fmac_xor_n(float v, int x, float mul) {
  switch (x) {
    case 1: return fmac_xor<1>(v, mul);
    case 2: return fmac_xor<2>(v, mul);
    case 4: return fmac_xor<4>(v, mul);
    case 8: return fmac_xor<8>(v, mul);
    case 16: return fmac_xor<16>(v, mul);
    default: return fmac_xor<32>(v, mul);
  }
}

// Elements j0 .. j0 + E - 1 of a row, zero at and past d. VEC: the row is 16-byte aligned, so
// whole float4 groups below d take one load and only the group holding d is read elementwise.
template <int E, bool VEC>
__device__ __forceinline__ void load_elems(const float* row, int d, int j0, float (&v)[E]) {
  if constexpr (VEC && E % 4 == 0) {
#pragma unroll
    for (int g4 = 0; g4 < E / 4; ++g4) {
      const int j = j0 + 4 * g4;
      if (j + 4 <= d) {
        const float4 x = *reinterpret_cast<const float4*>(row + j);
        v[4 * g4] = x.x;
        v[4 * g4 + 1] = x.y;
        v[4 * g4 + 2] = x.z;
        v[4 * g4 + 3] = x.w;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) v[4 * g4 + e] = (j + e < d) ? row[j + e] : 0.0f;
      }
    }
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = (j0 + e < d) ? row[j0 + e] : 0.0f;
  }
}

// Sign masks (0 or the float sign bit) of the three diagonals of function tf for elements
// j0 .. j0 + E - 1; sign_mask is [functions][3][P].
template <int P, int E>
__device__ __forceinline__ void load_sign_masks(const uint32_t* sign_mask, int tf, int j0,
                                                uint32_t (&smv)[3][E]) {
  const uint32_t* sm = sign_mask + (size_t)tf * 3 * P + j0;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    if constexpr (E % 4 == 0) {
#pragma unroll
      for (int g4 = 0; g4 < E / 4; ++g4) {
        const uint4 w = *reinterpret_cast<const uint4*>(sm + r * P + 4 * g4);
        smv[r][4 * g4] = w.x;
        smv[r][4 * g4 + 1] = w.y;
        smv[r][4 * g4 + 2] = w.z;
        smv[r][4 * g4 + 3] = w.w;
      }
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) smv[r][e] = sm[r * P + e];
    }
  }
}

// The three rounds on the item's elements (lane li of the item holds v[0..E)); afterwards v holds
// the true outputs y_j, j = li * E + e.
// Cross-lane stages use one fused multiply-add: v + w * (+1) in the lower lane of a pair and
// v - w (= -(w - v), the same rounding) in the upper one, so an upper lane holds the negated
// value. Partners of a later stage differ only in that stage's lane bit, so they carry the
// same sign; after a round lane li holds (-1)^popcount(li) times the true values, which the
// next round's sign flip and the end of the rotation undo with one XOR of the sign bit. (Only
// the sign of a zero can differ, and neither |y| nor the code rule y >= 0 sees it.)
template <int P>
__device__ __forceinline__ void rotate_item(float (&v)[QLayout<P>::E],
                                            const uint32_t (&smv)[3][QLayout<P>::E], int li) {
  constexpr int E = QLayout<P>::E, LPI = QLayout<P>::LPI;
  const uint32_t lane_sign = (__popc((unsigned)li) & 1) ? 0x80000000u : 0u;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = flip(v[e], r == 0 ? smv[r][e] : (smv[r][e] ^ lane_sign));
#pragma unroll
    for (int h = 1; h < E; h <<= 1) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        if ((e & h) == 0) {
          const float a = v[e], b = v[e + h];
          v[e] = a + b;
          v[e + h] = a - b;
        }
      }
    }
#pragma unroll
    for (int hl = 1; hl < LPI; hl <<= 1) {
      const float mul = (li & hl) ? -1.0f : 1.0f;
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = fmac_xor_n(v[e], hl, mul);
    }
  }
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = flip(v[e], lane_sign);
}

// Packed signs: bit j % 32 of word j / 32 of round r of function tf is set when element j of
// that diagonal is -1; sign_bits is [functions][3][WPR] with WPR = max(1, P / 32) words per round.
// Lane li of an item needs the E <= 16 bits of elements j0 .. j0 + E - 1 of each round, returned
// in the low E bits of w[r].
template <int P, int E>
__device__ __forceinline__ void load_sign_bits(const uint32_t* sign_bits, int tf, int j0,
                                               uint32_t (&w)[3]) {
  static_assert(E <= 16, "at most 16 elements per lane");
  constexpr int WPR = P / 32 > 1 ? P / 32 : 1;
  const uint32_t* b = sign_bits + (size_t)tf * 3 * WPR + j0 / 32;
#pragma unroll
  for (int r = 0; r < 3; ++r) w[r] = b[r * WPR] >> (j0 % 32);
}

// rotate_item with the diagonals as packed bits (load_sign_bits): the same operations in the same
// order, so the same values; the sign of element e of round r is bit e of w[r].
template <int P>
__device__ __forceinline__ void rotate_item_bits(float (&v)[QLayout<P>::E], const uint32_t (&w)[3],
                                                 int li) {
  constexpr int E = QLayout<P>::E, LPI = QLayout<P>::LPI;
  const uint32_t lane_sign = (__popc((unsigned)li) & 1) ? 0x80000000u : 0u;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    // every bit of the lane's word xor the lane's sign: one operation for the round, not per
    // element
    const uint32_t wr = r == 0 ? w[r] : (w[r] ^ (lane_sign ? 0xffffffffu : 0u));
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = flip(v[e], (wr << (31 - e)) & 0x80000000u);
#pragma unroll
    for (int h = 1; h < E; h <<= 1) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        if ((e & h) == 0) {
          const float a = v[e], b = v[e + h];
          v[e] = a + b;
          v[e + h] = a - b;
        }
      }
    }
#pragma unroll
    for (int hl = 1; hl < LPI; hl <<= 1) {
      const float mul = (li & hl) ? -1.0f : 1.0f;
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = fmac_xor_n(v[e], hl, mul);
    }
  }
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = flip(v[e], lane_sign);
}

}  // namespace fpp
