// Query-side cross-polytope hashing on gfx950 (Section 2.2 Eq. 1; Section 3.4 structured
// spinners), and the dispatch of the build-side kernels.
//
// Each hash function rotates the zero-padded vector with three rounds of "flip signs, then
// unnormalised Walsh-Hadamard transform" (stage h = 1, 2, ..., P/2; the lower element of a pair
// becomes a + b, the upper a - b) and reads the first D outputs y_i. Sign flips are XORs of the
// sign bit; there are no multiplications, so the float32 results are those of that order.
#include <algorithm>

#include "fpp_internal.hpp"
#include "lanes.hpp"

namespace fpp {

#define FPP_DECL_BUILD(K)                                                                    \
  hipError_t launch_hash_build_k##K##_short(const fpp_index*, int, int, uint32_t*, float*,     \
                                            hipStream_t);                                     \
  hipError_t launch_hash_build_k##K##_long(const fpp_index*, int, int, uint32_t*, float*, hipStream_t);
FPP_DECL_BUILD(1)
FPP_DECL_BUILD(4)
FPP_DECL_BUILD(16)
#undef FPP_DECL_BUILD

namespace {

__device__ __forceinline__ float flip(float v, uint32_t mask) {
  return __uint_as_float(__float_as_uint(v) ^ mask);
}

// ------------------------------------------------------------------------------------------
// Query side, everything in registers. An item (vector, function) spans LPI = P / E lanes of a
// wavefront; lane x of the item holds the E consecutive elements j = x * E + e. Butterfly stages
// h < E pair register e with e ^ h inside the lane; stages h >= E pair lane x with x ^ (h / E)
// (the lower lane adds, the upper subtracts) through DPP / row-swap lane exchanges; stages run in
// the order h = 1, 2, ..., P/2.
// The D keys (|y_i| bits << 32 | (0xffff - i) << 1 | sign) are then bitonic-sorted descending in
// the same layout, which orders the list by (|y| desc, i asc) and carries the code bit.
// ------------------------------------------------------------------------------------------
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

// Exact 64-bit list key: |y| bits << 32 | (0xffff - i) << 1 | sign; descending order of keys is
// (|y| desc, i asc), and the low bit carries the code (i or i + D).
__device__ __forceinline__ uint64_t exact_key(float y, int i) {
  const uint32_t neg = y >= 0.0f ? 0u : 1u;
  return ((uint64_t)__float_as_uint(fabsf(y)) << 32) | ((uint32_t)(0xffff - i) << 1) | neg;
}

__device__ __forceinline__ void ce_desc(uint32_t& a, uint32_t& b) {
  const uint32_t hi = a > b ? a : b, lo = a > b ? b : a;
  a = hi;
  b = lo;
}
__device__ __forceinline__ void ce_desc(uint64_t& a, uint64_t& b) {
  const bool sw = a < b;
  const uint64_t x = sw ? b : a, y = sw ? a : b;
  a = x;
  b = y;
}

// Batcher's odd-even merge sort of n keys: comparator number c (in the network's order) as
// lo * 1024 + hi, or -1 past the last one; all comparators keep the larger key at lo. 63
// comparators for n = 16 and 19 for n = 8, against 80 and 24 for the bitonic network.
constexpr int odd_even_pair(int n, int c) {
  int idx = 0;
  for (int p = 1; p < n; p <<= 1)
    for (int k = p; k >= 1; k >>= 1)
      for (int j = k % p; j + k < n; j += 2 * k)
        for (int i = 0; i < k && i < n - j - k; ++i)
          if ((i + j) / (2 * p) == (i + j + k) / (2 * p)) {
            if (idx == c) return (i + j) * 1024 + (i + j + k);
            ++idx;
          }
  return -1;
}

template <int E, int C = 0>
__device__ __forceinline__ void lane_sort_desc(uint32_t (&key)[E]) {
  constexpr int pr = odd_even_pair(E, C);
  if constexpr (pr >= 0) {
    ce_desc(key[pr / 1024], key[pr % 1024]);
    lane_sort_desc<E, C + 1>(key);
  }
}

// Bitonic merges (descending) in the item layout: lane li holds positions li * E + e. Every merge
// of two sorted blocks of k / 2 starts by comparing position p with its mirror image p ^ (k - 1)
// inside the block, which leaves two bitonic halves, every key of the first at least every key
// of the second; half-cleaners at distances k / 4, ..., 1 then sort them. All compare-exchanges
// keep the larger key in front, so no block runs in the other direction. Inside a lane the pairs
// are registers; across lanes the partner comes from one lane exchange, and the median of (key,
// partner, 0 or ~0) keeps the larger in the lower lane of the pair and the smaller in the upper.
template <int E, int J>
__device__ __forceinline__ void half_clean(uint32_t (&key)[E], int li) {
  if constexpr (J > 0) {
    if constexpr (J < E) {
#pragma unroll
      for (int e = 0; e < E; ++e)
        if ((e & J) == 0) ce_desc(key[e], key[e | J]);
    } else {
      const uint32_t lim = (li & (J / E)) == 0 ? 0xffffffffu : 0u;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const uint32_t o = xor_lanes<J / E>(key[e]);
        const uint32_t mx = key[e] > o ? key[e] : o, mn = key[e] > o ? o : key[e];
        const uint32_t c = mx < lim ? mx : lim;
        key[e] = mn > c ? mn : c;
      }
    }
    half_clean<E, J / 2>(key, li);
  }
}

template <int P, int E, int K>
__device__ __forceinline__ void sort_levels(uint32_t (&key)[E], int li, int D) {
  if constexpr (K <= P) {
    if (K > D) return;
    if constexpr (K <= E) {
#pragma unroll
      for (int e = 0; e < E; ++e)
        if ((e & (K >> 1)) == 0) ce_desc(key[e], key[e ^ (K - 1)]);
    } else {
      // position li * E + e pairs with (li ^ (K / E - 1)) * E + (E - 1 - e)
      const uint32_t lim = (li & (K / (2 * E))) == 0 ? 0xffffffffu : 0u;
#pragma unroll
      for (int e = 0; e < E / 2; ++e) {
        const uint32_t a = key[e], b = key[E - 1 - e];
        const uint32_t pa = mirror_lanes<K / E - 1>(b), pb = mirror_lanes<K / E - 1>(a);
        const uint32_t mxa = a > pa ? a : pa, mna = a > pa ? pa : a;
        const uint32_t mxb = b > pb ? b : pb, mnb = b > pb ? pb : b;
        const uint32_t ca = mxa < lim ? mxa : lim, cb = mxb < lim ? mxb : lim;
        key[e] = mna > ca ? mna : ca;
        key[E - 1 - e] = mnb > cb ? mnb : cb;
      }
    }
    half_clean<E, K / 4>(key, li);
    sort_levels<P, E, K * 2>(key, li, D);
  }
}

// Sorts the first D keys (D a power of two <= P) descending: each lane's E keys with the odd-even
// network when D >= E, then the bitonic merges across lanes (for D < E, bitonic merges only).
template <int P, int E, int LPI>
__device__ __forceinline__ void sort32_desc(uint32_t (&key)[E], int li, int j0, int D) {
  (void)j0;
  if (D >= E) {
    // each lane's E keys with the odd-even network, then the bitonic merges across lanes
    lane_sort_desc<E>(key);
    sort_levels<P, E, 2 * E>(key, li, D);
  } else {
    sort_levels<P, E, 2>(key, li, D);
  }
}

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Bitonic sort (descending) of an item's first D exact keys in its LDS slot, with run-time
// loops: the rare fallback when the transposition steps leave a list out of order.
template <int E>
__device__ __noinline__ void lds_sort64_desc(uint64_t* ks, int j0, int D) {
  for (int k = 2; k <= D; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int i = j0 + e, p = i ^ j;
        if (i < D && p > i) {
          const uint64_t a = ks[i], b = ks[p];
          if (((i & k) == 0) ? (a < b) : (a > b)) {
            ks[i] = b;
            ks[p] = a;
          }
        }
      }
      wave_lds_sync();
    }
  }
}

// Element p + 1 of the list from the next lane (wave_shl:1 DPP; lanes past the item or past D
// are never used).
__device__ __forceinline__ uint64_t from_next_lane(uint64_t v) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, 0x130, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), 0x130, 0xF, 0xF, false);
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}
__device__ __forceinline__ uint64_t from_prev_lane(uint64_t v) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, 0x138, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), 0x138, 0xF, 0xF, false);
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

// One even and one odd transposition step (descending) over positions [0, D).
template <int E, int LPI>
__device__ __forceinline__ void repair_runs(uint64_t (&key)[E], int j0, int D) {
#pragma unroll
  for (int e = 0; e + 1 < E; e += 2)
    if (j0 + e + 1 < D) ce_desc(key[e], key[e + 1]);
#pragma unroll
  for (int e = 1; e + 1 < E; e += 2)
    if (j0 + e + 1 < D) ce_desc(key[e], key[e + 1]);
  if constexpr (E % 2 == 0) {
    // pair (last element of lane li, first element of lane li + 1): both lanes exchange the
    // values before either changes; lane li keeps the larger, lane li + 1 the smaller
    const uint64_t nxt = from_next_lane(key[0]);
    const uint64_t prv = from_prev_lane(key[E - 1]);
    const bool has_next = j0 + E < D;        // implies li + 1 < LPI (D <= P)
    const bool has_prev = j0 > 0 && j0 < D;
    if (has_next && key[E - 1] < nxt) key[E - 1] = nxt;
    if (has_prev && prv < key[0]) key[0] = prv;
  }
}

template <int E, int LPI>
__device__ __forceinline__ bool out_of_order(const uint64_t (&key)[E], int j0, int D) {
  bool bad = false;
#pragma unroll
  for (int e = 0; e + 1 < E; ++e)
    if (j0 + e + 1 < D) bad |= key[e] <= key[e + 1];
  const uint64_t nxt = from_next_lane(key[0]);
  if (j0 + E < D) bad |= key[E - 1] <= nxt;
  return bad;
}

// Turns an item's first Dn sorted 32-bit keys (lane li holds positions li * E .. + E; Dn <= D, the
// keys' index bits and the codes refer to the D outputs) into exact 64-bit keys (values from the
// item's LDS copy yl, by index), repairs and, if needed, re-sorts them, and stores the first W
// entries of the list at ola / olc.
template <int E, int LPI>
__device__ __forceinline__ void finish_list(const uint32_t (&k32)[E], int li, int Dn, int D,
                                            const float* yl, uint64_t* slot, bool valid, int W,
                                            float* ola, uint16_t* olc) {
  const int j0 = li * E;
  const uint32_t imask = (uint32_t)D - 1u;
  wave_lds_sync();
  uint64_t key[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    if (j0 + e < Dn) {
      const int i = (int)(imask - (k32[e] & imask));
      key[e] = exact_key(yl[i], i);
    } else {
      key[e] = 0ull;
    }
  }
  repair_runs<E, LPI>(key, j0, Dn);
  if (__ballot(out_of_order<E, LPI>(key, j0, Dn)) != 0ull) {
    // wave-uniform: every y has been read before the slots are overwritten
    wave_lds_sync();
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (j0 + e < Dn) slot[j0 + e] = key[e];
    wave_lds_sync();
    lds_sort64_desc<E>(slot, j0, Dn);
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (j0 + e < Dn) key[e] = slot[j0 + e];
  }
  if (!valid || j0 >= W) return;
  uint32_t av[E], cv[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const uint64_t kk = key[e];
    const int idx = 0xffff - (int)(((uint32_t)kk & 0x1ffffu) >> 1);
    av[e] = (uint32_t)(kk >> 32);
    cv[e] = (uint32_t)((kk & 1u) ? idx + D : idx);
  }
  if constexpr (E % 8 == 0) {
    if (j0 + E <= Dn) {
      // Dn >= E is a power of two: the lane's 4E + 2E bytes are 16-byte aligned
#pragma unroll
      for (int g4 = 0; g4 < E / 4; ++g4)
        *reinterpret_cast<uint4*>(ola + j0 + 4 * g4) =
            make_uint4(av[4 * g4], av[4 * g4 + 1], av[4 * g4 + 2], av[4 * g4 + 3]);
#pragma unroll
      for (int g8 = 0; g8 < E / 8; ++g8) {
        const uint32_t* c = cv + 8 * g8;
        *reinterpret_cast<uint4*>(olc + j0 + 8 * g8) =
            make_uint4(c[0] | (c[1] << 16), c[2] | (c[3] << 16), c[4] | (c[5] << 16), c[6] | (c[7] << 16));
      }
      return;
    }
  }
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int p = j0 + e;
    if (p < Dn) {
      ola[p] = __uint_as_float(av[e]);
      olc[p] = (uint16_t)cv[e];
    }
  }
}

// Sorts an item's first D 32-bit keys (D <= SP; lane li holds positions li * E .. + E) and
// finishes the list. When at most D / 2 entries are stored and all SP positions are listed
// (D == SP), only the first D / 2 sorted keys are finished, spread over all lanes (E / 2 each,
// through the second half of the LDS slot): the 32-bit order is exact up to runs of equal
// truncated |y|, so when no run crosses position D / 2 those keys are exactly the D / 2 best
// entries. A wavefront where some list has such a run finishes all D keys.
template <int SP, int E, int LPI>
__device__ __forceinline__ void sort_and_store(uint32_t (&k32)[E], int li, int D, const float* yl,
                                               uint64_t* slot, bool valid, int W, float* ola,
                                               uint16_t* olc) {
  const int j0 = li * E;
  sort32_desc<SP, E, LPI>(k32, li, j0, D);
  if constexpr (E >= 2 && E % 2 == 0) {
    if (D == SP && 2 * W <= D) {   // uniform
      constexpr int C = SP / 2;
      constexpr uint32_t imask = (uint32_t)SP - 1u;
      bool cross;   // positions C - 1 and C hold equal truncated |y|
      if constexpr (C % E == 0) {
        // the last key of lane C / E - 1 and the first of the next lane
        const uint32_t nxt0 =
            (uint32_t)__builtin_amdgcn_update_dpp(0, (int)k32[0], 0x130, 0xF, 0xF, false);   // wave_shl:1
        cross = li == C / E - 1 && (k32[E - 1] ^ nxt0) <= imask;
      } else {
        cross = li == C / E && (k32[C % E - 1] ^ k32[C % E]) <= imask;
      }
      if (__ballot(cross) == 0ull) {
        constexpr int E2 = E / 2;
        uint32_t* kl = reinterpret_cast<uint32_t*>(slot) + D;
        wave_lds_sync();
#pragma unroll
        for (int e = 0; e < E; ++e)
          if (j0 + e < C) kl[j0 + e] = k32[e];
        wave_lds_sync();
        uint32_t k2[E2];
#pragma unroll
        for (int e = 0; e < E2; ++e) k2[e] = kl[li * E2 + e];
        finish_list<E2, LPI>(k2, li, C, D, yl, slot, valid, W, ola, olc);
        return;
      }
    }
  }
  finish_list<E, LPI>(k32, li, D, D, yl, slot, valid, W, ola, olc);
}

constexpr int kAnyD = 0;   // D <= P, checked per element
constexpr int kFull = 1;   // D == P: every output is listed, the bounds tests are constants
constexpr int kHalf = 2;   // D == P / 2: the listed outputs are redistributed over all lanes

// VEC: rows of V are 16-byte aligned and d % 4 == 0. MODE: kAnyD, kFull or kHalf. Only the first W
// entries of each sorted list are stored (rounded up to a lane's entries; W = D stores all).
template <int P, bool VEC, int MODE>
__global__ __launch_bounds__(256) void hash_query_kernel(
    const float* __restrict__ V, uint32_t m, int ldv, int d, const uint32_t* __restrict__ sign_mask,
    int LF, int D_arg, int W, float* __restrict__ la, uint16_t* __restrict__ lc) {
  const int D = MODE == kFull ? P : (MODE == kHalf ? P / 2 : D_arg);
  constexpr int E = QLayout<P>::E, LPI = QLayout<P>::LPI, IPW = QLayout<P>::IPW;
  const int lane = threadIdx.x & 63;
  const int li = lane % LPI;
  const uint32_t items = m * (uint32_t)LF;   // < 2^31 (checked by the launcher)
  const uint32_t first = (blockIdx.x * 4u + (threadIdx.x >> 6)) * IPW;
  if (first >= items) return;                // whole wavefront
  const uint32_t item = first + lane / LPI;
  const bool valid = item < items;           // uniform over the item's lanes
  const uint32_t it = valid ? item : 0u;
  const uint32_t q = it / (uint32_t)LF;
  const int tf = (int)(it - q * (uint32_t)LF);
  const int j0 = li * E;

  float v[E];
  const float* row = V + (size_t)q * ldv;
  if constexpr (VEC && E % 4 == 0) {
    // rows are 16-byte aligned: whole float4 groups below d, element loads in the tail group
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
  uint32_t smv[3][E];
  {
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
  // Cross-lane stages use one fused multiply-add: v + w * (+1) in the lower lane of a pair and
  // v - w (= -(w - v), the same rounding) in the upper one, so an upper lane holds the negated
  // value. Partners of a later stage differ only in that stage's lane bit, so they carry the
  // same sign; after a round lane li holds (-1)^popcount(li) times the true values, which the
  // next round's sign flip and the end of the rotation undo with one XOR of the sign bit. (Only
  // the sign of a zero can differ, and neither |y| nor the code rule y >= 0 sees it.)
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
  // ---- order the first D outputs by (|y| desc, i asc)
  // 32-bit keys: |y| bits with the low log2(D) bits replaced by D - 1 - i, sorted descending; the
  // order is exact except inside runs of equal truncated |y|, which hold their indices ascending.
  // Exact values come back from LDS by index, one even and one odd transposition step on the
  // exact 64-bit keys repair runs of two, and a wavefront whose lists are still out of order
  // (a run of three or more) re-sorts the exact keys with the 64-bit network.
  // LDS slot of the item: D floats (the signed outputs by index), reused as D 64-bit keys by the
  // fallback sort
  extern __shared__ uint64_t hq_lds[];
  uint64_t* slot = hq_lds + (size_t)((threadIdx.x >> 6) * IPW + lane / LPI) * D;
  float* yl = reinterpret_cast<float*>(slot);
  const uint32_t imask = (uint32_t)D - 1u;
  uint32_t k32[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int i = j0 + e;
    if (i < D) {
      yl[i] = v[e];
      k32[e] = (__float_as_uint(fabsf(v[e])) & ~imask) | (imask - (uint32_t)i);
    } else {
      k32[e] = 0u;
    }
  }
  float* ola = la + (size_t)it * D;
  uint16_t* olc = lc + (size_t)it * D;
  if constexpr (MODE == kHalf) {
    // D = P / 2: only the lower half of the item's lanes hold listed outputs. Their keys move
    // through the second half of the LDS slot so that every lane sorts E / 2 of them.
    constexpr int E2 = E / 2;
    uint32_t* kl = reinterpret_cast<uint32_t*>(slot) + D;
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (j0 + e < D) kl[j0 + e] = k32[e];
    wave_lds_sync();
    uint32_t k2[E2];
#pragma unroll
    for (int e = 0; e < E2; ++e) k2[e] = kl[li * E2 + e];
    sort_and_store<P / 2, E2, LPI>(k2, li, D, yl, slot, valid, W, ola, olc);
  } else {
    sort_and_store<P, E, LPI>(k32, li, D, yl, slot, valid, W, ola, olc);
  }
}

// One thread per (vector, signature word): scans the sorted lists of the functions the word
// covers and sets bit i of function g when the code at some position is i + D (y_i < 0).
__global__ __launch_bounds__(256) void pack_signs_kernel(const uint16_t* __restrict__ lc, int64_t m,
                                                         int lf, int D, int F, int ldsig,
                                                         uint32_t* __restrict__ out) {
  const int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (x >= m * ldsig) return;
  const int64_t v = x / ldsig;
  const int w = (int)(x - v * ldsig);
  const int64_t b0 = (int64_t)w * 32;
  uint32_t word = 0u;
  if (b0 < (int64_t)F * D) {
    const int g0 = (int)(b0 / D);
    const int g1 = (int)std::min<int64_t>(F - 1, (b0 + 31) / D);
    for (int g = g0; g <= g1; ++g) {
      const uint16_t* row = lc + ((size_t)v * lf + g) * D;
      for (int p = 0; p < D; ++p) {
        const int c = row[p];
        const int64_t b = (int64_t)g * D + (c - D) - b0;   // bit of index c - D, for c >= D
        if (c >= D && b >= 0 && b < 32) word |= 1u << b;
      }
    }
  }
  out[x] = word;
}

}  // namespace

hipError_t launch_pack_signs(const uint16_t* lc, int64_t m, int lf, int D, int F, int ldsig,
                             uint32_t* out, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  const int64_t tot = m * ldsig;
  hipLaunchKernelGGL(pack_signs_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, lc, m,
                     lf, D, F, ldsig, out);
  return hipGetLastError();
}

hipError_t launch_hash_build(const fpp_index* ix, int t0, int Tc, uint32_t* rec_bucket,
                             float* rec_key, hipStream_t s) {
  const bool lng = ix->P > 128;
  if (ix->iProbes <= 1)
    return lng ? launch_hash_build_k1_long(ix, t0, Tc, rec_bucket, rec_key, s)
               : launch_hash_build_k1_short(ix, t0, Tc, rec_bucket, rec_key, s);
  if (ix->iProbes <= 4)
    return lng ? launch_hash_build_k4_long(ix, t0, Tc, rec_bucket, rec_key, s)
               : launch_hash_build_k4_short(ix, t0, Tc, rec_bucket, rec_key, s);
  return lng ? launch_hash_build_k16_long(ix, t0, Tc, rec_bucket, rec_key, s)
             : launch_hash_build_k16_short(ix, t0, Tc, rec_bucket, rec_key, s);
}

hipError_t launch_hash_query(const fpp_index* ix, const float* V, int64_t m, int ldv, float* la,
                             uint16_t* lc, int W, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  if (W < 1 || W > ix->D) return hipErrorInvalidValue;
  const int LF = ix->L * ix->l;
  const int64_t items = m * LF;
  if (items >= (int64_t)1 << 31) return hipErrorInvalidValue;   // callers chunk the queries
  const bool vec = (ix->d % 4 == 0) && (ldv % 4 == 0) && ((uintptr_t)V % 16 == 0);
  const bool full = ix->D == ix->P, half = 2 * ix->D == ix->P;
#define FPP_HQ_LAUNCH(PP, VV, MM)                                                              \
  hipLaunchKernelGGL((hash_query_kernel<PP, VV, MM>), grid, dim3(256), lds, s, V, (uint32_t)m,   \
                     ldv, ix->d, ix->sign_mask, LF, ix->D, W, la, lc)
#define FPP_HQ(PP)                                                                             \
  case PP: {                                                                                   \
    const int64_t waves = (items + QLayout<PP>::IPW - 1) / QLayout<PP>::IPW;                   \
    const dim3 grid((unsigned)((waves + 3) / 4));                                              \
    const size_t lds = (size_t)4 * QLayout<PP>::IPW * ix->D * sizeof(uint64_t);               \
    if (vec && full) {                                                                         \
      FPP_HQ_LAUNCH(PP, true, kFull);                                                          \
    } else if (vec && half && PP >= 32) {                                                      \
      if constexpr (PP >= 32) FPP_HQ_LAUNCH(PP, true, kHalf);                                  \
    } else if (vec) {                                                                          \
      FPP_HQ_LAUNCH(PP, true, kAnyD);                                                          \
    } else {                                                                                   \
      FPP_HQ_LAUNCH(PP, false, kAnyD);                                                         \
    }                                                                                          \
    break;                                                                                     \
  }
  switch (ix->P) {
    FPP_HQ(2) FPP_HQ(4) FPP_HQ(8) FPP_HQ(16) FPP_HQ(32) FPP_HQ(64) FPP_HQ(128) FPP_HQ(256)
    FPP_HQ(512) FPP_HQ(1024) FPP_HQ(2048) FPP_HQ(4096)
    default: return hipErrorInvalidValue;
  }
#undef FPP_HQ
#undef FPP_HQ_LAUNCH
  return hipGetLastError();
}

}  // namespace fpp
