// Register sorting networks over the lanes of a wavefront (descending, 32-bit keys). A group of
// LPI lanes holds P = LPI * E keys, lane li positions li * E .. li * E + E - 1; compare-exchanges
// inside a lane are register pairs, across lanes the partner comes from a DPP / row-swap lane
// exchange (lanes.hpp). Used for the sorted projection lists of the query hash (a group per hash
// function) and, with the whole wavefront as one group, for short selections.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lanes.hpp"

namespace fpp {

__device__ __forceinline__ void ce_desc(uint32_t& a, uint32_t& b) {
  const uint32_t hi = a > b ? a : b, lo = a > b ? b : a;
  a = hi;
  b = lo;
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

}  // namespace fpp
