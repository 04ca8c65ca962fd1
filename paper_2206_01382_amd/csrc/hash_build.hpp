// Build-side cross-polytope hashing on gfx950 (Section 2.2 Eq. 1; Section 3.4 structured
// spinners). Included by the hash_build_k*.hip units, one per (bucket count, length range).
//
// Each hash function rotates the zero-padded vector with three rounds of
// "flip signs, then unnormalised Walsh-Hadamard transform" and reads the first D
// outputs y_i. The code is i when y_i >= 0 and i + D otherwise, for the index i of
// the largest |y_i| (ties: smallest i).
//
// Bit-exactness: every transform output is produced by the same float32 expression
// tree as the stated butterfly order (stage h = 1, 2, ..., P/2; the lower element of
// a pair becomes a + b, the upper a - b). Sign flips are XORs of the sign bit. There
// are no multiplications, so no contraction can change a result.
#pragma once
#include "fpp_internal.hpp"

namespace fpp {
namespace detail {

__device__ __forceinline__ float flip(float v, uint32_t mask) {
  return __uint_as_float(__float_as_uint(v) ^ mask);
}

// ------------------------------------------------------------------------------------------
// Build side. A group of G lanes owns one point; lane g of the group holds the E = P / G
// contiguous elements [g*E, (g+1)*E) in registers. Butterfly stages with h < E stay in the
// lane; stages with h >= E exchange with lane g ^ (h / E).
//
// After the rotation of one function the group keeps the KMAX best (|y|, index) entries in
// (|y| desc, index asc) order, as 64-bit list keys that also carry the codes. For l = 2 the
// candidate pairs are the list positions (i, j) with (i + 1)(j + 1) <= K: any other pair is
// preceded by at least K pairs of its row or column, because float addition is monotone and ties
// go to the smaller position. Records of a point are written at the slot given by the pair's
// rank.
// ------------------------------------------------------------------------------------------
template <int KMAX>
struct TopList {
  uint64_t k[KMAX];   // list keys, best first; 0 marks an empty slot
};

// List key of output i with value y: |y| bits << 32 | (0xffff - i) << 1 | sign. Keys compare as
// integers in list order (|y| desc, i asc) with no ties, and carry the code (i, or i + D when
// y < 0). Every key of a real output is > 0.
__device__ __forceinline__ uint64_t list_key(float y, int32_t i) {
  return ((uint64_t)__float_as_uint(fabsf(y)) << 32) | ((uint32_t)(0xffff - i) << 1) |
         (y >= 0.0f ? 0u : 1u);
}
__device__ __forceinline__ float key_abs(uint64_t k) { return __uint_as_float((uint32_t)(k >> 32)); }
__device__ __forceinline__ int32_t key_code(uint64_t k, int D) {
  const int32_t i = 0xffff - (int32_t)(((uint32_t)k & 0x1ffffu) >> 1);
  return (k & 1u) ? i + D : i;
}

template <int KMAX>
__device__ __forceinline__ void toplist_init(TopList<KMAX>& t) {
#pragma unroll
  for (int s = 0; s < KMAX; ++s) t.k[s] = 0ull;
}

// Insert a key, keeping the list in descending key order (one compare-exchange per slot).
template <int KMAX>
__device__ __forceinline__ void toplist_insert(TopList<KMAX>& t, uint64_t key) {
  uint64_t c = key;
#pragma unroll
  for (int s = 0; s < KMAX; ++s) {
    const bool sw = c > t.k[s];
    const uint64_t lo = sw ? t.k[s] : c;
    t.k[s] = sw ? c : t.k[s];
    c = lo;
  }
}

// Merge the per-lane lists of a G-lane group into lane-uniform group lists (all lanes of the
// group end with the same list). K rounds of a group argmax (keys are distinct); the winner drops
// its head.
template <int KMAX, int G>
__device__ __forceinline__ void toplist_group_merge(TopList<KMAX>& t) {
  if constexpr (G > 1) {
    TopList<KMAX> out;
#pragma unroll
    for (int r = 0; r < KMAX; ++r) {
      uint64_t best = t.k[0];
#pragma unroll
      for (int o = 1; o < G; o <<= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)best, o, G), hi = __shfl_xor((uint32_t)(best >> 32), o, G);
        const uint64_t other = ((uint64_t)hi << 32) | lo;
        best = other > best ? other : best;
      }
      out.k[r] = best;
      if (best != 0ull && t.k[0] == best) {   // the winning lane drops its head
#pragma unroll
        for (int s = 0; s + 1 < KMAX; ++s) t.k[s] = t.k[s + 1];
        t.k[KMAX - 1] = 0ull;
      }
    }
    t = out;
  }
}

// l = 2: rank every candidate pair (i, j) with (i+1)(j+1) <= K among the candidates by
// (score desc, i asc, j asc) and write the K best at the slot given by their rank.
// thr >= 0 (global-threshold filter): a pair whose |y1| or |y2| is below thr is written with the
// bucket kDropped, which the table build skips.
template <int KMAX>
__device__ __forceinline__ void select_pairs(const TopList<KMAX>& A, const TopList<KMAX>& B, int K,
                                             int D, float thr, uint32_t* rb, float* rk) {
  const int lim = K < D ? K : D;
  constexpr bool kUnroll = KMAX <= 8;
  if constexpr (kUnroll) {
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
#pragma unroll
      for (int j = 0; (i + 1) * (j + 1) <= KMAX; ++j) {
        if (i < lim && j < lim && (i + 1) * (j + 1) <= K) {
          const float s = key_abs(A.k[i]) + key_abs(B.k[j]);
          int rank = 0;
#pragma unroll
          for (int i2 = 0; i2 < KMAX; ++i2) {
#pragma unroll
            for (int j2 = 0; (i2 + 1) * (j2 + 1) <= KMAX; ++j2) {
              if (i2 < lim && j2 < lim && (i2 + 1) * (j2 + 1) <= K) {
                const float s2 = key_abs(A.k[i2]) + key_abs(B.k[j2]);
                rank += (s2 > s || (s2 == s && (i2 < i || (i2 == i && j2 < j)))) ? 1 : 0;
              }
            }
          }
          if (rank < K) {
            const bool keep = !(key_abs(A.k[i]) < thr) && !(key_abs(B.k[j]) < thr);
            rb[rank] = keep ? (uint32_t)(key_code(A.k[i], D) * (2 * D) + key_code(B.k[j], D)) : kDropped;
            rk[rank] = s;
          }
        }
      }
    }
  } else {
    for (int i = 0; i < lim; ++i) {
      for (int j = 0; j < lim && (i + 1) * (j + 1) <= K; ++j) {
        const float s = key_abs(A.k[i]) + key_abs(B.k[j]);
        int rank = 0;
        for (int i2 = 0; i2 < lim; ++i2) {
          for (int j2 = 0; j2 < lim && (i2 + 1) * (j2 + 1) <= K; ++j2) {
            const float s2 = key_abs(A.k[i2]) + key_abs(B.k[j2]);
            rank += (s2 > s || (s2 == s && (i2 < i || (i2 == i && j2 < j)))) ? 1 : 0;
          }
        }
        if (rank < K) {
          const bool keep = !(key_abs(A.k[i]) < thr) && !(key_abs(B.k[j]) < thr);
          rb[rank] = keep ? (uint32_t)(key_code(A.k[i], D) * (2 * D) + key_code(B.k[j], D)) : kDropped;
          rk[rank] = s;
        }
      }
    }
  }
}

template <int P, int G, int KMAX>
__global__ __launch_bounds__(64) void hash_build_kernel(
    const float* __restrict__ X, int64_t n, int d, int ldx, const uint32_t* __restrict__ sign_mask,
    int t0, int Tc, int l, int D, int K, float thr, uint32_t* __restrict__ rec_bucket,
    float* __restrict__ rec_key) {
  constexpr int E = P / G;          // elements per lane
  constexpr int PPB = 64 / G;       // points per block
  extern __shared__ float xs[];     // [d][PPB + 1]
  const int lane = threadIdx.x;
  const int pl = lane / G;
  const int g = lane % G;
  const int64_t p0 = (int64_t)blockIdx.x * PPB;
  const int64_t p = p0 + pl;

  // Stage the block's points in LDS, transposed (element-major) so lanes read consecutive words.
  for (int i = lane; i < PPB * d; i += 64) {
    const int r = i / d, e = i - r * d;
    const int64_t pr = p0 + r;
    xs[e * (PPB + 1) + r] = pr < n ? X[pr * ldx + e] : 0.0f;
  }
  __syncthreads();
  if (p >= n) return;   // no barrier follows

  const int64_t nK = n * (int64_t)K;
  for (int tt = 0; tt < Tc; ++tt) {
    const int t = t0 + tt;
    TopList<KMAX> list0, list1;
    for (int f = 0; f < l; ++f) {
      float v[E];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int j = g * E + e;
        v[e] = j < d ? xs[j * (PPB + 1) + pl] : 0.0f;
      }
      const uint32_t* sm = sign_mask + (size_t)((t * l + f) * 3) * P + g * E;
      for (int r = 0; r < 3; ++r) {
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = flip(v[e], sm[r * P + e]);
        // in-lane stages
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
        // cross-lane stages
#pragma unroll
        for (int hl = 1; hl < G; hl <<= 1) {
          const bool lower = (g & hl) == 0;
#pragma unroll
          for (int e = 0; e < E; ++e) {
            const float w = __shfl_xor(v[e], hl, G);
            v[e] = lower ? v[e] + w : w - v[e];
          }
        }
      }
      TopList<KMAX> tl;
      toplist_init(tl);
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int i = g * E + e;
        if (i < D) toplist_insert(tl, list_key(v[e], i));
      }
      toplist_group_merge<KMAX, G>(tl);
      if (f == 0) list0 = tl; else list1 = tl;
    }
    if (g != 0) continue;
    uint32_t* rb = rec_bucket + (size_t)tt * nK + p * K;
    float* rk = rec_key + (size_t)tt * nK + p * K;
    if (l == 1) {
#pragma unroll
      for (int s = 0; s < KMAX; ++s)
        if (s < K) {
          rb[s] = !(key_abs(list0.k[s]) < thr) ? (uint32_t)key_code(list0.k[s], D) : kDropped;
          rk[s] = key_abs(list0.k[s]);
        }
    } else {
      select_pairs<KMAX>(list0, list1, K, D, thr, rb, rk);
    }
  }
}

template <int P, int G, int KMAX>
inline hipError_t launch_build_p(const fpp_index* ix, int t0, int Tc, uint32_t* rb, float* rk,
                          hipStream_t s) {
  constexpr int PPB = 64 / G;
  const int64_t blocks = (ix->n + PPB - 1) / PPB;
  const size_t lds = (size_t)ix->d * (PPB + 1) * sizeof(float);
  hipLaunchKernelGGL((hash_build_kernel<P, G, KMAX>), dim3((unsigned)blocks), dim3(64), lds, s,
                     ix->Xh ? ix->Xh : ix->X, ix->n, ix->d, ix->ldx, ix->sign_mask, t0, Tc, ix->l,
                     ix->D, ix->iProbes, ix->filter == FPP_FILTER_THRESHOLD ? ix->thr : -1.0f, rb, rk);
  return hipGetLastError();
}

// Elements held per lane: 128 for short top lists; 32 when 16 buckets per point are kept, so
// that the unrolled insertion stays small. A point spans G = P / E lanes.
template <int KMAX>
constexpr int lane_elems() { return KMAX >= 16 ? 32 : 128; }
template <int P, int KMAX>
constexpr int group_lanes() {
  return P <= lane_elems<KMAX>() ? 1 : (P / lane_elems<KMAX>() > 64 ? 64 : P / lane_elems<KMAX>());
}

#define FPP_BUILD_CASE(PP) \
  case PP: return launch_build_p<PP, group_lanes<PP, KMAX>(), KMAX>(ix, t0, Tc, rb, rk, s);

template <int KMAX>
inline hipError_t launch_build_k_short(const fpp_index* ix, int t0, int Tc, uint32_t* rb, float* rk,
                                       hipStream_t s) {
  switch (ix->P) {
    FPP_BUILD_CASE(2)
    FPP_BUILD_CASE(4)
    FPP_BUILD_CASE(8)
    FPP_BUILD_CASE(16)
    FPP_BUILD_CASE(32)
    FPP_BUILD_CASE(64)
    FPP_BUILD_CASE(128)
    default: return hipErrorInvalidValue;
  }
}

template <int KMAX>
inline hipError_t launch_build_k_long(const fpp_index* ix, int t0, int Tc, uint32_t* rb, float* rk,
                                      hipStream_t s) {
  switch (ix->P) {
    FPP_BUILD_CASE(256)
    FPP_BUILD_CASE(512)
    FPP_BUILD_CASE(1024)
    FPP_BUILD_CASE(2048)
    FPP_BUILD_CASE(4096)
    default: return hipErrorInvalidValue;
  }
}
#undef FPP_BUILD_CASE

}  // namespace detail
}  // namespace fpp
