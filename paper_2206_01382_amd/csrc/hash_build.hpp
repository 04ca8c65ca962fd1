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
// (|y| desc, index asc) order together with their codes. For l = 2 the candidate pairs are the
// list positions (i, j) with (i + 1)(j + 1) <= K: any other pair is preceded by at least K
// pairs of its row or column, because float addition is monotone and ties go to the smaller
// position. Records of a point are written at the slot given by the pair's rank.
// ------------------------------------------------------------------------------------------
template <int KMAX>
struct TopList {
  float a[KMAX];
  int32_t idx[KMAX];
  int32_t code[KMAX];
};

template <int KMAX>
__device__ __forceinline__ void toplist_init(TopList<KMAX>& t) {
#pragma unroll
  for (int s = 0; s < KMAX; ++s) {
    t.a[s] = -1.0f;
    t.idx[s] = 0x7fffffff;
    t.code[s] = 0;
  }
}

// Insert (a, i, code) keeping (a desc, i asc). Elements arrive in increasing i within a
// lane, so a strict comparison keeps the earlier index ahead on ties.
template <int KMAX>
__device__ __forceinline__ void toplist_insert(TopList<KMAX>& t, float a, int32_t i, int32_t c) {
  float ca = a;
  int32_t ci = i, cc = c;
#pragma unroll
  for (int s = 0; s < KMAX; ++s) {
    const bool sw = ca > t.a[s];
    const float na = sw ? t.a[s] : ca;
    const int32_t ni = sw ? t.idx[s] : ci;
    const int32_t nc = sw ? t.code[s] : cc;
    t.a[s] = sw ? ca : t.a[s];
    t.idx[s] = sw ? ci : t.idx[s];
    t.code[s] = sw ? cc : t.code[s];
    ca = na;
    ci = ni;
    cc = nc;
  }
}

// (a, i) beats (b, j) in list order.
__device__ __forceinline__ bool list_before(float a, int32_t i, float b, int32_t j) {
  return a > b || (a == b && i < j);
}

// Merge the per-lane lists of a G-lane group into lane-uniform group lists (all lanes of the
// group end with the same list). K rounds of a group argmax; the winner drops its head.
template <int KMAX, int G>
__device__ __forceinline__ void toplist_group_merge(TopList<KMAX>& t) {
  if constexpr (G > 1) {
    TopList<KMAX> out;
    toplist_init(out);
    const int g = threadIdx.x % G;
#pragma unroll
    for (int r = 0; r < KMAX; ++r) {
      float ba = t.a[0];
      int32_t bi = t.idx[0], bc = t.code[0], bl = g;
#pragma unroll
      for (int o = 1; o < G; o <<= 1) {
        const float oa = __shfl_xor(ba, o, G);
        const int32_t oi = __shfl_xor(bi, o, G);
        const int32_t oc = __shfl_xor(bc, o, G);
        const int32_t ol = __shfl_xor(bl, o, G);
        if (list_before(oa, oi, ba, bi)) {
          ba = oa;
          bi = oi;
          bc = oc;
          bl = ol;
        }
      }
      out.a[r] = ba;
      out.idx[r] = bi;
      out.code[r] = bc;
      if (bl == g) {   // the winning lane drops its head
#pragma unroll
        for (int s = 0; s + 1 < KMAX; ++s) {
          t.a[s] = t.a[s + 1];
          t.idx[s] = t.idx[s + 1];
          t.code[s] = t.code[s + 1];
        }
        t.a[KMAX - 1] = -1.0f;
        t.idx[KMAX - 1] = 0x7fffffff;
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
          const float s = A.a[i] + B.a[j];
          int rank = 0;
#pragma unroll
          for (int i2 = 0; i2 < KMAX; ++i2) {
#pragma unroll
            for (int j2 = 0; (i2 + 1) * (j2 + 1) <= KMAX; ++j2) {
              if (i2 < lim && j2 < lim && (i2 + 1) * (j2 + 1) <= K) {
                const float s2 = A.a[i2] + B.a[j2];
                rank += (s2 > s || (s2 == s && (i2 < i || (i2 == i && j2 < j)))) ? 1 : 0;
              }
            }
          }
          if (rank < K) {
            const bool keep = !(A.a[i] < thr) && !(B.a[j] < thr);
            rb[rank] = keep ? (uint32_t)(A.code[i] * (2 * D) + B.code[j]) : kDropped;
            rk[rank] = s;
          }
        }
      }
    }
  } else {
    for (int i = 0; i < lim; ++i) {
      for (int j = 0; j < lim && (i + 1) * (j + 1) <= K; ++j) {
        const float s = A.a[i] + B.a[j];
        int rank = 0;
        for (int i2 = 0; i2 < lim; ++i2) {
          for (int j2 = 0; j2 < lim && (i2 + 1) * (j2 + 1) <= K; ++j2) {
            const float s2 = A.a[i2] + B.a[j2];
            rank += (s2 > s || (s2 == s && (i2 < i || (i2 == i && j2 < j)))) ? 1 : 0;
          }
        }
        if (rank < K) {
          const bool keep = !(A.a[i] < thr) && !(B.a[j] < thr);
          rb[rank] = keep ? (uint32_t)(A.code[i] * (2 * D) + B.code[j]) : kDropped;
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
        if (i < D) toplist_insert(tl, fabsf(v[e]), i, v[e] >= 0.0f ? i : i + D);
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
          rb[s] = !(list0.a[s] < thr) ? (uint32_t)list0.code[s] : kDropped;
          rk[s] = list0.a[s];
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
