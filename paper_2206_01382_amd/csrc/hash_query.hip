// Query-side cross-polytope hashing on gfx950 (Section 2.2 Eq. 1; Section 3.4 structured
// spinners), and the dispatch of the build-side kernels.
//
// Each hash function rotates the zero-padded vector with three rounds of "flip signs, then
// unnormalised Walsh-Hadamard transform" (stage h = 1, 2, ..., P/2; the lower element of a pair
// becomes a + b, the upper a - b) and reads the first D outputs y_i. Sign flips are XORs of the
// sign bit; there are no multiplications, so the float32 results are those of that order.
#include "fpp_internal.hpp"

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
// Query side. One wavefront per (vector, function), everything in registers: lane x holds the
// elements j = e * 64 + x (e < E = P / 64; for P < 64 lanes x < P hold one element). Butterfly
// stages h < 64 pair lane x with lane x ^ h (the lower lane adds, the upper subtracts), stages
// h >= 64 pair register e with e ^ (h / 64) inside the lane, in the order h = 1, 2, ..., P/2.
// The D keys (|y_i| bits << 32 | (0xffff - i) << 1 | sign) are then bitonic-sorted descending in
// the same layout, which orders the list by (|y| desc, i asc) and carries the code bit.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
  const uint32_t lo = __shfl_xor((uint32_t)v, m), hi = __shfl_xor((uint32_t)(v >> 32), m);
  return ((uint64_t)hi << 32) | lo;
}

template <int P>
__global__ __launch_bounds__(256) void hash_query_kernel(
    const float* __restrict__ V, int64_t m, int ldv, int d, const uint32_t* __restrict__ sign_mask,
    int LF, int D, float* __restrict__ la, uint16_t* __restrict__ lc) {
  constexpr int E = P >= 64 ? P / 64 : 1;
  constexpr int XS = P >= 64 ? 64 : P;   // lanes that hold elements
  const int lane = threadIdx.x & 63;
  const int64_t item = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (item >= m * LF) return;   // whole wavefront
  const int64_t q = item / LF;
  const int tf = (int)(item - q * LF);
  const bool on = lane < XS;

  float v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int j = e * 64 + lane;
    v[e] = (on && j < d) ? V[q * ldv + j] : 0.0f;
  }
  const uint32_t* sm = sign_mask + (size_t)tf * 3 * P;
  for (int r = 0; r < 3; ++r) {
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (on) v[e] = flip(v[e], sm[r * P + e * 64 + lane]);
#pragma unroll
    for (int h = 1; h < XS; h <<= 1) {
      const bool upper = (lane & h) != 0;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const float w = __shfl_xor(v[e], h);
        v[e] = upper ? w - v[e] : v[e] + w;
      }
    }
#pragma unroll
    for (int hh = 1; hh < E; hh <<= 1) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        if ((e & hh) == 0) {
          const float a = v[e], b = v[e + hh];
          v[e] = a + b;
          v[e + hh] = a - b;
        }
      }
    }
  }
  uint64_t key[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int i = e * 64 + lane;
    const uint32_t neg = v[e] >= 0.0f ? 0u : 1u;
    key[e] = (on && i < D) ? ((uint64_t)__float_as_uint(fabsf(v[e])) << 32) |
                                 ((uint32_t)(0xffff - i) << 1) | neg
                           : 0ull;
  }
  // bitonic sort (descending) of the first D keys, D a power of two
  for (int k = 2; k <= D; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      if (j < 64) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const int i = e * 64 + lane;
          const uint64_t o = shfl_xor_u64(key[e], j);
          const bool lower = (i & j) == 0, desc = (i & k) == 0;
          const uint64_t mx = key[e] > o ? key[e] : o, mn = key[e] > o ? o : key[e];
          key[e] = (lower == desc) ? mx : mn;
        }
      } else {
        const int jj = j >> 6;
#pragma unroll
        for (int e = 0; e < E; ++e) {
          if ((e & jj) == 0 && (e | jj) < E) {
            const int i = e * 64 + lane;
            const bool desc = (i & k) == 0;
            const uint64_t a = key[e], b = key[e | jj];
            if (desc ? (a < b) : (a > b)) {
              key[e] = b;
              key[e | jj] = a;
            }
          }
        }
      }
    }
  }
  float* ola = la + (size_t)item * D;
  uint16_t* olc = lc + (size_t)item * D;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int p = e * 64 + lane;
    if (on && p < D) {
      const uint64_t kk = key[e];
      const int idx = 0xffff - (int)(((uint32_t)kk & 0x1ffffu) >> 1);
      ola[p] = __uint_as_float((uint32_t)(kk >> 32));
      olc[p] = (uint16_t)((kk & 1u) ? idx + D : idx);
    }
  }
}

}  // namespace

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
                             uint16_t* lc, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  const int LF = ix->L * ix->l;
  const int64_t items = m * LF;
  const dim3 grid((unsigned)((items + 3) / 4)), block(256);
#define FPP_HQ(PP)                                                                             \
  case PP:                                                                                     \
    hipLaunchKernelGGL(hash_query_kernel<PP>, grid, block, 0, s, V, m, ldv, ix->d, ix->sign_mask, \
                       LF, ix->D, la, lc);                                                     \
    break;
  switch (ix->P) {
    FPP_HQ(2) FPP_HQ(4) FPP_HQ(8) FPP_HQ(16) FPP_HQ(32) FPP_HQ(64) FPP_HQ(128) FPP_HQ(256)
    FPP_HQ(512) FPP_HQ(1024) FPP_HQ(2048) FPP_HQ(4096)
    default: return hipErrorInvalidValue;
  }
#undef FPP_HQ
  return hipGetLastError();
}

}  // namespace fpp
