// Query-side cross-polytope hashing on gfx950 (Section 2.2 Eq. 1; Section 3.4 structured
// spinners), and the dispatch of the build-side kernels.
//
// Each hash function rotates the zero-padded vector with three rounds of "flip signs, then
// unnormalised Walsh-Hadamard transform" (stage h = 1, 2, ..., P/2; the lower element of a pair
// becomes a + b, the upper a - b) and reads the first D outputs y_i. Sign flips are XORs of the
// sign bit; there are no multiplications, so the float32 results are those of that order.
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
  static constexpr int E = P < 8 ? P : (P / 64 > 8 ? P / 64 : 8);   // elements per lane
  static constexpr int LPI = P / E;                                 // lanes per item
  static constexpr int IPW = 64 / LPI;                              // items per wavefront
};

template <int P>
__global__ __launch_bounds__(256) void hash_query_kernel(
    const float* __restrict__ V, int64_t m, int ldv, int d, const uint32_t* __restrict__ sign_mask,
    int LF, int D, float* __restrict__ la, uint16_t* __restrict__ lc) {
  constexpr int E = QLayout<P>::E, LPI = QLayout<P>::LPI, IPW = QLayout<P>::IPW;
  const int lane = threadIdx.x & 63;
  const int li = lane % LPI;
  const int64_t items = m * LF;
  const int64_t item = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * IPW + lane / LPI;
  if (((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * IPW >= items) return;   // whole wavefront
  const bool valid = item < items;   // uniform over the item's lanes
  const int64_t it = valid ? item : 0;
  const int64_t q = it / LF;
  const int tf = (int)(it - q * LF);
  const int j0 = li * E;

  float v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = (j0 + e < d) ? V[q * ldv + j0 + e] : 0.0f;
  const uint32_t* sm = sign_mask + (size_t)tf * 3 * P + j0;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = flip(v[e], sm[r * P + e]);
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
      // the upper lane of a pair computes w - v as w + (-v): the same rounded result
      const uint32_t neg = (li & hl) ? 0x80000000u : 0u;
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = xor_lanes_n(v[e], hl) + flip(v[e], neg);
    }
  }
  uint64_t key[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int i = j0 + e;
    const uint32_t neg = v[e] >= 0.0f ? 0u : 1u;
    key[e] = i < D ? ((uint64_t)__float_as_uint(fabsf(v[e])) << 32) | ((uint32_t)(0xffff - i) << 1) | neg
                   : 0ull;
  }
  // bitonic sort (descending) of the first D keys (D a power of two <= P)
#pragma unroll
  for (int k = 2; k <= P; k <<= 1) {
    if (k <= D) {
      // direction of element j0 + e in stage k: compile-time for k < E, lane-uniform for k >= E
      const bool desc_lane = (j0 & k) == 0;
#pragma unroll
      for (int j = k >> 1; j > 0; j >>= 1) {
        if (j < E) {
#pragma unroll
          for (int e = 0; e < E; ++e) {
            if ((e & j) == 0) {
              const bool desc = k < E ? ((e & k) == 0) : desc_lane;
              const uint64_t a = key[e], b = key[e | j];
              const bool sw = desc ? (a < b) : (b < a);
              key[e] = sw ? b : a;
              key[e | j] = sw ? a : b;
            }
          }
        } else {
          const bool keep_max = ((li & (j / E)) == 0) == desc_lane;
#pragma unroll
          for (int e = 0; e < E; ++e) {
            const uint64_t o = xor_lanes_n(key[e], j / E);
            key[e] = ((key[e] > o) == keep_max) ? key[e] : o;
          }
        }
      }
    }
  }
  if (!valid) return;
  float* ola = la + (size_t)item * D;
  uint16_t* olc = lc + (size_t)item * D;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int p = j0 + e;
    if (p < D) {
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
#define FPP_HQ(PP)                                                                             \
  case PP: {                                                                                   \
    const int64_t waves = (items + QLayout<PP>::IPW - 1) / QLayout<PP>::IPW;                   \
    hipLaunchKernelGGL(hash_query_kernel<PP>, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, \
                       V, m, ldv, ix->d, ix->sign_mask, LF, ix->D, la, lc);                    \
    break;                                                                                     \
  }
  switch (ix->P) {
    FPP_HQ(2) FPP_HQ(4) FPP_HQ(8) FPP_HQ(16) FPP_HQ(32) FPP_HQ(64) FPP_HQ(128) FPP_HQ(256)
    FPP_HQ(512) FPP_HQ(1024) FPP_HQ(2048) FPP_HQ(4096)
    default: return hipErrorInvalidValue;
  }
#undef FPP_HQ
  return hipGetLastError();
}

}  // namespace fpp
