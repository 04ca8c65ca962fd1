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
// Query side. One wavefront per (vector, function): the rotation runs in LDS with the same
// butterfly order, then the D (|y|, i) keys are bitonic-sorted in LDS, descending by
// (|y| bits << 32 | ~i), which is (|y| desc, i asc).
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(64) void hash_query_kernel(
    const float* __restrict__ V, int64_t m, int ldv, int d, const uint32_t* __restrict__ sign_mask,
    int LF, int P, int D, int Dp2, float* __restrict__ la, uint16_t* __restrict__ lc) {
  extern __shared__ unsigned char smem[];
  float* v = reinterpret_cast<float*>(smem);                        // [P]
  uint64_t* key = reinterpret_cast<uint64_t*>(smem + (size_t)P * 4);   // [Dp2], 8-byte aligned (P >= 2)
  const int lane = threadIdx.x;
  const int64_t item = blockIdx.x;   // vector * LF + function
  const int64_t q = item / LF;
  const int tf = (int)(item - q * LF);
  if (q >= m) return;   // uniform for the block

  for (int j = lane; j < P; j += 64) v[j] = j < d ? V[q * ldv + j] : 0.0f;
  __syncthreads();
  const uint32_t* sm = sign_mask + (size_t)tf * 3 * P;
  for (int r = 0; r < 3; ++r) {
    for (int j = lane; j < P; j += 64) v[j] = flip(v[j], sm[r * P + j]);
    __syncthreads();
    for (int h = 1; h < P; h <<= 1) {
      for (int b = lane; b < P / 2; b += 64) {
        const int j = (b / h) * 2 * h + (b % h);
        const float a = v[j], c = v[j + h];
        v[j] = a + c;
        v[j + h] = a - c;
      }
      __syncthreads();
    }
  }
  for (int i = lane; i < Dp2; i += 64)
    key[i] = i < D ? ((uint64_t)__float_as_uint(fabsf(v[i])) << 32) | (uint32_t)(0xffffffffu - i)
                   : 0ull;
  __syncthreads();
  for (int k = 2; k <= Dp2; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = lane; i < Dp2; i += 64) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const uint64_t a = key[i], b = key[ixj];
          const bool desc = (i & k) == 0;
          if (desc ? (a < b) : (a > b)) {
            key[i] = b;
            key[ixj] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  float* ola = la + (size_t)item * D;
  uint16_t* olc = lc + (size_t)item * D;
  for (int i = lane; i < D; i += 64) {
    const uint64_t kk = key[i];
    const int idx = (int)(0xffffffffu - (uint32_t)kk);
    ola[i] = __uint_as_float((uint32_t)(kk >> 32));
    olc[i] = (uint16_t)(v[idx] >= 0.0f ? idx : idx + D);
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
  int Dp2 = 1;
  while (Dp2 < ix->D) Dp2 <<= 1;
  const int LF = ix->L * ix->l;
  const size_t lds = (size_t)ix->P * 4 + (size_t)Dp2 * 8;
  const int64_t items = m * LF;
  hipLaunchKernelGGL(hash_query_kernel, dim3((unsigned)items), dim3(64), lds, s, V, m, ldv, ix->d,
                     ix->sign_mask, LF, ix->P, ix->D, Dp2, la, lc);
  return hipGetLastError();
}

}  // namespace fpp
