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
#include "rotation.hpp"
#include "wave_sort.hpp"

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

// Exact 64-bit list key: |y| bits << 32 | (0xffff - i) << 1 | sign; descending order of keys is
// (|y| desc, i asc), and the low bit carries the code (i or i + D).
__device__ __forceinline__ uint64_t exact_key(float y, int i) {
  const uint32_t neg = y >= 0.0f ? 0u : 1u;
  return ((uint64_t)__float_as_uint(fabsf(y)) << 32) | ((uint32_t)(0xffff - i) << 1) | neg;
}

__device__ __forceinline__ void ce_desc(uint64_t& a, uint64_t& b) {
  const bool sw = a < b;
  const uint64_t x = sw ? b : a, y = sw ? a : b;
  a = x;
  b = y;
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
// The wavefront's items first .. first + IPW - 1 (of m * LF).
template <int P, bool VEC, int MODE>
__device__ __forceinline__ void hash_wave(
    uint32_t first, const float* __restrict__ V, uint32_t m, int ldv, int d,
    const uint32_t* __restrict__ sign_mask, int LF, int D_arg, int W, float* __restrict__ la,
    uint16_t* __restrict__ lc) {
  extern __shared__ uint64_t hq_lds[];
  const int D = MODE == kFull ? P : (MODE == kHalf ? P / 2 : D_arg);
  constexpr int E = QLayout<P>::E, LPI = QLayout<P>::LPI, IPW = QLayout<P>::IPW;
  const int lane = threadIdx.x & 63;
  const int li = lane % LPI;
  const uint32_t items = m * (uint32_t)LF;   // < 2^31 (checked by the launcher)
  const uint32_t item = first + lane / LPI;
  const bool valid = item < items;           // uniform over the item's lanes
  const uint32_t it = valid ? item : 0u;
  const uint32_t q = it / (uint32_t)LF;
  const int tf = (int)(it - q * (uint32_t)LF);
  const int j0 = li * E;

  float v[E];
  load_elems<E, VEC>(V + (size_t)q * ldv, d, j0, v);
  uint32_t smv[3][E];
  load_sign_masks<P, E>(sign_mask, tf, j0, smv);
  rotate_item<P>(v, smv, li);
  // ---- order the first D outputs by (|y| desc, i asc)
  // 32-bit keys: |y| bits with the low log2(D) bits replaced by D - 1 - i, sorted descending; the
  // order is exact except inside runs of equal truncated |y|, which hold their indices ascending.
  // Exact values come back from LDS by index, one even and one odd transposition step on the
  // exact 64-bit keys repair runs of two, and a wavefront whose lists are still out of order
  // (a run of three or more) re-sorts the exact keys with the 64-bit network.
  // LDS slot of the item: D floats (the signed outputs by index), reused as D 64-bit keys by the
  // fallback sort
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

// Wavefront w of the grid takes items w * IPW .. w * IPW + IPW - 1. PICK (the rare vectors that the
// fused kernel leaves, marked by skip[q] < 0): wavefront w reads the marks of vectors
// 64 w .. 64 w + 63 at once and computes the lists of the marked ones (and of whatever vectors
// share their first or last group of IPW items).
template <int P, bool VEC, int MODE, bool PICK>
__global__ __launch_bounds__(256) void hash_query_kernel(
    const float* __restrict__ V, uint32_t m, int ldv, int d, const uint32_t* __restrict__ sign_mask,
    int LF, int D_arg, int W, float* __restrict__ la, uint16_t* __restrict__ lc,
    const int32_t* __restrict__ skip) {
  constexpr int IPW = QLayout<P>::IPW;
  const uint32_t wv = blockIdx.x * 4u + (threadIdx.x >> 6);
  if constexpr (!PICK) {
    const uint32_t first = wv * IPW;
    if (first < m * (uint32_t)LF)
      hash_wave<P, VEC, MODE>(first, V, m, ldv, d, sign_mask, LF, D_arg, W, la, lc);
  } else {
    const uint32_t q0 = wv * 64u;
    if (q0 >= m) return;   // whole wavefront
    const uint32_t qq = q0 + (threadIdx.x & 63);
    uint64_t marked = __ballot(qq < m && skip[qq] < 0);
    while (marked) {
      const uint32_t q = q0 + (uint32_t)__builtin_ctzll(marked);
      marked &= marked - 1ull;
      for (uint32_t first = q * (uint32_t)LF; first < (q + 1u) * (uint32_t)LF; first += IPW) {
        hash_wave<P, VEC, MODE>(first, V, m, ldv, d, sign_mask, LF, D_arg, W, la, lc);
        wave_lds_sync();   // the next round reuses the wavefront's LDS slots
      }
    }
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
                             uint16_t* lc, int W, hipStream_t s, const int32_t* skip) {
  if (m <= 0) return hipSuccess;
  if (W < 1 || W > ix->D) return hipErrorInvalidValue;
  const int LF = ix->L * ix->l;
  const int64_t items = m * LF;
  if (items >= (int64_t)1 << 31) return hipErrorInvalidValue;   // callers chunk the queries
  const bool vec = (ix->d % 4 == 0) && (ldv % 4 == 0) && ((uintptr_t)V % 16 == 0);
  const bool full = ix->D == ix->P, half = 2 * ix->D == ix->P;
#define FPP_HQ_LAUNCH(PP, VV, MM)                                                              \
  do {                                                                                         \
    if (skip)                                                                                  \
      hipLaunchKernelGGL((hash_query_kernel<PP, VV, MM, true>), grid, dim3(256), lds, s, V,     \
                         (uint32_t)m, ldv, ix->d, ix->sign_mask, LF, ix->D, W, la, lc, skip);    \
    else                                                                                       \
      hipLaunchKernelGGL((hash_query_kernel<PP, VV, MM, false>), grid, dim3(256), lds, s, V,    \
                         (uint32_t)m, ldv, ix->d, ix->sign_mask, LF, ix->D, W, la, lc, skip);    \
  } while (0)
#define FPP_HQ(PP)                                                                             \
  case PP: {                                                                                   \
    const int64_t waves = (items + QLayout<PP>::IPW - 1) / QLayout<PP>::IPW;                   \
    const dim3 grid((unsigned)(skip ? (m + 255) / 256 : (waves + 3) / 4));                     \
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
