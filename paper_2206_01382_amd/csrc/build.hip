// Table build on gfx950 (Algorithm 1, the per-bucket filter; Section 3.4 "alpha-fraction").
//
// For a chunk of Tc tables whose records (bucket, key) were produced by the hash kernel
// (record r of a table belongs to point r / iProbes):
//   1. count    records per bucket (atomics into a [Tc][NB] histogram);
//   2. scan     per table: bucket starts of the grouped records, keep(B) and the CSR offsets of
//               the kept ids (relative to the table), table size and largest kept bucket;
//   3. bases    absolute start of each table in the shared ids array (running over chunks);
//   4. scatter  records grouped by bucket (arbitrary order inside a bucket);
//   5. order    every bucket is ordered by (key desc, id asc) and its first keep(B) ids are
//               written at the bucket's CSR offset: buckets of <= 64 records by one wavefront
//               (each lane counts the records that precede its own), larger ones (listed by the
//               scan) by a workgroup that bitonic-sorts them in LDS; the result does not depend on
//               the scatter order;
//   6. absolute CSR offsets += table start.
// keep(B) = ceil(A * B / (iProbes * 10^6)) (or floor) with A = alpha in millionths, at least
// min(B, kappa) under limit scaling; under the global-threshold filter the hash kernel has already
// dropped the records below the threshold and every bucket keeps all of its records.
#include "fpp_internal.hpp"

namespace fpp {
namespace {

constexpr int kScanThreads = 1024;

// Records a bucket of B keeps: all of them under the global-threshold filter (A < 0), else the
// alpha fraction keep(B), raised to min(B, kappa) by limit scaling (Section 3.4, heuristic 2).
__device__ __forceinline__ uint32_t keep_of(uint32_t B, int64_t A, int K, int rounding, int kappa) {
  if (A < 0) return B;
  const uint64_t den = (uint64_t)K * 1000000ull;
  const uint64_t num = (uint64_t)B * (uint64_t)A;
  const uint32_t kp = (uint32_t)(rounding == 0 ? (num + den - 1) / den : num / den);
  const uint32_t lim = B < (uint32_t)kappa ? B : (uint32_t)kappa;
  return kp > lim ? kp : lim;
}

__global__ __launch_bounds__(256) void count_kernel(const uint32_t* __restrict__ rec_bucket,
                                                    int64_t nK, int64_t NB,
                                                    uint32_t* __restrict__ cnt) {
  const int tt = blockIdx.y;
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= nK) return;
  const uint32_t b = rec_bucket[(size_t)tt * nK + r];
  if (b == kDropped) return;
  atomicAdd(&cnt[(size_t)tt * NB + b], 1u);
}

// Exclusive scan of two u32 sequences over the block (one value pair per thread).
__device__ void block_scan2(uint32_t& a, uint32_t& b, uint32_t& tot_a, uint32_t& tot_b,
                            uint32_t* sa, uint32_t* sb) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int nw = blockDim.x >> 6;
  uint32_t ia = a, ib = b;   // inclusive within the wave
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t ta = __shfl_up(ia, o), tb = __shfl_up(ib, o);
    if (lane >= o) {
      ia += ta;
      ib += tb;
    }
  }
  if (lane == 63) {
    sa[w] = ia;
    sb[w] = ib;
  }
  __syncthreads();
  if (tid == 0) {
    uint32_t ra = 0, rb = 0;
    for (int i = 0; i < nw; ++i) {
      const uint32_t xa = sa[i], xb = sb[i];
      sa[i] = ra;
      sb[i] = rb;
      ra += xa;
      rb += xb;
    }
    sa[nw] = ra;
    sb[nw] = rb;
  }
  __syncthreads();
  a = sa[w] + ia - a;
  b = sb[w] + ib - b;
  tot_a = sa[nw];
  tot_b = sb[nw];
  __syncthreads();
}

constexpr uint32_t kSmallBucket = 64;     // buckets up to this size are ordered by one wavefront
constexpr int kLdsSortMax = 8192;         // larger buckets are ranked by counting

// One block per table of the chunk.
__global__ __launch_bounds__(kScanThreads) void scan_kernel(
    const uint32_t* __restrict__ cnt, int64_t NB, int64_t A, int K, int rounding, int kappa,
    uint32_t* __restrict__ start, uint32_t* __restrict__ offsets_chunk,
    uint64_t* __restrict__ meta, uint64_t* __restrict__ large, uint32_t* __restrict__ n_large) {
  __shared__ uint32_t sa[kScanThreads / 64 + 1], sb[kScanThreads / 64 + 1];
  const int tt = blockIdx.x;
  const uint32_t* c = cnt + (size_t)tt * NB;
  uint32_t* st = start + (size_t)tt * (NB + 1);
  uint32_t* of = offsets_chunk + (size_t)tt * (NB + 1);
  const int64_t seg = (NB + kScanThreads - 1) / kScanThreads;
  const int64_t b0 = (int64_t)threadIdx.x * seg;
  const int64_t b1 = b0 + seg < NB ? b0 + seg : NB;
  uint32_t sc = 0, sk = 0, mk = 0;
  for (int64_t b = b0; b < b1; ++b) {
    const uint32_t B = c[b];
    const uint32_t kp = keep_of(B, A, K, rounding, kappa);
    sc += B;
    sk += kp;
    mk = kp > mk ? kp : mk;
  }
  uint32_t tc, tk;
  block_scan2(sc, sk, tc, tk, sa, sb);
  for (int64_t b = b0; b < b1; ++b) {
    const uint32_t B = c[b];
    const uint32_t kp = keep_of(B, A, K, rounding, kappa);
    st[b] = sc;
    of[b] = sk;
    sc += B;
    sk += kp;
    if (B > kSmallBucket && kp > 0) large[atomicAdd(n_large, 1u)] = ((uint64_t)tt << 32) | (uint64_t)b;
  }
  if (threadIdx.x == 0) {
    st[NB] = tc;
    of[NB] = tk;
    meta[2 + tt] = tk;   // table size
  }
  if (mk) atomicMax((unsigned long long*)&meta[1], (unsigned long long)mk);
}

// Table starts: tbase[t] = running total (meta[0]) before table t.
__global__ void bases_kernel(int t0, int Tc, uint64_t* __restrict__ meta,
                             uint64_t* __restrict__ tbase) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  uint64_t run = meta[0];
  for (int tt = 0; tt < Tc; ++tt) {
    tbase[t0 + tt] = run;
    run += meta[2 + tt];
  }
  meta[0] = run;
  tbase[t0 + Tc] = run;
}

__global__ __launch_bounds__(256) void scatter_kernel(
    const uint32_t* __restrict__ rec_bucket, const float* __restrict__ rec_key, int64_t nK, int K,
    int64_t NB, const uint32_t* __restrict__ start, uint32_t* __restrict__ fill,
    float* __restrict__ srt_key, int32_t* __restrict__ srt_id) {
  const int tt = blockIdx.y;
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= nK) return;
  const size_t o = (size_t)tt * nK;
  const uint32_t b = rec_bucket[o + r];
  if (b == kDropped) return;
  const uint32_t pos = start[(size_t)tt * (NB + 1) + b] + atomicAdd(&fill[(size_t)tt * NB + b], 1u);
  srt_key[o + pos] = rec_key[o + r];
  srt_id[o + pos] = (int32_t)(r / K);
}

// Order key of a record: ascending (2^32 - 1 - key bits, id) is (key desc, id asc); keys are
// non-negative floats, whose bit patterns order like their values.
__device__ __forceinline__ uint64_t order_key(float key, int32_t id) {
  return ((uint64_t)(0xffffffffu - __float_as_uint(key)) << 32) | (uint32_t)id;
}

// Buckets of at most 64 records: one wavefront per bucket, lane x holds record x and counts
// the records that precede it.
__global__ __launch_bounds__(256) void order_small_kernel(
    int64_t NB, int64_t nK, int t0, const uint32_t* __restrict__ start,
    const uint32_t* __restrict__ offsets_chunk, const float* __restrict__ srt_key,
    const int32_t* __restrict__ srt_id, const uint64_t* __restrict__ tbase,
    int32_t* __restrict__ ids) {
  const int tt = blockIdx.y;
  const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (b >= NB) return;
  const int lane = threadIdx.x & 63;
  const uint32_t* st = start + (size_t)tt * (NB + 1);
  const uint32_t* of = offsets_chunk + (size_t)tt * (NB + 1);
  const uint32_t s0 = st[b], B = st[b + 1] - s0;
  const uint32_t keep = of[b + 1] - of[b];
  if (B == 0 || B > kSmallBucket || keep == 0) return;   // uniform over the wavefront
  const size_t o = (size_t)tt * nK + s0;
  const uint64_t mine = (uint32_t)lane < B ? order_key(srt_key[o + lane], srt_id[o + lane]) : ~0ull;
  uint32_t rank = 0;
  for (uint32_t x = 0; x < B; ++x) {
    const uint64_t other = ((uint64_t)__shfl((uint32_t)(mine >> 32), (int)x) << 32) |
                           __shfl((uint32_t)mine, (int)x);
    rank += other < mine ? 1u : 0u;
  }
  if ((uint32_t)lane < B && rank < keep)
    ids[tbase[t0 + tt] + of[b] + rank] = (int32_t)(uint32_t)mine;
}

// Buckets of more than 64 records (listed by the scan), one persistent workgroup at a time:
// bitonic sort of the order keys in LDS (up to 8192 records), else ranking by counting over
// LDS tiles with an early exit once a record is out of the kept prefix.
__global__ __launch_bounds__(256) void order_large_kernel(
    int64_t NB, int64_t nK, int t0, const uint64_t* __restrict__ large,
    const uint32_t* __restrict__ n_large, const uint32_t* __restrict__ start,
    const uint32_t* __restrict__ offsets_chunk, const float* __restrict__ srt_key,
    const int32_t* __restrict__ srt_id, const uint64_t* __restrict__ tbase,
    int32_t* __restrict__ ids) {
  extern __shared__ uint64_t sk[];   // kLdsSortMax keys
  const uint32_t total = *n_large;
  for (uint32_t w = blockIdx.x; w < total; w += gridDim.x) {
    const uint64_t tb = large[w];
    const int tt = (int)(tb >> 32);
    const int64_t b = (int64_t)(uint32_t)tb;
    const uint32_t* st = start + (size_t)tt * (NB + 1);
    const uint32_t* of = offsets_chunk + (size_t)tt * (NB + 1);
    const uint32_t s0 = st[b], B = st[b + 1] - s0;
    const uint32_t keep = of[b + 1] - of[b];
    const size_t o = (size_t)tt * nK + s0;
    int32_t* out = ids + tbase[t0 + tt] + of[b];
    if (B <= (uint32_t)kLdsSortMax) {
      uint32_t n = 1;
      while (n < B) n <<= 1;
      for (uint32_t i = threadIdx.x; i < n; i += 256)
        sk[i] = i < B ? order_key(srt_key[o + i], srt_id[o + i]) : ~0ull;
      __syncthreads();
      for (uint32_t k = 2; k <= n; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
          for (uint32_t i = threadIdx.x; i < n; i += 256) {
            const uint32_t ixj = i ^ j;
            if (ixj > i) {
              const uint64_t a = sk[i], c = sk[ixj];
              const bool asc = (i & k) == 0;
              if (asc ? (a > c) : (a < c)) {
                sk[i] = c;
                sk[ixj] = a;
              }
            }
          }
          __syncthreads();
        }
      }
      for (uint32_t r = threadIdx.x; r < keep; r += 256) out[r] = (int32_t)(uint32_t)sk[r];
      __syncthreads();
    } else {
      // rank by counting, tile by tile
      for (uint32_t r0 = 0; r0 < B; r0 += 256) {
        const uint32_t r = r0 + threadIdx.x;
        const uint64_t mine = r < B ? order_key(srt_key[o + r], srt_id[o + r]) : ~0ull;
        uint32_t rank = 0;
        for (uint32_t t0x = 0; t0x < B; t0x += (uint32_t)kLdsSortMax) {
          const uint32_t tn = B - t0x < (uint32_t)kLdsSortMax ? B - t0x : (uint32_t)kLdsSortMax;
          for (uint32_t i = threadIdx.x; i < tn; i += 256)
            sk[i] = order_key(srt_key[o + t0x + i], srt_id[o + t0x + i]);
          __syncthreads();
          if (r < B && rank < keep)
            for (uint32_t i = 0; i < tn; ++i) rank += sk[i] < mine ? 1u : 0u;
          __syncthreads();
        }
        if (r < B && rank < keep) out[rank] = (int32_t)(uint32_t)mine;
      }
    }
  }
}

__global__ __launch_bounds__(256) void absolute_kernel(int64_t NB, int t0,
                                                       const uint64_t* __restrict__ tbase,
                                                       uint32_t* __restrict__ offsets_chunk) {
  const int tt = blockIdx.y;
  const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (b > NB) return;
  offsets_chunk[(size_t)tt * (NB + 1) + b] += (uint32_t)tbase[t0 + tt];
}

}  // namespace

hipError_t launch_build_tables(const fpp_index* ix, int t0, int Tc, const BuildScratch& bs,
                               hipStream_t s) {
  const int64_t nK = ix->n * (int64_t)ix->iProbes;
  const int64_t NB = ix->NB;
  const int K = ix->iProbes;
  uint32_t* offc = ix->offsets + (size_t)t0 * (NB + 1);
  hipError_t e;
  if ((e = hipMemsetAsync(bs.cnt, 0, sizeof(uint32_t) * (size_t)Tc * NB, s)) != hipSuccess) return e;
  if ((e = hipMemsetAsync(bs.fill, 0, sizeof(uint32_t) * (size_t)Tc * NB, s)) != hipSuccess) return e;
  const dim3 grid_r((unsigned)((nK + 255) / 256), (unsigned)Tc);
  hipLaunchKernelGGL(count_kernel, grid_r, dim3(256), 0, s, bs.rec_bucket, nK, NB, bs.cnt);
  if ((e = hipMemsetAsync(bs.n_large, 0, sizeof(uint32_t), s)) != hipSuccess) return e;
  hipLaunchKernelGGL(scan_kernel, dim3(Tc), dim3(kScanThreads), 0, s, bs.cnt, NB,
                     ix->filter == FPP_FILTER_THRESHOLD ? (int64_t)-1 : (int64_t)ix->alpha_micro, K,
                     ix->keep_rounding, ix->kappa, bs.start, offc, bs.meta,
                     bs.large, bs.n_large);
  hipLaunchKernelGGL(bases_kernel, dim3(1), dim3(64), 0, s, t0, Tc, bs.meta, bs.tbase);
  hipLaunchKernelGGL(scatter_kernel, grid_r, dim3(256), 0, s, bs.rec_bucket, bs.rec_key, nK, K, NB,
                     bs.start, bs.fill, bs.srt_key, bs.srt_id);
  hipLaunchKernelGGL(order_small_kernel, dim3((unsigned)((NB + 3) / 4), (unsigned)Tc), dim3(256), 0,
                     s, NB, nK, t0, bs.start, offc, bs.srt_key, bs.srt_id, bs.tbase, ix->ids);
  hipLaunchKernelGGL(order_large_kernel, dim3(2048), dim3(256), sizeof(uint64_t) * kLdsSortMax, s,
                     NB, nK, t0, bs.large, bs.n_large, bs.start, offc, bs.srt_key, bs.srt_id,
                     bs.tbase, ix->ids);
  const dim3 grid_o((unsigned)((NB + 1 + 255) / 256), (unsigned)Tc);
  hipLaunchKernelGGL(absolute_kernel, grid_o, dim3(256), 0, s, NB, t0, bs.tbase, offc);
  return hipGetLastError();
}

}  // namespace fpp
