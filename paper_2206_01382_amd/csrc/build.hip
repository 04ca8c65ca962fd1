// Table build on gfx950 (Algorithm 1, the per-bucket filter; Section 3.4 "alpha-fraction").
//
// For a chunk of Tc tables whose records (bucket, key) were produced by the hash kernel
// (record r of a table belongs to point r / iProbes):
//   1. count    records per bucket (atomics into a [Tc][NB] histogram);
//   2. scan     per table: bucket starts of the grouped records, keep(B) and the CSR offsets of
//               the kept ids (relative to the table), table size and largest kept bucket;
//   3. bases    absolute start of each table in the shared ids array (running over chunks);
//   4. scatter  records grouped by bucket (arbitrary order inside a bucket);
//   5. rank     every record counts the records of its bucket that precede it in
//               (key desc, id asc) order, stopping once it is out of the kept prefix; a kept
//               record writes its id at offset + rank, which makes the result independent of the
//               scatter order;
//   6. absolute CSR offsets += table start.
// keep(B) = ceil(A * B / (iProbes * 10^6)) (or floor) with A = alpha in millionths.
#include "fpp_internal.hpp"

namespace fpp {
namespace {

constexpr int kScanThreads = 1024;

__device__ __forceinline__ uint32_t keep_of(uint32_t B, int64_t A, int K, int rounding) {
  const uint64_t den = (uint64_t)K * 1000000ull;
  const uint64_t num = (uint64_t)B * (uint64_t)A;
  return (uint32_t)(rounding == 0 ? (num + den - 1) / den : num / den);
}

__global__ __launch_bounds__(256) void count_kernel(const uint32_t* __restrict__ rec_bucket,
                                                    int64_t nK, int64_t NB,
                                                    uint32_t* __restrict__ cnt) {
  const int tt = blockIdx.y;
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= nK) return;
  const uint32_t b = rec_bucket[(size_t)tt * nK + r];
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

// One block per table of the chunk.
__global__ __launch_bounds__(kScanThreads) void scan_kernel(
    const uint32_t* __restrict__ cnt, int64_t NB, int64_t A, int K, int rounding,
    uint32_t* __restrict__ start, uint32_t* __restrict__ offsets_chunk,
    uint64_t* __restrict__ meta) {
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
    const uint32_t kp = keep_of(B, A, K, rounding);
    sc += B;
    sk += kp;
    mk = kp > mk ? kp : mk;
  }
  uint32_t tc, tk;
  block_scan2(sc, sk, tc, tk, sa, sb);
  for (int64_t b = b0; b < b1; ++b) {
    const uint32_t B = c[b];
    st[b] = sc;
    of[b] = sk;
    sc += B;
    sk += keep_of(B, A, K, rounding);
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
  const uint32_t pos = start[(size_t)tt * (NB + 1) + b] + atomicAdd(&fill[(size_t)tt * NB + b], 1u);
  srt_key[o + pos] = rec_key[o + r];
  srt_id[o + pos] = (int32_t)(r / K);
}

__global__ __launch_bounds__(256) void rank_kernel(
    const uint32_t* __restrict__ rec_bucket, const float* __restrict__ rec_key, int64_t nK, int K,
    int64_t NB, int t0, const uint32_t* __restrict__ start,
    const uint32_t* __restrict__ offsets_chunk, const float* __restrict__ srt_key,
    const int32_t* __restrict__ srt_id, const uint64_t* __restrict__ tbase,
    int32_t* __restrict__ ids) {
  const int tt = blockIdx.y;
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= nK) return;
  const size_t o = (size_t)tt * nK;
  const uint32_t b = rec_bucket[o + r];
  const uint32_t* of = offsets_chunk + (size_t)tt * (NB + 1);
  const uint32_t keep = of[b + 1] - of[b];
  if (keep == 0) return;
  const float key = rec_key[o + r];
  const int32_t id = (int32_t)(r / K);
  const uint32_t* st = start + (size_t)tt * (NB + 1);
  const uint32_t s0 = st[b], s1 = st[b + 1];
  uint32_t rank = 0;
  for (uint32_t i = s0; i < s1; ++i) {
    const float k2 = srt_key[o + i];
    if (k2 > key || (k2 == key && srt_id[o + i] < id)) {
      if (++rank >= keep) return;
    }
  }
  ids[tbase[t0 + tt] + of[b] + rank] = id;
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
  hipLaunchKernelGGL(scan_kernel, dim3(Tc), dim3(kScanThreads), 0, s, bs.cnt, NB,
                     (int64_t)ix->alpha_micro, K, ix->keep_rounding, bs.start, offc, bs.meta);
  hipLaunchKernelGGL(bases_kernel, dim3(1), dim3(64), 0, s, t0, Tc, bs.meta, bs.tbase);
  hipLaunchKernelGGL(scatter_kernel, grid_r, dim3(256), 0, s, bs.rec_bucket, bs.rec_key, nK, K, NB,
                     bs.start, bs.fill, bs.srt_key, bs.srt_id);
  hipLaunchKernelGGL(rank_kernel, grid_r, dim3(256), 0, s, bs.rec_bucket, bs.rec_key, nK, K, NB,
                     t0, bs.start, offc, bs.srt_key, bs.srt_id, bs.tbase, ix->ids);
  const dim3 grid_o((unsigned)((NB + 1 + 255) / 256), (unsigned)Tc);
  hipLaunchKernelGGL(absolute_kernel, grid_o, dim3(256), 0, s, NB, t0, bs.tbase, offc);
  return hipGetLastError();
}

}  // namespace fpp
