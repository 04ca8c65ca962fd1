// Candidate gather, dedup, scoring and top-k on gfx950 (Section 3.4 multi-probe querying;
// Section 1 problem statement: the answer is the top-k of x^T q).
//
// Persistent 256-thread workgroups (three per CU) take queries one at a time from a device
// counter. For each query:
//   A. the probed CSR ranges are loaded 256 at a time and prefix-summed; every thread takes four
//      consecutive entries, reads their ids and inserts them into an LDS open-addressing set
//      (set semantics: an id is scored once however many buckets hold it). Past 3072 distinct
//      ids the workgroup moves the set into its n-bit bitmap in device memory and continues
//      there. First-time ids enter an LDS queue. A query with more than 16,384 entries (by
//      default; they must fit the workgroup's bitmap region as a buffer) is deduplicated by id
//      range instead: its ids are grouped by id >> 18 into that buffer and each group is tested
//      against an LDS bitmap of its 2^18 ids.
//   B. when the queue holds >= 1024 ids (and at the end) the waves score it: G lanes cover one
//      row with 16-byte loads, each lane folds its chunks into a float32 partial in a fixed order,
//      and a fixed xor-shuffle tree over the G lanes finishes the sum. Scores therefore do not
//      depend on batching or on which workgroup computes them.
//   C. candidates above the running kk-th best key go to an LDS buffer that is sorted and cut to
//      the best kk once it holds more than 255 (kk <= 128; else 3 kk); the final sort gives
//      (score desc, id asc) order.
// Keys are 64-bit: order-preserving float bits << 32 | (0xffffffff - id).
// The low-precision stores (BF16, FP8) produce a short list of R ids (and their approximate
// scores) that the rerank kernel scores exactly in float32 from the FP32 store. For BF16 both
// kernels also drop what provably cannot reach the final top k (rerank_kernel states the bound).
#include <cmath>

#include "fpp_internal.hpp"
#include "lanes.hpp"

namespace fpp {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kEPT = 4;                         // entries per thread per dedup round
constexpr int kRound = kBlock * kEPT;           // entries per dedup round
constexpr int kQueueCap = 2048;
constexpr int kQueueFlush = kQueueCap - kRound; // flush before a round could overflow the queue
constexpr int kCandCap = 1024;
constexpr int kProbeChunk = kBlock;
constexpr int kSetSlots = 8192;                 // LDS id set (open addressing), 2^13 slots
constexpr int kSetLimit = kSetSlots / 2 - kRound;   // switch to the bitmap above this many ids
constexpr uint32_t kEmpty = 0xffffffffu;
constexpr int kBlocksPerCU = 3;                 // ~51 KB of LDS per workgroup
// partitioned dedup (queries with many probed entries): ids are grouped by id >> shift, and each
// group is deduplicated in a bitmap over its 2^shift ids that occupies the set's LDS
constexpr int kMaxPartShift = 18;               // 2^18 bits = kSetSlots words
constexpr int kMaxParts = kBlock;               // id ranges, one count per thread
static_assert((1 << kMaxPartShift) == kSetSlots * 32, "a range's bitmap fits the set's LDS");

template <int STORE>
struct Elems;
template <>
struct Elems<FPP_STORE_FP32> {
  static constexpr int kPerChunk = 4;
};
template <>
struct Elems<FPP_STORE_BF16> {
  static constexpr int kPerChunk = 8;
};
template <>
struct Elems<FPP_STORE_FP8> {
  static constexpr int kPerChunk = 16;
};
template <>
struct Elems<FPP_STORE_SIMHASH> {
  static constexpr int kPerChunk = 4;   // 32-bit signature words; the query row holds its words
};

__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }

// Exact values of the four OCP E4M3 codes of a word (bytes 0..3), by the gfx950 conversion
// instruction, which decodes the OCP format (subnormals m * 2^-9 included) without rounding.
__device__ __forceinline__ void e4m3x4(uint32_t w, float v[4]) {
  const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)w, false);
  const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)w, true);
  v[0] = lo[0];
  v[1] = lo[1];
  v[2] = hi[0];
  v[3] = hi[1];
}

// Fold one 16-byte chunk of a stored row into the running partial p (fixed element order).
template <int STORE>
__device__ __forceinline__ float fold_chunk(float p, const float* qv, uint4 w) {
  if constexpr (STORE == FPP_STORE_FP32) {
    p = __fmaf_rn(qv[0], __uint_as_float(w.x), p);
    p = __fmaf_rn(qv[1], __uint_as_float(w.y), p);
    p = __fmaf_rn(qv[2], __uint_as_float(w.z), p);
    p = __fmaf_rn(qv[3], __uint_as_float(w.w), p);
  } else if constexpr (STORE == FPP_STORE_BF16) {
    const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      p = __fmaf_rn(qv[2 * i], bf16_lo(ws[i]), p);
      p = __fmaf_rn(qv[2 * i + 1], bf16_hi(ws[i]), p);
    }
  } else if constexpr (STORE == FPP_STORE_SIMHASH) {
    // Hamming distance to the query's signature words (small integers, exact in float)
    const int h = __popc(w.x ^ __float_as_uint(qv[0])) + __popc(w.y ^ __float_as_uint(qv[1])) +
                  __popc(w.z ^ __float_as_uint(qv[2])) + __popc(w.w ^ __float_as_uint(qv[3]));
    p += (float)h;
  } else {
    const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float v[4];
      e4m3x4(ws[i], v);
#pragma unroll
      for (int b = 0; b < 4; ++b) p = __fmaf_rn(qv[4 * i + b], v[b], p);
    }
  }
  return p;
}

template <int G>
__device__ __forceinline__ float tree_sum(float p) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) p += xor_lanes_n(p, o);
  return p;
}

// Short-list length of a query with k results (same rule as the host: R, else max(100, 2k),
// at most kMaxK and at least k).
__device__ __forceinline__ int short_len(int R_opt, int k) {
  int R = R_opt > 0 ? R_opt : (2 * k > 100 ? 2 * k : 100);
  R = R < kMaxK ? R : kMaxK;
  return R > k ? R : k;
}

__device__ __forceinline__ uint64_t make_key(float s, int32_t id) {
  s = s + 0.0f;   // -0 -> +0
  const uint32_t u = __float_as_uint(s);
  const uint32_t ord = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
  return ((uint64_t)ord << 32) | (uint32_t)(0xffffffffu - (uint32_t)id);
}
__device__ __forceinline__ int32_t key_id(uint64_t k) {
  return k ? (int32_t)(0xffffffffu - (uint32_t)k) : -1;
}
__device__ __forceinline__ float key_score(uint64_t k) {
  if (!k) return -INFINITY;
  const uint32_t ord = (uint32_t)(k >> 32);
  return __uint_as_float((ord & 0x80000000u) ? (ord & 0x7fffffffu) : ~ord);
}

// Load the query's elements matching the lane's chunks: chunk index c * G + g holds elements
// [(c*G+g)*EPC, +EPC); elements past d are zero.
template <int STORE, int G, int C>
__device__ __forceinline__ void load_query(const float* qrow, int d, int g,
                                           float (&qv)[C][Elems<STORE>::kPerChunk]) {
  constexpr int EPC = Elems<STORE>::kPerChunk;
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int e = 0; e < EPC; ++e) {
      const int el = (c * G + g) * EPC + e;
      qv[c][e] = el < d ? qrow[el] : 0.0f;
    }
}

// Reduce U rows at once over a G-lane group (U, G powers of two). Levels run at distances G/2,
// G/4, ..., 1 like tree_sum, so every row is summed over exactly the same pairs in the same order
// (float addition is commutative), but while a lane still holds several rows it sends half of
// them to its partner and keeps the other half: 8 rows over 32 lanes take 9 shuffles instead of
// 40. Afterwards lane g holds the total of row reduced_row<G, U>(g) in part[0].
template <int G, int U, int O = G / 2, int N = U>
__device__ __forceinline__ void reduce_rows(float (&part)[U], int g) {
  if constexpr (O > 0) {
    if constexpr (N > 1) {
      const bool upper = (g & O) != 0;
#pragma unroll
      for (int i = 0; i < N / 2; ++i) {
        const float send = upper ? part[i] : part[i + N / 2];
        const float keep = upper ? part[i + N / 2] : part[i];
        part[i] = keep + xor_lanes<O>(send);
      }
      reduce_rows<G, U, O / 2, N / 2>(part, g);
    } else {
      part[0] += xor_lanes<O>(part[0]);
      reduce_rows<G, U, O / 2, 1>(part, g);
    }
  }
}

// Row whose total lane g holds after reduce_rows, and whether g reports it (one lane per row).
template <int G, int U>
__device__ __forceinline__ int reduced_row(int g) {
  int row = 0, n = U;
#pragma unroll
  for (int o = G / 2; o > 0 && n > 1; o >>= 1) {
    n >>= 1;
    if (g & o) row += n;
  }
  return row;
}
template <int G, int U>
__device__ __forceinline__ bool reports_row(int g) {
  // the transposing levels use the top log2(U) bits of g; the butterfly levels below them leave
  // equal totals in lanes that differ only in the low bits, of which the one with zeros reports
  static_assert(U <= G, "more rows than lanes per group");
  return (g & (G / U - 1)) == 0;
}

// One bitonic stage (partner distance J, block size k) on a 128-key chunk held as two keys per
// lane (indices i0 = base + lane, i1 = i0 + 64). J is a compile-time constant, so every exchange
// is a DPP move or a row swap (no LDS round trip): the stages form one dependent chain, and
// their latency is what a compaction costs.
template <int J>
__device__ __forceinline__ void chunk_stage(uint64_t& a, uint64_t& b, int i0, int k) {
  if constexpr (J == 64) {
    const bool desc = (i0 & k) == 0;
    if (desc ? (a < b) : (a > b)) {
      const uint64_t t = a;
      a = b;
      b = t;
    }
  } else {
    const uint64_t oa = xor_lanes<J>(a), ob = xor_lanes<J>(b);
    const bool lower = (threadIdx.x & J) == 0;
    const bool da = (i0 & k) == 0, db = ((i0 + 64) & k) == 0;
    const uint64_t amx = a > oa ? a : oa, amn = a > oa ? oa : a;
    const uint64_t bmx = b > ob ? b : ob, bmn = b > ob ? ob : b;
    a = (lower == da) ? amx : amn;
    b = (lower == db) ? bmx : bmn;
  }
}

// Stages J = JTOP, JTOP / 2, ..., 1 of block size k.
template <int JTOP>
__device__ __forceinline__ void chunk_stages(uint64_t& a, uint64_t& b, int i0, int k) {
  chunk_stage<JTOP>(a, b, i0, k);
  if constexpr (JTOP > 1) chunk_stages<JTOP / 2>(a, b, i0, k);
}

// Block sizes k = 2, 4, ..., K of the chunk (K <= 128): the chunk sorted, descending where
// (i0 & K) == 0 and ascending elsewhere.
template <int K>
__device__ __forceinline__ void chunk_sort(uint64_t& a, uint64_t& b, int i0) {
  if constexpr (K > 2) chunk_sort<K / 2>(a, b, i0);
  chunk_stages<K / 2>(a, b, i0, K);
}

// Block-wide bitonic sort (descending) of n keys in LDS, n a power of two >= 128. Stages with a
// partner distance below 128 run in registers (two keys per lane, DPP moves and row swaps), the
// others in LDS.
__device__ __noinline__ void block_sort_desc(uint64_t* key, int n) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int chunks = n >> 7;
  for (int c = wave; c < chunks; c += kWaves) {
    const int i0 = (c << 7) + lane;
    uint64_t a = key[i0], b = key[i0 + 64];
    chunk_sort<128>(a, b, i0);
    key[i0] = a;
    key[i0 + 64] = b;
  }
  __syncthreads();
  for (int k = 256; k <= n; k <<= 1) {
    for (int j = k >> 1; j >= 128; j >>= 1) {
      for (int i = threadIdx.x; i < n; i += kBlock) {
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
    for (int c = wave; c < chunks; c += kWaves) {
      const int i0 = (c << 7) + lane;
      uint64_t a = key[i0], b = key[i0 + 64];
      chunk_stages<64>(a, b, i0, k);
      key[i0] = a;
      key[i0 + 64] = b;
    }
    __syncthreads();
  }
}

__device__ __forceinline__ int sort_size(uint32_t c) {
  int n = 128;
  while ((uint32_t)n < c) n <<= 1;
  return n;
}

// Exclusive block scan of one u32 per thread.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t& total, uint32_t* wsum) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t inc = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(inc, o);
    if (lane >= o) inc += t;
  }
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  uint32_t before = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kWaves; ++i) {
    const uint32_t x = wsum[i];
    before += i < w ? x : 0u;
    tot += x;
  }
  total = tot;
  __syncthreads();
  return before + inc - v;
}

__device__ __forceinline__ uint32_t set_hash(uint32_t id) {
  return (id * 0x9E3779B1u) >> (32 - 13);   // kSetSlots = 2^13
}

struct ScoreParams {
  const unsigned char* Xs;   // store base
  uint32_t ld_bytes;         // store row stride in bytes (at most 4 KB: the offset of a row is
                             // one 32 x 32 -> 64-bit multiply-add)
  int nchunks;               // 16-byte chunks per stored row
  const unsigned char* sc_base;   // FP8 per-row scale of row i at sc_base + i * sc_stride
  uint32_t sc_stride;
  const uint32_t* offsets;
  const int32_t* ids;
  int64_t n;
  int d;
  const float* Q;
  int ldq;
  int64_t m;
  const uint32_t* probes;
  const int32_t* nprobe;
  int32_t qcap;
  const int32_t* k_arr;
  int32_t k_uniform;
  const int64_t* out_off;
  int32_t lowp;              // 0: FP32 store, final answer; 1: short list for the rerank
  int32_t R_opt;             // short-list length option (0 = max(100, 2k))
  int32_t* ids_out;
  float* scores_out;
  int32_t* short_ids;        // [m][short_ld]
  float* short_sc;           // [m][short_ld] approximate scores, or null
  int32_t short_ld;
  float cut_c;               // > 0: bound constant of the rerank's cut (see rerank_kernel)
  int64_t* stats;
  uint32_t* gbitmap;         // [gridDim.x][bm_words], zero on entry and on exit
  uint32_t* work;            // [2]: next query, finished workgroups; zero on entry and on exit
  const unsigned char* zero16;   // 16 bytes that stay zero (after the work counters)
  int64_t bm_words;
  int64_t part_min;          // more probed entries than this: dedup by id range
  int32_t part_shift;        // ids per range: 2^part_shift <= 2^kMaxPartShift
  float sig_bits;            // SimHash: bits per signature
};

struct SharedState {
  uint32_t qcount;
  uint32_t ccount;
  uint32_t uniq;
  uint32_t overflow;
  uint64_t thr;
  int64_t qnext;       // the workgroup's current query
};

// LDS carve-up (byte offsets).
constexpr size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
constexpr size_t kOffCand = 0;
constexpr size_t kOffSet = kOffCand + (size_t)kCandCap * 8;
constexpr size_t kOffQueue = kOffSet + (size_t)kSetSlots * 4;
constexpr size_t kOffBeg = kOffQueue + (size_t)kQueueCap * 4;
constexpr size_t kOffPre = kOffBeg + (size_t)kProbeChunk * 4;
constexpr size_t kOffPart = kOffPre + (size_t)(kProbeChunk + 1) * 4;
constexpr size_t kOffWsum = kOffPart + (size_t)kMaxParts * 4;
constexpr size_t kOffState = align_up(kOffWsum + (size_t)(kWaves + 2) * 4, 8);
constexpr size_t kLdsBytes = align_up(kOffState + sizeof(SharedState), 16);

// Insert into the LDS set; returns true when the id was not there yet.
__device__ __forceinline__ bool set_insert(uint32_t* set, uint32_t id) {
  uint32_t h = set_hash(id);
  for (;;) {
    const uint32_t old = atomicCAS(&set[h], kEmpty, id);
    if (old == kEmpty) return true;
    if (old == id) return false;
    h = (h + 1) & (kSetSlots - 1);
  }
}

__device__ __forceinline__ bool bitmap_insert(uint32_t* bm, uint32_t id) {
  const uint32_t bit = 1u << (id & 31);
  return !(atomicOr(&bm[id >> 5], bit) & bit);
}

template <int STORE, int G, int C>
__global__ __launch_bounds__(kBlock) void score_kernel(ScoreParams p) {
  constexpr int EPC = Elems<STORE>::kPerChunk;
  constexpr int U = 8 / C;                 // rows in flight per lane
  constexpr int RPI = 64 / G;              // rows per wave instruction
  constexpr int RPW = U * RPI;             // rows per wave pass
  constexpr int RPB = RPW * kWaves;        // rows per block pass
  constexpr int PPC = 2;                   // passes between block syncs (double-buffered)
  // after a compaction at most max(kk, trig) <= kCandCap - PPC * RPB candidates remain, and one
  // sync group appends at most PPC * RPB
  static_assert(PPC * RPB <= kCandCap - kMaxK, "candidate buffer too small");

  extern __shared__ __align__(16) unsigned char smem[];
  uint64_t* cand = reinterpret_cast<uint64_t*>(smem + kOffCand);
  uint32_t* set = reinterpret_cast<uint32_t*>(smem + kOffSet);
  uint32_t* queue = reinterpret_cast<uint32_t*>(smem + kOffQueue);
  uint32_t* s_beg = reinterpret_cast<uint32_t*>(smem + kOffBeg);
  uint32_t* s_pre = reinterpret_cast<uint32_t*>(smem + kOffPre);
  uint32_t* s_part = reinterpret_cast<uint32_t*>(smem + kOffPart);
  uint32_t* wsum = reinterpret_cast<uint32_t*>(smem + kOffWsum);
  SharedState* st = reinterpret_cast<SharedState*>(smem + kOffState);
  uint32_t* bitmap = p.gbitmap + (size_t)blockIdx.x * p.bm_words;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane % G, sub = lane / G;

  for (int i = tid; i < kSetSlots; i += kBlock) set[i] = kEmpty;
  __syncthreads();

  // queries are handed out one at a time from a device counter, so that workgroups that draw
  // cheap queries take more of them and the launch ends evenly
  for (;;) {
    if (tid == 0) st->qnext = (int64_t)atomicAdd(&p.work[0], 1u);
    __syncthreads();
    const int64_t q = st->qnext;
    if (q >= p.m) break;   // uniform
    const int k = p.k_arr ? p.k_arr[q] : p.k_uniform;
    const int kk = p.lowp ? short_len(p.R_opt, k) : k;   // list length kept by this pass
    float qv[C][EPC];
    load_query<STORE, G, C>(p.Q + q * p.ldq, p.d, g, qv);
    // with a rerank cut (see rerank_kernel): 2 * its bound for this query, else 0
    float cut_b2 = 0.0f;
    if constexpr (STORE == FPP_STORE_BF16) {
      if (p.cut_c > 0.0f) {
        float ss = 0.0f;
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
          for (int e = 0; e < EPC; ++e) ss = fmaf(qv[c][e], qv[c][e], ss);
        cut_b2 = 2.0f * p.cut_c * (sqrtf(tree_sum<G>(ss)) * 1.0000152587890625f);
      }
    }
    if (tid == 0) {
      st->qcount = 0;
      st->ccount = 0;
      st->uniq = 0;
      st->overflow = 0;
      st->thr = 0;
    }
    __syncthreads();

    // keep the best kk candidates (sorted) and raise the threshold. With a rerank cut the
    // threshold is at least the k-th best approximate score so far minus 2 * the bound: a later
    // candidate below it scores below the final short list's k-th approximate score minus that,
    // which the rerank would not rescore, so the result does not change
    auto compact = [&]() {
      const uint32_t c0 = st->ccount;
      const int n = sort_size(c0);
      for (int i = tid; i < n; i += kBlock)
        if ((uint32_t)i >= c0) cand[i] = 0ull;
      __syncthreads();
      block_sort_desc(cand, n);
      if (tid == 0) {
        st->ccount = c0 < (uint32_t)kk ? c0 : (uint32_t)kk;
        uint64_t thr = st->thr;
        if (c0 >= (uint32_t)kk) thr = cand[kk - 1];
        if (cut_b2 > 0.0f && c0 >= (uint32_t)k) {
          const float a = key_score(cand[k - 1]);
          // the last term covers the rounding of the subtraction
          const float t2 = a - cut_b2 - (fabsf(a) + cut_b2) * 2.384185791015625e-07f;   // 2^-22
          const uint32_t u = __float_as_uint(t2 + 0.0f);
          const uint32_t ord = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
          const uint64_t thr2 = ((uint64_t)ord << 32) - 1ull;   // every key scoring >= t2 passes
          thr = thr2 > thr ? thr2 : thr;
        }
        st->thr = thr;
      }
      __syncthreads();
    };

    // ---- B: scoring of the queued ids. Each wave walks its rows in passes of RPW rows; the
    // loads of the next pass are issued before the current pass is folded (two register sets).
    // The block synchronises every PPC passes, when the candidate buffer may need compaction.
    // loads the pass's row chunks and, for the FP8 store, the per-row scale of the row this lane
    // reports after the reduction (issued with the rows, so its latency overlaps theirs)
    // Every lane issues all its loads unconditionally, so that no load sits in a branch: the wait
    // before a fold then covers exactly that pass's loads and lets the other pass's stay in
    // flight. A row past the queue re-reads the queue's last row (its score is not used); a chunk
    // past the row's end reads the 16 zero bytes at p.zero16. Requires rows > 0.
    auto load_pass = [&](uint32_t rbase, uint32_t rows, uint4 (&w)[U][C], float& scl) {
      if constexpr (STORE == FPP_STORE_FP8) {
        const uint32_t myrow = rbase + (uint32_t)reduced_row<G, U>(g) * RPI + sub;
        // (inside the row itself when the store keeps it there: the same line as the codes)
        scl = *reinterpret_cast<const float*>(
            p.sc_base + (uint64_t)queue[myrow < rows ? myrow : rows - 1] * p.sc_stride);
      }
      uint32_t rid[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t row = rbase + u * RPI + sub;
        rid[u] = queue[row < rows ? row : rows - 1];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t row = rbase + u * RPI + sub;
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const int ci = c * G + g;
          const unsigned char* a = ci < p.nchunks
                                       ? p.Xs + (uint64_t)rid[u] * p.ld_bytes + (uint32_t)ci * 16u
                                       : p.zero16;
          w[u][c] = *reinterpret_cast<const uint4*>(a);
        }
      }
    };
    auto fold_pass = [&](uint32_t rbase, uint32_t rows, const uint4 (&w)[U][C], float scl, uint64_t thr) {
      float part[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        part[u] = 0.0f;
#pragma unroll
        for (int c = 0; c < C; ++c) part[u] = fold_chunk<STORE>(part[u], qv[c], w[u][c]);
      }
      reduce_rows<G, U>(part, g);
      // the lane that reports row `myrow` reads the row's id from the queue
      const uint32_t myrow = rbase + (uint32_t)reduced_row<G, U>(g) * RPI + sub;
      const int32_t myid = myrow < rows ? (int32_t)queue[myrow] : -1;
      float s = part[0];
      if constexpr (STORE == FPP_STORE_FP8) s = s * scl;
      if constexpr (STORE == FPP_STORE_SIMHASH) s = p.sig_bits - 2.0f * s;   // F*D - 2 Hamming
      const uint64_t key = make_key(s, myid);
      const bool pass = reports_row<G, U>(g) && myid >= 0 && key > thr;
      const uint64_t mask = __ballot(pass);
      if (mask) {
        uint32_t basepos = 0;
        if (lane == 0) basepos = atomicAdd(&st->ccount, (uint32_t)__popcll(mask));
        basepos = __builtin_amdgcn_readfirstlane(basepos);
        if (pass) cand[basepos + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull))] = key;
      }
    };

    // flush the queue through the scoring passes; `last` also leaves the candidates sorted
    auto score_queue = [&](bool last) {
      const uint32_t rows = st->qcount;
      static_assert(PPC == 2, "two passes per barrier: set a folds while set b loads");
      for (uint32_t sb = 0; sb < rows || (last && sb == 0); sb += PPC * RPB) {
        const uint64_t thr = st->thr;
        // wave-uniform branches, no sync inside. Both passes' loads are issued before either
        // fold (set b re-reads the queue's last row when its pass is past the queue).
        const uint32_t b0 = sb + wave * RPW, b1 = b0 + RPB;
        if (b0 < rows) {
          uint4 wa[U][C], wb[U][C];
          float sa = 0.0f, sbs = 0.0f;
          load_pass(b0, rows, wa, sa);
          load_pass(b1, rows, wb, sbs);
          fold_pass(b0, rows, wa, sa, thr);
          if (b1 < rows) fold_pass(b1, rows, wb, sbs, thr);
        }
        __syncthreads();
        const bool fin = last && sb + PPC * RPB >= rows;
        // compact once the buffer holds more than 255 entries (kk <= 128; else 3 kk): the first
        // sync group's rows then sort as one 256-key block, the threshold rises early enough that
        // most later rows are rejected without a store (with the rerank cut's threshold, nearly
        // all), and a query needs about two sorts (a trigger of 200 took three at kk = 100)
        uint32_t trig = (uint32_t)(kk <= 128 ? 255 : 3 * kk);
        if (trig > (uint32_t)(kCandCap - PPC * RPB)) trig = (uint32_t)(kCandCap - PPC * RPB);
        if (fin || st->ccount > trig) compact();
      }
      if (tid == 0) st->qcount = 0;
      __syncthreads();
    };

    // ---- A: gather + dedup, flushing the queue into B whenever it fills
    const int32_t np = p.nprobe[q];
    const uint32_t* pr = p.probes + (size_t)q * p.qcap;

    // CSR ranges of probes [c, c + nc) into s_beg / s_pre (exclusive prefix of the lengths);
    // returns the chunk's entry count
    // (rc: the ranges come from the copy the entry count left at the tail of the bitmap region,
    // a contiguous read, instead of the probe list and two offset lookups per probe)
    uint32_t* rcache = nullptr;   // [np] range begins, then [np] lengths
    auto scan_chunk = [&](int32_t c, int nc, bool rc = false) -> uint32_t {
      uint32_t beg = 0, len = 0;
      if (tid < nc) {
        if (rc) {
          beg = rcache[c + tid];
          len = rcache[np + c + tid];
        } else {
          const uint32_t gb = pr[c + tid];
          beg = p.offsets[gb];
          len = p.offsets[gb + 1] - beg;
        }
      }
      uint32_t ec;
      const uint32_t pre = block_excl_scan(len, ec, wsum);
      s_beg[tid] = beg;
      s_pre[tid] = pre;
      if (tid == 0) s_pre[kProbeChunk] = ec;
      __syncthreads();
      return ec;
    };
    // the ids of entries [e, e + kEPT) of the scanned chunk (-1 past its end): one search, then a
    // linear walk over the probes
    auto load_entries = [&](uint32_t e, uint32_t ec, int nc, int32_t (&idv)[kEPT]) {
#pragma unroll
      for (int u = 0; u < kEPT; ++u) idv[u] = -1;
      if (e < ec) {
        int lo = 0, hi = nc;   // s_pre[lo] <= e < s_pre[hi]
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (s_pre[mid] <= e) lo = mid;
          else hi = mid;
        }
#pragma unroll
        for (int u = 0; u < kEPT; ++u) {
          const uint32_t eu = e + u;
          if (eu < ec) {
            while (s_pre[lo + 1] <= eu) ++lo;
            idv[u] = p.ids[s_beg[lo] + (eu - s_pre[lo])];
          }
        }
      }
    };
    // queue the first occurrences (bit u of `fresh`) in lane-major order: one ballot per entry
    // slot gives every lane the count of fresh entries of the lanes below it
    auto enqueue = [&](const int32_t (&idv)[kEPT], uint32_t fresh) {
      const uint64_t below = (1ull << lane) - 1ull;
      uint32_t before = 0, wtot = 0;
#pragma unroll
      for (int u = 0; u < kEPT; ++u) {
        const uint64_t mk = __ballot((fresh >> u) & 1u);
        before += (uint32_t)__popcll(mk & below);
        wtot += (uint32_t)__popcll(mk);
      }
      uint32_t basepos = 0;
      if (lane == 0 && wtot) {
        basepos = atomicAdd(&st->qcount, wtot);
        atomicAdd(&st->uniq, wtot);
      }
      basepos = __builtin_amdgcn_readfirstlane(basepos);
      uint32_t pos = basepos + before;
#pragma unroll
      for (int u = 0; u < kEPT; ++u)
        if (fresh & (1u << u)) queue[pos++] = (uint32_t)idv[u];
      __syncthreads();
    };

    // entry count: the first chunk's scan, or (more than one chunk) a pass over all the ranges
    uint64_t entries = 0;
    int32_t pc = 0;      // next probe chunk
    int npc = 0;         // probes in the current chunk
    uint32_t ec = 0;     // entries of the current chunk
    if (np > 0 && np <= kProbeChunk) {
      npc = np;
      ec = scan_chunk(0, npc);
      entries = ec;
      pc = kProbeChunk;
    } else if (np > kProbeChunk) {
      // more than one chunk: the ranges are also copied to the tail of the workgroup's bitmap
      // region (zero on entry), for the id-range passes below; the copy is cleared again if the
      // query does not take them
      if (2 * (int64_t)np <= p.bm_words) rcache = bitmap + (p.bm_words - 2 * (int64_t)np);
      for (int32_t c = 0; c < np; c += kProbeChunk) {
        const int nc = np - c < kProbeChunk ? np - c : kProbeChunk;
        uint32_t len = 0;
        if (tid < nc) {
          const uint32_t gb = pr[c + tid];
          const uint32_t beg = p.offsets[gb];
          len = p.offsets[gb + 1] - beg;
          if (rcache) {
            rcache[c + tid] = beg;
            rcache[np + c + tid] = len;
          }
        }
        uint32_t tot;
        (void)block_excl_scan(len, tot, wsum);
        entries += tot;
      }
    }
    const int pshift = p.part_shift;
    const int64_t nparts = (p.n + ((int64_t)1 << pshift) - 1) >> pshift;
    // the id buffer [0, entries) must stay clear of the range copy at the region's tail
    const uint64_t room = (uint64_t)p.bm_words - (rcache ? 2 * (uint64_t)np : 0);
    const bool partitioned = (int64_t)entries > p.part_min && entries <= room &&
                             nparts <= (int64_t)kMaxParts && (np <= kProbeChunk || rcache);
    if (rcache && !partitioned) {
      // the region is the dedup bitmap on the other path: the copy returns to zero first
      for (int32_t i = tid; i < 2 * np; i += kBlock) rcache[i] = 0u;
      __threadfence();
      __syncthreads();
      rcache = nullptr;
    }
    const bool rc = rcache != nullptr;

    if (partitioned) {
      // ---- A': many entries. Pass 1 counts the entries of each id range, pass 2 writes their ids
      // range by range into the workgroup's bitmap region (used as a buffer: it holds at least
      // `entries` words), pass 3 deduplicates each range in an LDS bitmap over its 2^pshift ids
      // (the set's memory) and queues the first occurrences. Three reads of the probed ids
      // and one write of them replace one device atomic per entry and the clearing of an n-bit
      // bitmap; with more than one probe chunk, passes 1 and 2 take the probe ranges from the
      // copy the entry count made (a contiguous read) instead of two offset lookups per probe.
      uint32_t* buf = bitmap;
      const uint32_t E = (uint32_t)entries;
      static_assert(kMaxParts == kBlock, "one range count per thread");
      s_part[tid] = 0u;
      __syncthreads();
      for (int pass = 0; pass < 2; ++pass) {
        for (int32_t c = 0; c < np; c += kProbeChunk) {
          const int nc = np - c < kProbeChunk ? np - c : kProbeChunk;
          const uint32_t ecc = scan_chunk(c, nc, rc);
          for (uint32_t r = 0; r < ecc; r += kRound) {
            int32_t idv[kEPT];
            load_entries(r + (uint32_t)tid * kEPT, ecc, nc, idv);
#pragma unroll
            for (int u = 0; u < kEPT; ++u) {
              if (idv[u] >= 0) {
                const uint32_t pi = (uint32_t)idv[u] >> pshift;
                const uint32_t at = atomicAdd(&s_part[pi], 1u);
                if (pass == 1) buf[at] = (uint32_t)idv[u];
              }
            }
          }
        }
        __syncthreads();
        if (pass == 0) {
          // counts -> first position of each range; after pass 2 s_part[i] is the end of range i
          const uint32_t v = s_part[tid];
          uint32_t tot;
          const uint32_t ex = block_excl_scan(v, tot, wsum);
          s_part[tid] = ex;
          __syncthreads();
        }
      }
      uint32_t* bm = set;
      for (int i = tid; i < kSetSlots; i += kBlock) bm[i] = 0u;
      __syncthreads();
      const uint32_t kLow = (1u << pshift) - 1u;
      for (int pi = 0; pi < (int)nparts; ++pi) {
        const uint32_t beg = pi ? s_part[pi - 1] : 0u, end = s_part[pi];
        for (uint32_t r = beg; r < end; r += kRound) {
          int32_t idv[kEPT];
          uint32_t fresh = 0;
#pragma unroll
          for (int u = 0; u < kEPT; ++u) {
            const uint32_t e = r + (uint32_t)tid * kEPT + u;
            idv[u] = e < end ? (int32_t)buf[e] : -1;
          }
#pragma unroll
          for (int u = 0; u < kEPT; ++u) {
            if (idv[u] >= 0) {
              const uint32_t b = (uint32_t)idv[u] & kLow, m = 1u << (b & 31u);
              fresh |= (atomicOr(&bm[b >> 5], m) & m) ? 0u : (1u << u);
            }
          }
          enqueue(idv, fresh);
          if (st->qcount >= (uint32_t)kQueueFlush) score_queue(false);
        }
        // clear the words of this range's ids
        for (uint32_t e = beg + tid; e < end; e += kBlock) bm[(buf[e] & kLow) >> 5] = 0u;
        __syncthreads();
      }
      score_queue(true);
      // the buffer and the range copy return to zero (they are the bitmap region), the set's
      // memory to empty slots
      for (uint32_t e = tid; e < E; e += kBlock) buf[e] = 0u;
      if (rc)
        for (int32_t i = tid; i < 2 * np; i += kBlock) rcache[i] = 0u;
      __threadfence();
    } else {
      uint32_t e0 = 0;     // next entry of the current chunk
      for (;;) {
        bool exhausted = false;
        while (st->qcount < (uint32_t)kQueueFlush) {
          if (e0 >= ec) {
            if (pc >= np) {
              exhausted = true;
              break;
            }
            npc = np - pc < kProbeChunk ? np - pc : kProbeChunk;
            ec = scan_chunk(pc, npc);   // (entries were counted above)
            pc += kProbeChunk;
            e0 = 0;
            continue;
          }
          const bool ovf = st->overflow != 0;
          int32_t idv[kEPT];
          load_entries(e0 + (uint32_t)tid * kEPT, ec, npc, idv);
          e0 += kRound;
          uint32_t fresh = 0;   // bit u: entry u is a first occurrence
#pragma unroll
          for (int u = 0; u < kEPT; ++u) {
            if (idv[u] >= 0) {
              const bool f = ovf ? bitmap_insert(bitmap, (uint32_t)idv[u]) : set_insert(set, (uint32_t)idv[u]);
              fresh |= f ? (1u << u) : 0u;
            }
          }
          enqueue(idv, fresh);
          if (!st->overflow && st->uniq > (uint32_t)kSetLimit) {
            // move the set into the device bitmap; later entries are tested there
            for (int i = tid; i < kSetSlots; i += kBlock) {
              const uint32_t v = set[i];
              if (v != kEmpty) {
                atomicOr(&bitmap[v >> 5], 1u << (v & 31));
                set[i] = kEmpty;
              }
            }
            __threadfence_block();
            __syncthreads();
            if (tid == 0) st->overflow = 1;
            __syncthreads();
          }
        }
        score_queue(exhausted);
        if (exhausted) break;
      }
    }

    // ---- C: output (the candidates are sorted)
    {
      const uint32_t c0 = st->ccount;
      if (!p.lowp) {
        const int64_t o = p.out_off ? p.out_off[q] : q * (int64_t)k;
        for (int r = tid; r < k; r += kBlock) {
          const uint64_t key = (uint32_t)r < c0 ? cand[r] : 0ull;
          p.ids_out[o + r] = key_id(key);
          p.scores_out[o + r] = key_score(key);
        }
      } else {
        int32_t* so = p.short_ids + (size_t)q * p.short_ld;
        float* ss = p.short_sc ? p.short_sc + (size_t)q * p.short_ld : nullptr;
        for (int r = tid; r < kk; r += kBlock) {
          const uint64_t key = (uint32_t)r < c0 ? cand[r] : 0ull;
          so[r] = key_id(key);
          if (ss) ss[r] = (uint32_t)r < c0 ? key_score(key) : -INFINITY;
        }
      }
      if (tid == 0 && p.stats) {
        p.stats[q * 3 + 0] = np;
        p.stats[q * 3 + 1] = (int64_t)entries;
        p.stats[q * 3 + 2] = st->uniq;
      }
    }

    // ---- clear the dedup state
    if (st->overflow) {
      // the whole bitmap returns to zero (coalesced 16-byte stores)
      uint4* bm4 = reinterpret_cast<uint4*>(bitmap);
      const int64_t n4 = p.bm_words / 4;
      for (int64_t i = tid; i < n4; i += kBlock) bm4[i] = make_uint4(0u, 0u, 0u, 0u);
      for (int64_t i = n4 * 4 + tid; i < p.bm_words; i += kBlock) bitmap[i] = 0u;
      __threadfence();
    } else {
      // the set holds exactly the query's distinct ids (at most kSetLimit + kRound): reset slots
      for (int i = tid; i < kSetSlots; i += kBlock) set[i] = kEmpty;
    }
    __syncthreads();
  }
  // the last workgroup to finish returns the counters to zero for the next launch (every
  // workgroup has drawn its last query before it counts itself finished)
  if (tid == 0) {
    __threadfence();
    if (atomicAdd(&p.work[1], 1u) == gridDim.x - 1) {
      atomicExch(&p.work[0], 0u);
      atomicExch(&p.work[1], 0u);
    }
  }
}

// Exact float32 rerank of a short list (one 256-thread block per query); the same lane layout
// and reduction tree as the FP32 scoring pass, so a reranked score equals the FP32-path score.
// With bound_c > 0 (every row's approximate score is within bound_c * ||q|| of its FP32 score,
// and the list is in descending approximate order), rows from the first one past position k - 1
// whose approximate score is below a(k-1) - 2 bound_c ||q|| are not rescored: each of them scores
// below a(k-1) - bound_c ||q||, and so below the k listed rows before it, so the top k is the
// same as over the whole list.
template <int G, int C>
__global__ __launch_bounds__(256) void rerank_kernel(
    const float* __restrict__ X, int64_t ldx, int nchunks, int d, const float* __restrict__ Q,
    int ldq, int64_t m, const int32_t* __restrict__ short_ids, const float* __restrict__ short_sc,
    int short_ld, float bound_c, const int32_t* __restrict__ k_arr, int k_uniform, int R_opt,
    const int64_t* __restrict__ out_off, int32_t* __restrict__ ids_out,
    float* __restrict__ scores_out) {
  constexpr int RPI = 64 / G;
  __shared__ uint64_t key[kMaxK];
  __shared__ int s_cut;
  const int64_t q = blockIdx.x;
  if (q >= m) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane % G, sub = lane / G;
  const int k = k_arr ? k_arr[q] : k_uniform;
  int R = short_len(R_opt, k);
  float qv[C][4];
  load_query<FPP_STORE_FP32, G, C>(Q + q * ldq, d, g, qv);
  const int32_t* sl = short_ids + (size_t)q * short_ld;
  if (bound_c > 0.0f && short_sc && R > k) {
    // ||q||: the G lanes of a row group hold all of q; the factor covers the rounding of the sum
    // of squares and of the root, so qn >= ||q||
    float ss = 0.0f;
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int e = 0; e < 4; ++e) ss = fmaf(qv[c][e], qv[c][e], ss);
    const float qn = sqrtf(tree_sum<G>(ss)) * 1.0000152587890625f;
    const float* sa = short_sc + (size_t)q * short_ld;
    const float ak = sa[k - 1];
    const float b2 = 2.0f * bound_c * qn;
    // the last term covers the rounding of b2 and of the subtraction
    const float t = ak - b2 - (fabsf(ak) + b2) * 2.384185791015625e-07f;   // 2^-22
    if (tid == 0) s_cut = R;
    __syncthreads();
    for (int r = k + tid; r < R; r += 256)
      if (!(sa[r] >= t)) atomicMin(&s_cut, r);
    __syncthreads();
    R = s_cut;
  }
  const int Rp2 = sort_size((uint32_t)R);
  for (int r0 = 0; r0 < Rp2; r0 += 4 * RPI) {
    const int r = r0 + wave * RPI + sub;
    const int32_t id = r < R ? sl[r] : -1;
    float part = 0.0f;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int ci = c * G + g;
      uint4 w = make_uint4(0u, 0u, 0u, 0u);
      if (id >= 0 && ci < nchunks)
        w = *reinterpret_cast<const uint4*>(X + (size_t)id * ldx + (size_t)ci * 4);
      part = fold_chunk<FPP_STORE_FP32>(part, qv[c], w);
    }
    const float s = tree_sum<G>(part);
    if (g == 0 && r < Rp2) key[r] = id >= 0 ? make_key(s, id) : 0ull;
  }
  __syncthreads();
  block_sort_desc(key, Rp2);
  const int64_t o = out_off ? out_off[q] : q * (int64_t)k;
  for (int r = tid; r < k; r += 256) {
    const uint64_t kk = r < Rp2 ? key[r] : 0ull;
    ids_out[o + r] = key_id(kk);
    scores_out[o + r] = key_score(kk);
  }
}

template <int STORE, int G, int C>
hipError_t launch_score_t(const ScoreParams& sp, int grid, hipStream_t s) {
  auto kern = score_kernel<STORE, G, C>;
  const hipError_t e = hipFuncSetAttribute((const void*)kern,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), kLdsBytes, s, sp);
  return hipGetLastError();
}

// (G, C) per store and chunk count: G = lanes per row (power of two), C = chunks per lane. Up to
// 32 chunks (512 bytes) a row takes 8 lanes: each load instruction still covers whole 128-byte
// lines of a row, and fewer lanes per row mean fewer reduction levels and address computations.
template <int STORE>
hipError_t dispatch_store(const ScoreParams& sp, int grid, hipStream_t s) {
  const int nc = sp.nchunks;
  if (nc <= 8) return launch_score_t<STORE, 8, 1>(sp, grid, s);
  if (nc <= 16) return launch_score_t<STORE, 8, 2>(sp, grid, s);
  if (nc <= 32) return launch_score_t<STORE, 8, 4>(sp, grid, s);
  if (nc <= 64) return launch_score_t<STORE, 64, 1>(sp, grid, s);
  if (nc <= 128) return launch_score_t<STORE, 64, 2>(sp, grid, s);
  if (nc <= 256) return launch_score_t<STORE, 64, 4>(sp, grid, s);
  return hipErrorInvalidValue;
}

}  // namespace

int64_t overflow_bitmap_words(const fpp_index* ix) {
  return ((ix->n + 31) / 32 + 3) & ~(int64_t)3;   // per workgroup, a multiple of 16 bytes
}

int score_grid_blocks(const fpp_index* ix) {
  (void)ix;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256 * kBlocksPerCU;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 256 * kBlocksPerCU;
  return (cus > 0 ? cus : 256) * kBlocksPerCU;
}

// |approximate - FP32 score| for a BF16 row: the rounding of x to BF16 (at most 2^-9 |x_j|) and
// the float32 rounding of the two sums (chains of at most d + 16 steps, gamma = (d + 16) u /
// (1 - (d + 16) u), u = 2^-24, for each), against sum_j |q_j x_j| <= ||q|| ||x||:
// (2^-9 + 2.01 gamma) ||q|| max_i ||x_i||, rounded up.
float bf16_rerank_bound(const fpp_index* ix) {
  if (!(ix->xnorm_max > 0.0f)) return -1.0f;
  const double u = std::ldexp(1.0, -24), mm = (double)ix->d + 16.0;
  const double gamma = mm * u / (1.0 - mm * u);
  const double c = (std::ldexp(1.0, -9) + 2.01 * gamma) * (double)ix->xnorm_max * (1.0 + 1e-6);
  return std::nextafter((float)c, INFINITY);
}

hipError_t launch_score(const fpp_index* ix, const ScoreArgs& a, hipStream_t s) {
  if (a.m <= 0) return hipSuccess;
  if (!a.gbitmap) return hipErrorInvalidValue;
  ScoreParams sp{};
  sp.offsets = ix->offsets;
  sp.ids = ix->ids;
  sp.n = ix->n;
  sp.d = ix->d;
  sp.Q = a.Q;
  sp.ldq = a.ldq;
  sp.m = a.m;
  sp.probes = a.probes;
  sp.nprobe = a.nprobe;
  sp.qcap = a.qcap;
  sp.k_arr = a.k_arr;
  sp.k_uniform = a.k_uniform;
  sp.out_off = a.out_off;
  sp.ids_out = a.ids_out;
  sp.scores_out = a.scores_out;
  sp.stats = a.stats;
  sp.gbitmap = a.gbitmap;
  sp.bm_words = overflow_bitmap_words(ix);
  sp.part_min = ix->part_min;
  sp.part_shift = ix->part_shift;
  sp.work = a.gbitmap + (size_t)a.grid * (size_t)sp.bm_words;   // after the bitmaps
  sp.zero16 = reinterpret_cast<const unsigned char*>(sp.work + 4);   // never written
  sp.short_ids = a.short_ids;
  sp.short_sc = a.short_sc;
  sp.short_ld = a.short_ld;
  sp.cut_c = a.cut_c;
  sp.lowp = (a.store == FPP_STORE_FP32 || a.rerank_R < 0) ? 0 : 1;
  sp.R_opt = a.rerank_R;
  const int grid = a.grid;
  switch (a.store) {
    case FPP_STORE_FP32:
      sp.Xs = reinterpret_cast<const unsigned char*>(ix->X);
      sp.ld_bytes = (uint32_t)ix->ldx * 4u;
      sp.nchunks = ix->ldx / 4;
      return dispatch_store<FPP_STORE_FP32>(sp, grid, s);
    case FPP_STORE_BF16:
      sp.Xs = reinterpret_cast<const unsigned char*>(ix->Xbf16);
      sp.ld_bytes = (uint32_t)ix->ld16 * 2u;
      sp.nchunks = ix->ld16 / 8;
      return dispatch_store<FPP_STORE_BF16>(sp, grid, s);
    case FPP_STORE_FP8:
      sp.Xs = reinterpret_cast<const unsigned char*>(ix->Xfp8);
      sp.ld_bytes = (uint32_t)ix->ld8;
      sp.nchunks = (ix->d + 15) / 16;   // code chunks only
      if (ix->fp8_sc_off >= 0) {
        sp.sc_base = reinterpret_cast<const unsigned char*>(ix->Xfp8) + ix->fp8_sc_off;
        sp.sc_stride = (uint32_t)ix->ld8;
      } else {
        sp.sc_base = reinterpret_cast<const unsigned char*>(ix->fp8_scale);
        sp.sc_stride = 4u;
      }
      return dispatch_store<FPP_STORE_FP8>(sp, grid, s);
    case FPP_STORE_SIMHASH:
      // the query rows (a.Q, a.ldq) are signature words; F * D <= 1024 bits: 8 chunks at most
      if (ix->ldsig > 32) return hipErrorInvalidValue;
      sp.Xs = reinterpret_cast<const unsigned char*>(ix->Xsig);
      sp.ld_bytes = (uint32_t)ix->ldsig * 4u;
      sp.nchunks = ix->ldsig / 4;
      sp.d = ix->ldsig;
      sp.sig_bits = (float)(ix->sigF * ix->D);
      return launch_score_t<FPP_STORE_SIMHASH, 8, 1>(sp, grid, s);
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_rerank(const fpp_index* ix, const float* Q, int ldq, int64_t m,
                         const int32_t* short_ids, const float* short_sc, int short_ld,
                         float bound_c, const int32_t* k_arr, int k_uniform, int R_opt,
                         const int64_t* out_off, int32_t* ids_out, float* scores_out,
                         hipStream_t s) {
  if (m <= 0) return hipSuccess;
  const int nc = ix->ldx / 4;
#define FPP_RERANK(GG, CC)                                                                      \
  hipLaunchKernelGGL((rerank_kernel<GG, CC>), dim3((unsigned)m), dim3(256), 0, s, ix->X,       \
                     (int64_t)ix->ldx, nc, ix->d, Q, ldq, m, short_ids, short_sc, short_ld,     \
                     bound_c, k_arr, k_uniform, R_opt, out_off, ids_out, scores_out)
  if (nc <= 8) FPP_RERANK(8, 1);      // the FP32 gather's (G, C) for the same chunk count
  else if (nc <= 16) FPP_RERANK(8, 2);
  else if (nc <= 32) FPP_RERANK(8, 4);
  else if (nc <= 64) FPP_RERANK(64, 1);
  else if (nc <= 128) FPP_RERANK(64, 2);
  else if (nc <= 256) FPP_RERANK(64, 4);
  else return hipErrorInvalidValue;
#undef FPP_RERANK
  return hipGetLastError();
}

}  // namespace fpp
