// Global probe selection across tables (Section 3.4, multi-probing for querying; Section 2.2
// for qProbes as a total over all L tables).
//
// A query's candidate buckets in table t are the pairs of list positions (i, j) of its two
// sorted |projection| lists (one list for l = 1), scored s = fl32(a_i + b_j). The qProbes best
// over all tables in the order (s desc, table asc, i asc, j asc) are selected without
// materialising the L * D^l pairs:
//   * count_ge(tau) = #{pairs with s >= tau} is a two-pointer walk per table (the number of
//     j with a_i + b_j >= tau does not increase with i because float addition is monotone);
//   * bisection over the bit patterns of non-negative floats finds tau* with
//     count_ge(next(tau*)) < qProbes <= count_ge(tau*);
//   * every pair with s > tau* is taken, then the first pairs with s == tau* in
//     (table, i, j) order until qProbes are selected.
// One workgroup per query; thread x walks tables x, x + 128, ... with the first M entries of
// every sorted list staged in LDS (entries past M are read from device memory).
// When 4 qProbes <= L, a lower bound from the tables' best pairs usually leaves few candidate
// pairs; a first kernel ranks those directly, and the bisection runs only for the queries where
// it could not. (With more probes per table the candidates grow faster than the bisection's
// cost, which is why the direct ranking is kept to this range.)
#include <algorithm>

#include "fpp_internal.hpp"
#include "lanes.hpp"

namespace fpp {
namespace {

constexpr int kProbeThreads = 128;
constexpr int kRankTables = 1024;   // rank the tables' best pairs for the lower bound up to this L
constexpr int kProbeWaves = kProbeThreads / 64;
constexpr int kDirectCap = 256;     // candidate pairs the sparse selection sorts in LDS
constexpr int kDeepFloats = 3328;   // sparse selection: list entries staged per chunk of tables

// Sorted-list access: the first M entries of every list of the query sit in LDS. List f of table
// t (list index l * t + f) is LDS row f * L + t with a row stride of M + 1 words (M is a power of
// two), so the threads of a wavefront, which walk consecutive tables, hit distinct banks.
struct Lists {
  const float* lds;     // [l][L][M + 1]
  const float* glob;    // [LF][D] of this query
  int M, D, L, l;
  __device__ __forceinline__ float get(int list, int i) const {
    const int t = l == 2 ? list >> 1 : list, f = l == 2 ? list & 1 : 0;
    return i < M ? lds[(f * L + t) * (M + 1) + i] : glob[(size_t)list * D + i];
  }
};

// Order-preserving map of floats to u32 (and back): the bisection runs on these keys so that the
// (non-positive) gap scores search like the (non-negative) sums.
__device__ __forceinline__ uint32_t ord_of(float f) {
  const uint32_t b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float of_ord(uint32_t o) {
  return __uint_as_float((o & 0x80000000u) ? (o & 0x7fffffffu) : ~o);
}

// Probe score of a pair: the float32 sum of its |projections|, minus `off` (0 for Falconn++;
// the table's best pair for the gap score of plain Falconn). x - 0 == x, so both modes share
// every walk below.
__device__ __forceinline__ float pair_score(float a, float b, float off) { return (a + b) - off; }

// Offset of table t: 0, or its best pair under the gap score.
__device__ __forceinline__ float table_offset(const Lists& ls, int t, int l, bool gap) {
  if (!gap) return 0.0f;
  return l == 1 ? ls.get(t, 0) : ls.get(2 * t, 0) + ls.get(2 * t + 1, 0);
}

// min(cap, #pairs of table t with score >= tau); A = list 2t (or t for l = 1), B = list 2t + 1.
// The walk stops once `cap` pairs are counted, so its depth is bounded by cap.
// #positions p < lim of list `list` whose score reaches tau: a + list[p] - off for a pair row
// (a >= 0), list[p] - off alone for l = 1 (a < 0). The scores do not increase with p (the list is
// sorted and float addition is monotone), so a binary search finds the boundary; the last LDS
// position is tested first, so that a boundary inside the LDS prefix costs no device read.
__device__ __forceinline__ int count_prefix(const Lists& ls, int list, float a, float tau, float off,
                                            int lim) {
  auto reaches = [&](int p) {
    const float v = ls.get(list, p);
    return (a < 0.0f ? v - off : pair_score(a, v, off)) >= tau;
  };
  int lo = 0, hi = lim;   // reaches(p) for p < lo, not for p >= hi
  const int mp = ls.M < lim ? ls.M : lim;
  if (mp > 0) {
    if (reaches(mp - 1)) lo = mp;
    else hi = mp - 1;
  }
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (reaches(mid)) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ uint64_t count_table(const Lists& ls, int t, int l, float tau,
                                                uint64_t cap, float off) {
  const int D = ls.D;
  const int lim = cap < (uint64_t)D ? (int)cap : D;
  if (l == 1) return (uint64_t)count_prefix(ls, t, -1.0f, tau, off, lim);
  const int la = 2 * t, lb = 2 * t + 1;
  const float a0 = ls.get(la, 0);
  int j = count_prefix(ls, lb, a0, tau, off, lim);
  uint64_t c = 0;
  for (int i = 0; i < D && j > 0; ++i) {
    const float ai = ls.get(la, i);
    while (j > 0 && !(pair_score(ai, ls.get(lb, j - 1), off) >= tau)) --j;
    c += (uint64_t)j;
    if (c >= cap) return cap;
  }
  return c < cap ? c : cap;
}

__device__ __forceinline__ uint64_t block_sum_u64(uint64_t v, uint64_t* red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += xor_lanes_n(v, o);
  if (lane == 0) red[w] = v;
  __syncthreads();
  uint64_t t = 0;
#pragma unroll
  for (int i = 0; i < kProbeWaves; ++i) t += red[i];
  __syncthreads();
  return t;
}

__device__ __forceinline__ float block_max(float v, float* red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, xor_lanes_n(v, o));
  if (lane == 0) red[w] = v;
  __syncthreads();
  float t = red[0];
#pragma unroll
  for (int i = 1; i < kProbeWaves; ++i) t = fmaxf(t, red[i]);
  __syncthreads();
  return t;
}

// Exclusive scan over the block (thread order); returns the prefix and the block total.
__device__ __forceinline__ uint64_t block_scan_u64(uint64_t v, uint64_t& total, uint64_t* red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint64_t inc = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t t = __shfl_up(inc, o);
    if (lane >= o) inc += t;
  }
  if (lane == 63) red[w] = inc;
  __syncthreads();
  uint64_t before = 0;
  total = 0;
#pragma unroll
  for (int i = 0; i < kProbeWaves; ++i) {
    if (i < w) before += red[i];
    total += red[i];
  }
  __syncthreads();
  return before + inc - v;
}

// Emits the candidates of one table for the sparse selection: pairs (i, j) with score >= tau and
// (i + 1)(j + 1) <= qP, from the table's staged list prefixes A and B (positions < lim =
// min(qP, D)). Each goes to the next free slot of `key` (while slots remain; `count` keeps
// counting) as order-preserving score bits << 32 | ~(t * R + i * D + j), R = D^l, so that a larger
// key ranks first in (score desc, table asc, i asc, j asc) order.
__device__ __forceinline__ void emit_region(const float* A, const float* B, int l, int D, int lim,
                                            uint32_t qP, float tau, bool gap, uint32_t pos0,
                                            uint64_t* key, uint32_t* count) {
  if (l == 1) {
    const float off = gap ? A[0] : 0.0f;
    for (int c = 0; c < lim; ++c) {
      const float sc = A[c] - off;
      if (!(sc >= tau)) break;
      const uint32_t p = atomicAdd(count, 1u);
      if (p < (uint32_t)kDirectCap) key[p] = ((uint64_t)ord_of(sc) << 32) | (uint32_t)~(pos0 + (uint32_t)c);
    }
    return;
  }
  const float off = gap ? A[0] + B[0] : 0.0f;
  const float a0 = A[0];
  int j = 0;
  while (j < lim && pair_score(a0, B[j], off) >= tau) ++j;
  for (int i = 0; i < lim && j > 0; ++i) {
    const float ai = A[i];
    while (j > 0 && !(pair_score(ai, B[j - 1], off) >= tau)) --j;
    const int r = (int)(qP / (uint32_t)(i + 1));
    const int n = j < r ? j : r;
    for (int jj = 0; jj < n; ++jj) {
      const uint32_t p = atomicAdd(count, 1u);
      if (p < (uint32_t)kDirectCap)
        key[p] = ((uint64_t)ord_of(pair_score(ai, B[jj], off)) << 32) |
                 (uint32_t)~(pos0 + (uint32_t)i * (uint32_t)D + (uint32_t)jj);
    }
  }
}

// Descending bitonic sort of n keys in LDS (n a power of two, at most 2 * kProbeThreads).
__device__ __forceinline__ void probe_sort_desc(uint64_t* key, int n) {
  for (int k = 2; k <= n; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < n; i += kProbeThreads) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const uint64_t a = key[i], b = key[ixj];
          if ((i & k) == 0 ? (a < b) : (a > b)) {
            key[i] = b;
            key[ixj] = a;
          }
        }
      }
      __syncthreads();
    }
}

constexpr size_t sparse_lds_bytes(int L) {
  return 64 + (size_t)kDirectCap * 8 + (size_t)kDeepFloats * 4 + (size_t)L * 8 + 8;
}
static_assert((64 + kDirectCap * 8) % 16 == 0, "staged lists must be 16-byte aligned");

// Sparse selection, one workgroup per query with 4 qP <= L (others get nprobe = -1, as do queries
// it cannot finish). The qP-th best of the tables' best pairs is a lower bound mn of the qP-th
// best pair (the qP tables ranked at or above it each hold a pair scoring at least that). Only
// tables whose best pair reaches mn can hold a selected pair, and only at positions with
// (i + 1)(j + 1) <= qP, so those tables' first min(qP, D) list entries (rounded up to 4; D is a
// multiple of 4) are staged in LDS a chunk of tables at a time and every pair of the region
// scoring >= mn becomes a candidate. Sorted by key, the first qP candidates are the probes, in
// rank order; only they read their bucket codes. Past kDirectCap candidates the query is left to
// the bisection.
__global__ __launch_bounds__(kProbeThreads) void probe_sparse_kernel(
    const float* __restrict__ la, const uint16_t* __restrict__ lc, int64_t m, int L, int l, int D,
    int64_t NB, const int32_t* __restrict__ qp_arr, int32_t qp_uniform, int32_t qcap, int gap_score,
    uint32_t* __restrict__ probes, int32_t* __restrict__ nprobe) {
  extern __shared__ __align__(16) unsigned char smem[];   // sparse_lds_bytes(L)
  uint64_t* red = reinterpret_cast<uint64_t*>(smem);        // kProbeWaves words
  uint64_t* dkey = reinterpret_cast<uint64_t*>(smem + 64);  // [kDirectCap] candidate keys
  float* deep = reinterpret_cast<float*>(dkey + kDirectCap);   // [kDeepFloats] staged lists
  float* tops = deep + kDeepFloats;                         // [L] best pair of every table
  int32_t* act = reinterpret_cast<int32_t*>(tops + L);      // [L] tables reaching mn
  float& sel = *reinterpret_cast<float*>(act + L);
  uint32_t& count = *reinterpret_cast<uint32_t*>(act + L + 1);
  const int64_t q = blockIdx.x;
  if (q >= m) return;   // uniform
  const int tid = threadIdx.x;
  const int LF = L * l;
  const float* Aq = la + (size_t)q * LF * D;
  const uint16_t* Cq = lc + (size_t)q * LF * D;
  const bool gap = gap_score != 0;
  const uint64_t total = (uint64_t)L * (l == 1 ? (uint64_t)D : (uint64_t)D * D);
  const int64_t want = qp_arr ? qp_arr[q] : qp_uniform;
  uint64_t qP = want < 1 ? 0 : ((uint64_t)want < total ? (uint64_t)want : total);
  if (qP > (uint64_t)qcap) qP = (uint64_t)qcap;
  const int lim = qP < (uint64_t)D ? (int)qP : D;        // positions a candidate can occupy
  const int lim4 = (lim + 3) / 4;
  const int per4 = l * lim4;                              // staged float4 per table
  const uint32_t R = l == 1 ? (uint32_t)D : (uint32_t)D * (uint32_t)D;
  if (qP == 0 || 4 * qP > (uint64_t)L || L > kRankTables || D % 4 != 0 || per4 * 4 > kDeepFloats ||
      (uint64_t)L * R > 0xffffffffull) {
    if (tid == 0) nprobe[q] = -1;
    return;
  }

  // every table's best pair (position 0 of its lists)
  for (int t = tid; t < L; t += kProbeThreads) {
    float top;
    if (l == 1) {
      const float a0 = Aq[(size_t)t * D];
      top = a0 - (gap ? a0 : 0.0f);
    } else {
      const float a0 = Aq[(size_t)(2 * t) * D], b0 = Aq[(size_t)(2 * t + 1) * D];
      top = pair_score(a0, b0, gap ? a0 + b0 : 0.0f);
    }
    tops[t] = top;
  }
  if (tid == 0) count = 0u;
  __syncthreads();
  // mn: the best pair of the table of rank qP - 1 in (best pair desc, table asc) order
  for (int t = tid; t < L; t += kProbeThreads) {
    const float v = tops[t];
    int r = 0;
    for (int u = 0; u < L; ++u) {
      const float w = tops[u];
      r += (w > v || (w == v && u < t)) ? 1 : 0;
    }
    if ((uint64_t)r == qP - 1) sel = v;
  }
  __syncthreads();
  const float mn = sel;
  // tables whose best pair reaches mn, in table order
  int A = 0;
  for (int t0 = 0; t0 < L; t0 += kProbeThreads) {
    const int t = t0 + tid;
    const uint64_t f = (t < L && tops[t] >= mn) ? 1u : 0u;
    uint64_t tot;
    const uint64_t p = block_scan_u64(f, tot, red);
    if (f) act[A + (int)p] = t;
    A += (int)tot;
  }
  __syncthreads();
  const int CH = kDeepFloats / (per4 * 4);                // tables per staged chunk
  float4* deep4 = reinterpret_cast<float4*>(deep);
  for (int k0 = 0; k0 < A; k0 += CH) {
    const int nk = A - k0 < CH ? A - k0 : CH;
    const int n4 = nk * per4;
    for (int x0 = 0; x0 < n4; x0 += 8 * kProbeThreads) {
      // eight loads in flight per thread (indices past the chunk reload its last entry, so the
      // loads need no branch and stay in registers)
      float4 v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        int x = x0 + u * kProbeThreads + tid;
        x = x < n4 ? x : n4 - 1;
        const int k = x / per4, r = x - k * per4;
        const int f = r / lim4, e4 = r - f * lim4;
        const int t = act[k0 + k];
        v[u] = *reinterpret_cast<const float4*>(Aq + (size_t)(l == 2 ? 2 * t + f : t) * D + 4 * e4);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int x = x0 + u * kProbeThreads + tid;
        if (x < n4) deep4[x] = v[u];
      }
    }
    __syncthreads();
    for (int k = tid; k < nk; k += kProbeThreads) {
      const int t = act[k0 + k];
      const float* Ak = deep + k * per4 * 4;
      emit_region(Ak, Ak + lim4 * 4, l, D, lim, (uint32_t)qP, mn, gap, (uint32_t)t * R, dkey, &count);
    }
    __syncthreads();
  }
  const uint32_t C = count;
  if (C > (uint32_t)kDirectCap) {
    if (tid == 0) nprobe[q] = -1;
    return;
  }
  int n = 2;
  while ((uint32_t)n < C) n <<= 1;
  for (int c = (int)C + tid; c < n; c += kProbeThreads) dkey[c] = 0ull;
  __syncthreads();
  probe_sort_desc(dkey, n);
  uint32_t* out = probes + (size_t)q * qcap;
  const int64_t stride = NB + 1;
  for (int r = tid; (uint64_t)r < qP; r += kProbeThreads) {
    const uint32_t pos = ~(uint32_t)dkey[r];
    const uint32_t t = pos / R, rem = pos - t * R;
    const uint32_t tbase = (uint32_t)((int64_t)t * stride);
    if (l == 1) {
      out[r] = tbase + Cq[(size_t)t * D + rem];
    } else {
      const uint32_t i = rem / (uint32_t)D, j = rem - i * (uint32_t)D;
      out[r] = tbase + (uint32_t)Cq[(size_t)(2 * t) * D + i] * (uint32_t)(2 * D) +
               Cq[(size_t)(2 * t + 1) * D + j];
    }
  }
  if (tid == 0) nprobe[q] = (int32_t)qP;
}

// One workgroup per query; thread x walks tables x, x + 128, ... With `skip_done`, queries whose
// nprobe the sparse selection has already set (>= 0) are skipped.
__global__ __launch_bounds__(kProbeThreads) void probe_kernel(
    const float* __restrict__ la, const uint16_t* __restrict__ lc, int64_t m, int L, int l, int D,
    int M, int64_t NB, const int32_t* __restrict__ qp_arr, int32_t qp_uniform, int32_t qcap,
    int gap_score, int skip_done, uint32_t* __restrict__ probes, int32_t* __restrict__ nprobe) {
  extern __shared__ __align__(16) unsigned char smem[];
  uint64_t* red = reinterpret_cast<uint64_t*>(smem);        // kProbeWaves words
  float* pre = reinterpret_cast<float*>(smem + 64);         // [l][L][M + 1] list prefixes
  const int64_t q = blockIdx.x;
  if (q >= m) return;   // uniform
  if (skip_done && nprobe[q] >= 0) return;
  const int tid = threadIdx.x;
  const int LF = L * l;
  const float* Aq = la + (size_t)q * LF * D;
  const uint16_t* Cq = lc + (size_t)q * LF * D;
  float* tops = pre + (size_t)l * L * (M + 1);             // [L] best pair of every table
  float* sel = tops + L;                                    // one value
  float* heads = sel + 1;   // [3L] pairs (0,0), (0,1), (1,0); allocated when qcap <= 3L, l = 2
  if (M % 4 == 0) {
    // 16-byte loads, eight per thread in flight before their LDS stores
    const int per = M / 4, total4 = LF * per;
    for (int b = tid; b < total4; b += 8 * kProbeThreads) {
      float4 r[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i = b + u * kProbeThreads;
        if (i < total4) {
          const int list = i / per, e4 = i - list * per;
          r[u] = *reinterpret_cast<const float4*>(Aq + (size_t)list * D + 4 * e4);
        }
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i = b + u * kProbeThreads;
        if (i < total4) {
          const int list = i / per, e4 = i - list * per;
          const int t = l == 2 ? list >> 1 : list, f = l == 2 ? list & 1 : 0;
          float* row = pre + (f * L + t) * (M + 1) + 4 * e4;
          row[0] = r[u].x;
          row[1] = r[u].y;
          row[2] = r[u].z;
          row[3] = r[u].w;
        }
      }
    }
  } else {
    for (int i = tid; i < LF * M; i += kProbeThreads) {
      const int list = i / M, e = i - list * M;
      const int t = l == 2 ? list >> 1 : list, f = l == 2 ? list & 1 : 0;
      pre[(f * L + t) * (M + 1) + e] = Aq[(size_t)list * D + e];
    }
  }
  __syncthreads();
  const Lists ls{pre, Aq, M, D, L, l};

  const uint64_t total = (uint64_t)L * (l == 1 ? (uint64_t)D : (uint64_t)D * D);
  const int64_t want = qp_arr ? qp_arr[q] : qp_uniform;
  uint64_t qP = want < 1 ? 0 : ((uint64_t)want < total ? (uint64_t)want : total);
  if (qP > (uint64_t)qcap) qP = (uint64_t)qcap;
  if (qP == 0) {
    if (tid == 0) nprobe[q] = 0;
    return;
  }
  // Bracket. hi: just above the best pair of all tables (no pair reaches it). lo: with
  // c = ceil(qP / L), every table has at least c pairs scoring >= its bound (row 0 for c <= D,
  // else the first ceil(c / D) full rows), so the minimum bound over tables counts >= L c >= qP.
  const uint64_t cpt = (qP + L - 1) / L;
  const bool gap = gap_score != 0;
  float mx = -INFINITY, mn = INFINITY;
  for (int t = tid; t < L; t += kProbeThreads) {
    float top, bound;
    const float off = table_offset(ls, t, l, gap);
    if (l == 1) {
      top = ls.get(t, 0) - off;
      bound = cpt <= (uint64_t)D ? ls.get(t, (int)cpt - 1) - off : -INFINITY;
    } else {
      top = pair_score(ls.get(2 * t, 0), ls.get(2 * t + 1, 0), off);
      if (cpt <= (uint64_t)D) {
        bound = pair_score(ls.get(2 * t, 0), ls.get(2 * t + 1, (int)cpt - 1), off);
      } else {
        const uint64_t rows = (cpt + D - 1) / D;
        bound = rows <= (uint64_t)D ? pair_score(ls.get(2 * t, (int)rows - 1), ls.get(2 * t + 1, D - 1), off)
                                    : -INFINITY;
      }
    }
    mx = fmaxf(mx, top);
    mn = fminf(mn, bound);
    tops[t] = top;
  }
  mx = block_max(mx, reinterpret_cast<float*>(red));      // (its barriers publish `tops`)
  mn = -block_max(-mn, reinterpret_cast<float*>(red));
  if (qP <= (uint64_t)L && L <= kRankTables) {
    // A tighter lo: the table of rank qP - 1 in (best pair desc, table asc) order. The qP tables
    // ranked before or at it each hold a pair scoring >= its best pair, so cnt(lo) >= qP.
    for (int t = tid; t < L; t += kProbeThreads) {
      const float v = tops[t];
      int r = 0;
#pragma unroll 4
      for (int u = 0; u < L; ++u) {
        const float w = tops[u];
        r += (w > v || (w == v && u < t)) ? 1 : 0;
      }
      if ((uint64_t)r == qP - 1) *sel = v;
    }
    __syncthreads();
    mn = fmaxf(mn, *sel);
  } else if (!gap && l == 2 && D >= 2 && (uint64_t)qcap <= 3 * (uint64_t)L && L <= kRankTables) {
    // A tighter lo for up to three probes per table: the pairs at list positions (0, 0), (0, 1)
    // and (1, 0) of every table are 3L distinct pairs with known scores, so the qP-th largest of
    // them is reached by at least qP pairs: cnt(lo) >= qP.
    const int H = 3 * L;
    for (int t = tid; t < L; t += kProbeThreads) {
      const float a0 = ls.get(2 * t, 0), a1 = ls.get(2 * t, 1);
      const float b0 = ls.get(2 * t + 1, 0), b1 = ls.get(2 * t + 1, 1);
      heads[3 * t] = a0 + b0;
      heads[3 * t + 1] = a0 + b1;
      heads[3 * t + 2] = a1 + b0;
    }
    __syncthreads();
    for (int c = tid; c < H; c += kProbeThreads) {
      const float v = heads[c];
      int r = 0;
#pragma unroll 4
      for (int u = 0; u < H; ++u) {
        const float w = heads[u];
        r += (w > v || (w == v && u < c)) ? 1 : 0;
      }
      if ((uint64_t)r == qP - 1) *sel = v;
    }
    __syncthreads();
    mn = fmaxf(mn, *sel);
  }

  // Counts are capped at qP + 1 per table: a capped sum is >= qP exactly when the true sum is,
  // and equals qP only when no table was capped, so every decision below is the uncapped one.
  const uint64_t cap = qP + 1;
  uint32_t lo = ord_of(mn), hi = ord_of(mx) + 1u;   // cnt(lo) >= qP > cnt(hi), in key order
  // The next key comes from the secant through (lo, c_lo) and (hi, c_hi) once c_lo is known,
  // kept at least 1/16 of the bracket from either end; a secant step that does not halve the
  // bracket is followed by a bisection step, so the search takes at most twice the bisection's
  // steps. Any key inside the bracket keeps the invariant, so the result does not depend on
  // these choices.
  uint64_t c_hi = 0, c_lo = 0;
  bool exact = false, bisect = true;
  while (hi - lo > 1u) {
    const uint32_t span = hi - lo;
    uint32_t mid = lo + span / 2u;
    const bool secant = !bisect && c_lo > qP;
    if (secant) {
      const float f = (float)(c_lo - qP) / (float)(c_lo - c_hi);
      const uint32_t g = span / 16u > 1u ? span / 16u : 1u;
      const float o = f * (float)span;
      uint32_t off = o < (float)g ? g : (o > (float)(span - g) ? span - g : (uint32_t)o);
      if (off < 1u) off = 1u;
      if (off > span - 1u) off = span - 1u;
      mid = lo + off;
    }
    const float tau = of_ord(mid);
    uint64_t c = 0;
    for (int t = tid; t < L; t += kProbeThreads) c += count_table(ls, t, l, tau, cap, table_offset(ls, t, l, gap));
    c = block_sum_u64(c, red);
    if (c == qP) {
      lo = mid;
      exact = true;
      break;
    }
    if (c > qP) {
      lo = mid;
      c_lo = c;
    } else {
      hi = mid;
      c_hi = c;
    }
    bisect = secant && hi - lo > span / 2u;
  }
  const float thr_gt = of_ord(exact ? lo : hi);
  const float tau_eq = of_ord(lo);
  const uint64_t c_gt = exact ? qP : c_hi;
  const uint64_t need = qP - c_gt;
  uint32_t* out = probes + (size_t)q * qcap;
  const int64_t stride = NB + 1;
  const int twoD = 2 * D;

  uint64_t run_gt = 0, run_eq = 0;
  for (int tb = 0; tb < L; tb += kProbeThreads) {
    const int t = tb + tid;
    uint64_t n_gt = 0, n_eq = 0;
    const float off = t < L ? table_offset(ls, t, l, gap) : 0.0f;
    if (t < L) {
      // every table holds at most c_gt <= qP pairs above thr_gt; ties are only needed up to `need`
      n_gt = count_table(ls, t, l, thr_gt, cap, off);
      if (need) n_eq = count_table(ls, t, l, tau_eq, n_gt + need, off) - n_gt;
    }
    uint64_t tot_gt, tot_eq;
    const uint64_t pos_gt0 = run_gt + block_scan_u64(n_gt, tot_gt, red);
    const uint64_t tie0 = run_eq + block_scan_u64(n_eq, tot_eq, red);
    run_gt += tot_gt;
    run_eq += tot_eq;
    if (t >= L) continue;
    const uint32_t tbase = (uint32_t)((int64_t)t * stride);
    uint64_t pg = pos_gt0, te = tie0;
    if (l == 1) {
      const uint16_t* C1 = Cq + (size_t)t * D;
      for (uint64_t i = 0; i < n_gt; ++i) out[pg++] = tbase + C1[i];
      for (uint64_t i = n_gt; i < n_gt + n_eq && te < need; ++i, ++te) out[c_gt + te] = tbase + C1[i];
      continue;
    }
    const uint16_t* C1 = Cq + (size_t)(2 * t) * D;
    const uint16_t* C2 = C1 + D;
    const int la_ = 2 * t, lb_ = 2 * t + 1;
    // row 0's counts, searched within the qP + 1 positions a selected pair can reach (a larger
    // count changes no emission, since at most qP pairs are emitted)
    const int lim_e = qP + 1 < (uint64_t)D ? (int)qP + 1 : D;
    const float a0 = ls.get(la_, 0);
    int jg = count_prefix(ls, lb_, a0, thr_gt, off, lim_e), je = 0;
    if (need) je = count_prefix(ls, lb_, a0, tau_eq, off, lim_e);
    for (int i = 0; i < D && (jg > 0 || (je > 0 && te < need)); ++i) {
      const float ai = ls.get(la_, i);
      while (jg > 0 && !(pair_score(ai, ls.get(lb_, jg - 1), off) >= thr_gt)) --jg;
      if (need)
        while (je > 0 && !(pair_score(ai, ls.get(lb_, je - 1), off) >= tau_eq)) --je;
      const uint32_t rowb = tbase + (uint32_t)C1[i] * twoD;
      for (int j = 0; j < jg; ++j) out[pg++] = rowb + C2[j];
      for (int j = jg; j < je && te < need; ++j, ++te) out[c_gt + te] = rowb + C2[j];
    }
  }
  if (tid == 0) nprobe[q] = (int32_t)qP;
}

}  // namespace

// LDS floats of the probe kernel besides the list prefixes: the tables' best pairs, one value,
// and the 3L leading pairs when the search bracket uses them (l = 2, qcap <= 3L)
static int64_t probe_extra_floats(const fpp_index* ix, int32_t qcap) {
  const bool heads = ix->l == 2 && (int64_t)qcap <= 3LL * ix->L;
  return (int64_t)ix->L + 1 + (heads ? 3LL * ix->L : 0);
}

// Prefix length of each sorted list staged in LDS: enough for about twice the average number of
// probes per table, at most D and at most 30 KB of LDS per query. Small prefixes keep many
// queries resident per CU, which hides the latency of the walks; entries past the prefix come
// from device memory. (At n = 10M, L = 64, D = 256 and 6,400 probes, 32-entry prefixes take
// 69 ms per 100,000 queries, 64-entry ones 119 ms and 128-entry ones 217 ms.)
int probe_prefix(const fpp_index* ix, int32_t qcap) {
  const int64_t LF = (int64_t)ix->L * ix->l;
  int want = 16;
  const int64_t per_t = (2LL * qcap + ix->L - 1) / ix->L;
  while (want < per_t && want < ix->D) want <<= 1;
  if (want > ix->D) want = ix->D;
  while (want > 1 && (LF * (want + 1) + probe_extra_floats(ix, qcap)) * 4 > 30 * 1024) want >>= 1;
  return want;
}

// List entries the selection can need: every selected pair (i, j) of a query with qP <= qcap
// probes has (i + 1)(j + 1) <= qP, and the count walks read positions <= qP only (they stop at a
// count of qP + 1). The emission walk reads further only once the table has nothing left to
// emit, where the values it reads decide nothing. Positions [0, qcap + 2) and the LDS prefix are
// therefore enough.
int probe_list_len(const fpp_index* ix, int32_t qcap) {
  const int64_t w = std::max<int64_t>((int64_t)qcap + 2, probe_prefix(ix, qcap));
  return (int)std::min<int64_t>(w, ix->D);
}

hipError_t launch_probe_select(const fpp_index* ix, const float* la, const uint16_t* lc, int64_t m,
                               const int32_t* qp_arr, int32_t qp_uniform, int32_t qcap,
                               int32_t probe_score, uint32_t* probes, int32_t* nprobe, hipStream_t s,
                               bool only_unfinished) {
  if (m <= 0) return hipSuccess;
  const int M = probe_prefix(ix, qcap);
  const size_t lds = 64 + ((size_t)ix->L * ix->l * (M + 1) + probe_extra_floats(ix, qcap)) * 4;
  if (lds > 64 * 1024) {   // at most 131 KB (L = 4096, l = 2, M = 1), within the 160 KB of a CU
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(probe_kernel),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  // the sparse selection first, where some query may qualify (4 qP <= L); the bisection then
  // takes the queries it left (nprobe = -1)
  const bool sparse = !only_unfinished && ix->L <= kRankTables && ix->D % 4 == 0 &&
                      (qp_arr != nullptr || 4 * (int64_t)std::min(qp_uniform, qcap) <= ix->L);
  if (sparse)
    hipLaunchKernelGGL(probe_sparse_kernel, dim3((unsigned)m), dim3(kProbeThreads),
                       sparse_lds_bytes(ix->L), s, la, lc, m,
                       ix->L, ix->l, ix->D, ix->NB, qp_arr, qp_uniform, qcap, probe_score, probes,
                       nprobe);
  hipLaunchKernelGGL(probe_kernel, dim3((unsigned)m), dim3(kProbeThreads), lds, s, la, lc, m, ix->L,
                     ix->l, ix->D, M, ix->NB, qp_arr, qp_uniform, qcap, probe_score,
                     (sparse || only_unfinished) ? 1 : 0,
                     probes, nprobe);
  return hipGetLastError();
}

}  // namespace fpp
