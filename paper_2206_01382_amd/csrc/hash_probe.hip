// Query hashing and probe selection in one kernel, for probe budgets of up to about two probes per
// table and D = P <= 256 or D = P / 2 <= 256 (Section 3.4, multi-probing for querying; Section 2.2
// Eq. 1 for the hash; qProbes is a total over the L tables).
//
// The selection needs the qProbes best (table, bucket) pairs of a query by the pair score
// s = fl32(|y1_a| + |y2_b|) (l = 2; s = |y_a| for l = 1), in the order (s desc, table asc,
// position in list 1 asc, position in list 2 asc). Sorting every function's D outputs, as the
// list-based path does, is most of the work of hashing. Here one workgroup owns one query:
//   1. it rotates all L * l functions and records each function's best and second-best |y|,
//      and its best output, in LDS;
//   2. every table holds the pairs at positions (0, 0), (0, 1) and (1, 0) (l = 1: positions 0
//      and 1) with scores known from those two values, so the qProbes-th best of these 3L
//      scores, mn, is a lower bound of the qProbes-th best pair overall;
//   3. an output y_a of function f can only be in a pair scoring >= mn if fl32(|y_a| + M) >= mn,
//      with M the best |y| of the table's other function (float addition is monotone), so only
//      tables whose best pair reaches mn matter (about a third of them at one probe per two
//      tables). Of their functions, one whose second-best |y| fails that test contributes only its
//      best output, recorded in pass 1 (about two thirds of them); the others are rotated again
//      (the same expression tree, so the same values) and only the outputs passing that test are
//      written to LDS. Every output ranking above an
//      emitted one in its list is emitted too, so an output's position in its list is its rank
//      among the emitted outputs of its function;
//   4. the emitted outputs of each table are paired, pairs scoring >= mn are ranked by the full
//      order above, and the first qProbes are the probes.
// A query whose emitted outputs or candidate pairs exceed the LDS capacity gets nprobe = -1 and
// is finished by the list-based kernels (which skip every query that already has its probes).
#include "fpp_internal.hpp"
#include "lanes.hpp"
#include "rotation.hpp"
#include "wave_sort.hpp"

namespace fpp {
namespace {

constexpr int kEntCap = 1024;    // emitted outputs per query
constexpr int kPairCap = 1024;   // candidate pairs per query
constexpr int kMaxTables = 256;  // tables of an index on this path (3L scores are ranked)

__device__ __forceinline__ uint32_t ord_f(float f) {
  const uint32_t b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// An emitted output: function (16 bits) << 48 | index j (16 bits) << 32 | float bits of y.
__device__ __forceinline__ uint64_t pack_entry(int f, int j, float y) {
  return ((uint64_t)(uint32_t)f << 48) | ((uint64_t)(uint32_t)j << 32) | __float_as_uint(y);
}
__device__ __forceinline__ int entry_f(uint64_t e) { return (int)(e >> 48); }
__device__ __forceinline__ int entry_j(uint64_t e) { return (int)((e >> 32) & 0xffffu); }
__device__ __forceinline__ float entry_y(uint64_t e) { return __uint_as_float((uint32_t)e); }

struct HPState {
  uint32_t ecount, pcount;
  float mn;
  uint32_t nact;
};

// LDS carve-up for LF functions and L tables (byte offsets, 8-byte aligned arrays first).
struct HPLayout {
  size_t ent, grp, pkey, pval, rk, M1, M2, cnt, start, tops, act, by, bj, state, total;
  __host__ __device__ HPLayout(int LF, int L, int l) {
    size_t o = 0;
    ent = o;   o += (size_t)kEntCap * 8;
    grp = o;   o += (size_t)kEntCap * 8;
    pkey = o;  o += (size_t)kPairCap * 8;
    state = o; o += sizeof(HPState);
    pval = o;  o += (size_t)kPairCap * 4;
    M1 = o;    o += (size_t)LF * 4;
    M2 = o;    o += (size_t)LF * 4;
    cnt = o;   o += (size_t)LF * 4;
    start = o; o += (size_t)(LF + 1) * 4;
    tops = o;  o += (size_t)(l == 2 ? 3 : 2) * L * 4;
    act = o;   o += (size_t)LF * 4;
    by = o;    o += (size_t)LF * 4;
    bj = o;    o += (size_t)LF * 4;
    rk = o;    o += (size_t)kEntCap * 2;
    total = (o + 15) / 16 * 16;
  }
};

// Called by one whole wavefront: *out = the q-th largest of the n <= 64 E non-negative values
// v[0 .. n) (sorted in registers, E per lane).
template <int E>
__device__ __forceinline__ void qth_largest(const float* v, int n, int q, float* out) {
  const int lane = threadIdx.x & 63;
  uint32_t key[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int i = lane * E + e;
    key[e] = i < n ? __float_as_uint(v[i]) : 0u;
  }
  sort32_desc<64 * E, E, 64>(key, lane, lane * E, 64 * E);
#pragma unroll
  for (int e = 0; e < E; ++e)
    if (lane * E + e == q - 1) *out = __uint_as_float(key[e]);
}

// One workgroup per query; its threads take the functions in passes of IPB = blockDim.x / LPI
// (function base + thread / LPI).
// HALF: D = P / 2 (the listed outputs are j < D, held by the lower half of an item's lanes), else
// D = P.
template <int P, bool VEC, bool HALF>
__global__ __launch_bounds__(512) void hash_probe_kernel(
    const float* __restrict__ V, int64_t m, int ldv, int d, const uint32_t* __restrict__ sign_bits,
    int L, int l, int64_t NB, const int32_t* __restrict__ qp_arr, int32_t qp_uniform, int32_t qcap,
    uint32_t* __restrict__ probes, int32_t* __restrict__ nprobe) {
  constexpr int E = QLayout<P>::E, LPI = QLayout<P>::LPI;
  constexpr int D = HALF ? P / 2 : P;
  const int64_t q = blockIdx.x;
  if (q >= m) return;   // uniform
  const int LF = L * l;
  const int tid = threadIdx.x, bs = blockDim.x;
  const int g = tid / LPI, li = tid % LPI, j0 = li * E;
  const int IPB = bs / LPI;
  extern __shared__ __align__(16) unsigned char smem[];
  const HPLayout lo(LF, L, l);
  uint64_t* ent = reinterpret_cast<uint64_t*>(smem + lo.ent);
  uint64_t* grp = reinterpret_cast<uint64_t*>(smem + lo.grp);
  uint64_t* pkey = reinterpret_cast<uint64_t*>(smem + lo.pkey);
  HPState* st = reinterpret_cast<HPState*>(smem + lo.state);
  uint32_t* pval = reinterpret_cast<uint32_t*>(smem + lo.pval);
  float* M1 = reinterpret_cast<float*>(smem + lo.M1);
  float* M2 = reinterpret_cast<float*>(smem + lo.M2);
  uint32_t* cnt = reinterpret_cast<uint32_t*>(smem + lo.cnt);
  uint32_t* start = reinterpret_cast<uint32_t*>(smem + lo.start);
  float* tops = reinterpret_cast<float*>(smem + lo.tops);
  uint16_t* rk = reinterpret_cast<uint16_t*>(smem + lo.rk);
  int32_t* act = reinterpret_cast<int32_t*>(smem + lo.act);
  float* BY = reinterpret_cast<float*>(smem + lo.by);      // each function's best output y
  int32_t* BJ = reinterpret_cast<int32_t*>(smem + lo.bj);  // and its index
  const float* row = V + (size_t)q * ldv;

  // the lane's elements of the query, loaded once for both passes
  float xq[E];
  load_elems<E, VEC>(row, d, j0, xq);

  // ---- 1. rotations; each function's best and second-best |y|, and its best output (the
  // first in list order: largest |y|, then smallest index)
  for (int base = 0; base < LF; base += IPB) {
    const int item = base + g;
    const bool valid = item < LF;   // uniform over the item's lanes
    float v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = xq[e];
    uint32_t sw[3];
    load_sign_bits<P, E>(sign_bits, valid ? item : 0, j0, sw);
    rotate_item_bits<P>(v, sw, li);
    float m1 = -1.0f, m2 = -1.0f;   // below every |y|
    float by = 0.0f;
    int bj = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const float a = (!HALF || j0 + e < D) ? fabsf(v[e]) : -1.0f;   // listed outputs only
      m2 = __builtin_amdgcn_fmed3f(m1, m2, a);   // m1 >= m2: the new second best
      const bool gt = a > m1;                    // strictly: the smaller index keeps a tie
      by = gt ? v[e] : by;
      bj = gt ? j0 + e : bj;
      m1 = fmaxf(m1, a);
    }
#pragma unroll
    for (int o = 1; o < LPI; o <<= 1) {
      const float p1 = xor_lanes_n(m1, o), p2 = xor_lanes_n(m2, o);
      const float pby = xor_lanes_n(by, o);
      const int pbj = xor_lanes_n(bj, o);
      m2 = fmaxf(fminf(m1, p1), fmaxf(m2, p2));
      const bool take = p1 > m1 || (p1 == m1 && pbj < bj);
      by = take ? pby : by;
      bj = take ? pbj : bj;
      m1 = fmaxf(m1, p1);
    }
    if (valid && li == 0) {
      M1[item] = m1;
      M2[item] = m2;
      BY[item] = by;
      BJ[item] = bj;
    }
  }
  for (int i = tid; i < LF; i += bs) cnt[i] = 0u;
  if (tid == 0) {
    st->ecount = 0u;
    st->pcount = 0u;
    st->nact = 0u;
  }
  __syncthreads();

  // ---- 2. the lower bound mn
  const int64_t want = qp_arr ? qp_arr[q] : qp_uniform;
  const int per = l == 2 ? 3 : 2;
  const int NT = per * L;
  int qP = want < 1 ? 0 : (want < (int64_t)NT ? (int)want : NT);
  if (qP > qcap) qP = qcap;
  for (int t = tid; t < L; t += bs) {
    if (l == 2) {
      const float a1 = M1[2 * t], a2 = M2[2 * t], b1 = M1[2 * t + 1], b2 = M2[2 * t + 1];
      tops[3 * t] = a1 + b1;       // positions (0, 0)
      tops[3 * t + 1] = a1 + b2;   // (0, 1)
      tops[3 * t + 2] = a2 + b1;   // (1, 0)
    } else {
      tops[2 * t] = M1[t];
      tops[2 * t + 1] = M2[t];
    }
  }
  __syncthreads();
  if (qP == 0 || want > (int64_t)NT) {
    // outside this path's range (a larger budget): the list-based kernels take the query
    if (tid == 0) nprobe[q] = qP == 0 ? 0 : -1;
    return;
  }
  // the qP-th largest of the NT scores: the first wavefront sorts them (non-negative floats
  // order like their bit patterns; padding is 0)
  if (tid < 64) {
    if (NT <= 512) qth_largest<8>(tops, NT, qP, &st->mn);
    else qth_largest<16>(tops, NT, qP, &st->mn);
  }
  __syncthreads();
  const float mn = st->mn;

  // ---- 3. the functions of the tables whose best pair reaches mn: a function whose second-best
  // output cannot reach mn (with the other function's best) contributes only its best output,
  // known from pass 1; the others are rotated again and emit every output that can reach mn
  for (int t = tid; t < L; t += bs) {
    if (tops[(l == 2 ? 3 : 2) * t] >= mn) {
      for (int f = 0; f < l; ++f) {
        const int item = l * t + f;
        const float mo = l == 2 ? M1[item ^ 1] : 0.0f;
        const float s2 = l == 2 ? M2[item] + mo : M2[item];
        if (s2 >= mn) {
          act[atomicAdd(&st->nact, 1u)] = item;
        } else {
          const uint32_t x = atomicAdd(&st->ecount, 1u);
          if (x < (uint32_t)kEntCap) {
            ent[x] = pack_entry(item, BJ[item], BY[item]);
            atomicAdd(&cnt[item], 1u);
          }
        }
      }
    }
  }
  __syncthreads();
  const int nact = (int)st->nact;
  for (int base = 0; base < nact; base += IPB) {
    const int idx = base + g;
    const bool valid = idx < nact;
    const int item = valid ? act[idx] : 0;
    float v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = xq[e];
    uint32_t sw[3];
    load_sign_bits<P, E>(sign_bits, item, j0, sw);
    rotate_item_bits<P>(v, sw, li);
    if (valid) {
      const float mo = l == 2 ? M1[item ^ 1] : 0.0f;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const float a = fabsf(v[e]);
        const float s = l == 2 ? a + mo : a;
        if ((!HALF || j0 + e < D) && s >= mn) {
          const uint32_t x = atomicAdd(&st->ecount, 1u);
          if (x < (uint32_t)kEntCap) {
            ent[x] = pack_entry(item, j0 + e, v[e]);
            atomicAdd(&cnt[item], 1u);
          }
        }
      }
    }
  }
  __syncthreads();
  const uint32_t ne = st->ecount;
  bool fail = ne > (uint32_t)kEntCap;   // uniform
  uint32_t np = 0;
  if (!fail) {
    // group the emitted outputs by function: exclusive scan of the counts (one wavefront), then
    // a scatter through the counts reused as fill pointers
    if (tid < 64) {
      const int per_lane = (LF + 63) / 64;
      const int b = tid * per_lane;
      uint32_t s = 0;
      for (int i = b; i < b + per_lane && i < LF; ++i) s += cnt[i];
      uint32_t inc = s;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(inc, o);
        if (tid >= o) inc += t;
      }
      uint32_t run = inc - s;
      for (int i = b; i < b + per_lane && i < LF; ++i) {
        start[i] = run;
        run += cnt[i];
        cnt[i] = 0u;
      }
      if (tid == 63) start[LF] = inc;
    }
    __syncthreads();
    for (uint32_t i = tid; i < ne; i += bs) {
      const uint64_t e = ent[i];
      const int f = entry_f(e);
      grp[start[f] + atomicAdd(&cnt[f], 1u)] = e;
    }
    __syncthreads();
    // position of each emitted output in its list: (|y| desc, j asc) among its function's
    for (uint32_t i = tid; i < ne; i += bs) {
      const uint64_t e = grp[i];
      const int f = entry_f(e), j = entry_j(e);
      const float a = fabsf(entry_y(e));
      int r = 0;
      for (uint32_t u = start[f]; u < start[f + 1]; ++u) {
        const uint64_t o = grp[u];
        const float b = fabsf(entry_y(o));
        r += (b > a || (b == a && entry_j(o) < j)) ? 1 : 0;
      }
      rk[i] = (uint16_t)r;
    }
    __syncthreads();
    // candidate pairs scoring >= mn, keyed so that a larger key ranks first:
    // order-preserving score bits << 32 | ~(t * R + pos1 * D + pos2), R = D^l
    const uint32_t stride = (uint32_t)(NB + 1);
    for (uint32_t i = tid; i < ne; i += bs) {
      const uint64_t e = grp[i];
      const int f = entry_f(e);
      const float ya = entry_y(e);
      const float a = fabsf(ya);
      const uint32_t ca = (uint32_t)entry_j(e) + (ya >= 0.0f ? 0u : (uint32_t)D);
      if (l == 1) {
        if (a >= mn) {
          const uint32_t x = atomicAdd(&st->pcount, 1u);
          if (x < (uint32_t)kPairCap) {
            pkey[x] = ((uint64_t)ord_f(a) << 32) | (uint32_t)~((uint32_t)f * (uint32_t)D + rk[i]);
            pval[x] = (uint32_t)f * stride + ca;
          }
        }
        continue;
      }
      if (f & 1) continue;
      const int t = f >> 1;
      for (uint32_t u = start[f + 1]; u < start[f + 2]; ++u) {
        const uint64_t o = grp[u];
        const float yb = entry_y(o);
        const float sc = a + fabsf(yb);
        if (sc >= mn) {
          const uint32_t x = atomicAdd(&st->pcount, 1u);
          if (x < (uint32_t)kPairCap) {
            const uint32_t cb = (uint32_t)entry_j(o) + (yb >= 0.0f ? 0u : (uint32_t)D);
            const uint32_t pos = (uint32_t)t * (uint32_t)(D * D) + (uint32_t)rk[i] * (uint32_t)D + rk[u];
            pkey[x] = ((uint64_t)ord_f(sc) << 32) | (uint32_t)~pos;
            pval[x] = (uint32_t)t * stride + ca * (uint32_t)(2 * D) + cb;
          }
        }
      }
    }
    __syncthreads();
    np = st->pcount;
    fail = np > (uint32_t)kPairCap || np < (uint32_t)qP;
  }
  if (fail) {
    if (tid == 0) nprobe[q] = -1;
    return;
  }
  // ---- 4. the first qP pairs in key order are the probes (keys are distinct)
  uint32_t* out = probes + (size_t)q * qcap;
  for (uint32_t i = tid; i < np; i += bs) {
    const uint64_t k = pkey[i];
    uint32_t r = 0;
    for (uint32_t u = 0; u < np; ++u) r += pkey[u] > k ? 1u : 0u;
    if (r < (uint32_t)qP) out[r] = pval[i];
  }
  if (tid == 0) nprobe[q] = qP;
}

// Workgroup of W wavefronts, W in [4, 8] with the fewest idle item slots over the passes of the
// L * l functions (ties: the larger W).
template <int P>
int hp_waves(int LF) {
  constexpr int IPW = QLayout<P>::IPW;
  int best = 4;
  long waste_best = -1;
  for (int w = 4; w <= 8; ++w) {
    const long per = (long)w * IPW;
    const long waste = (LF + per - 1) / per * per - LF;
    if (waste_best < 0 || waste <= waste_best) {
      waste_best = waste;
      best = w;
    }
  }
  return best;
}

template <int P, bool HALF>
hipError_t launch_hp_p(const fpp_index* ix, const float* V, int64_t m, int ldv, const int32_t* qp_arr,
                       int32_t qp_uniform, int32_t qcap, uint32_t* probes, int32_t* nprobe,
                       hipStream_t s) {
  const bool vec = (ix->d % 4 == 0) && (ldv % 4 == 0) && ((uintptr_t)V % 16 == 0);
  const int LF = ix->L * ix->l;
  const HPLayout lo(LF, ix->L, ix->l);
  const dim3 block(64 * hp_waves<P>(LF));
  if (vec)
    hipLaunchKernelGGL((hash_probe_kernel<P, true, HALF>), dim3((unsigned)m), block, lo.total, s, V,
                       m, ldv, ix->d, ix->sign_bits, ix->L, ix->l, ix->NB, qp_arr, qp_uniform, qcap,
                       probes, nprobe);
  else
    hipLaunchKernelGGL((hash_probe_kernel<P, false, HALF>), dim3((unsigned)m), block, lo.total, s, V,
                       m, ldv, ix->d, ix->sign_bits, ix->L, ix->l, ix->NB, qp_arr, qp_uniform, qcap,
                       probes, nprobe);
  return hipGetLastError();
}

}  // namespace

bool hash_probe_applies(const fpp_index* ix, int32_t qp_max, int32_t probe_score, int32_t store) {
  if (probe_score != FPP_PROBE_SUM || store == FPP_STORE_SIMHASH) return false;
  const bool full = ix->D == ix->P && ix->P >= 16 && ix->P <= 256;
  // D = P / 2 up to P = 512; at P = 512 only for at most one probe per table: beyond that the
  // second rotation of the active tables costs more than the list kernel's sort saves (measured
  // at d = 300, L = 128: 2.58 against 3.39 ms per 10,000 queries at qProbes = 101, 4.39 against
  // 4.10 ms at qProbes = 200)
  const bool half = 2 * ix->D == ix->P && ix->P >= 32 && ix->P <= 512;
  if (!full && !half) return false;
  if (ix->P == 512 && (int64_t)qp_max > ix->L) return false;
  if (ix->L > kMaxTables || (ix->l != 1 && ix->l != 2)) return false;
  if ((int64_t)ix->L * ix->D * ix->D >= ((int64_t)1 << 32) || (ix->NB + 1) * (int64_t)ix->L >= ((int64_t)1 << 32))
    return false;
  // about two probes per table at most: beyond that the candidate outputs outgrow LDS
  return qp_max >= 1 && (int64_t)qp_max <= 2LL * ix->L;
}

hipError_t launch_hash_probe(const fpp_index* ix, const float* V, int64_t m, int ldv,
                             const int32_t* qp_arr, int32_t qp_uniform, int32_t qcap,
                             uint32_t* probes, int32_t* nprobe, hipStream_t s) {
  if (m <= 0) return hipSuccess;
#define FPP_HP(PP, HH) return launch_hp_p<PP, HH>(ix, V, m, ldv, qp_arr, qp_uniform, qcap, probes, nprobe, s)
  if (ix->D == ix->P) {
    switch (ix->P) {
      case 16: FPP_HP(16, false);
      case 32: FPP_HP(32, false);
      case 64: FPP_HP(64, false);
      case 128: FPP_HP(128, false);
      case 256: FPP_HP(256, false);
      default: return hipErrorInvalidValue;
    }
  }
  if (2 * ix->D == ix->P) {
    switch (ix->P) {
      case 32: FPP_HP(32, true);
      case 64: FPP_HP(64, true);
      case 128: FPP_HP(128, true);
      case 256: FPP_HP(256, true);
      case 512: FPP_HP(512, true);
      default: return hipErrorInvalidValue;
    }
  }
#undef FPP_HP
  return hipErrorInvalidValue;
}

}  // namespace fpp
