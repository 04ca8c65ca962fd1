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
// One wavefront per query; lane x walks tables x, x + 64, ...
#include "fpp_internal.hpp"

namespace fpp {
namespace {

__device__ __forceinline__ uint64_t count_table(const float* A, const float* B, int l, int D,
                                                float tau) {
  if (l == 1) {
    int c = 0;
    while (c < D && A[c] >= tau) ++c;
    return (uint64_t)c;
  }
  int j = 0;
  const float a0 = A[0];
  while (j < D && a0 + B[j] >= tau) ++j;
  uint64_t c = 0;
  for (int i = 0; i < D && j > 0; ++i) {
    const float ai = A[i];
    while (j > 0 && !(ai + B[j - 1] >= tau)) --j;
    c += (uint64_t)j;
  }
  return c;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ __forceinline__ uint64_t wave_excl_scan_u64(uint64_t v, uint64_t& total) {
  const int lane = threadIdx.x & 63;
  uint64_t inc = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t t = __shfl_up(inc, o);
    if (lane >= o) inc += t;
  }
  total = __shfl(inc, 63);
  return inc - v;
}

__global__ __launch_bounds__(256) void probe_kernel(
    const float* __restrict__ la, const uint16_t* __restrict__ lc, int64_t m, int L, int l, int D,
    int64_t NB, const int32_t* __restrict__ qp_arr, int32_t qp_uniform, int32_t qcap,
    uint32_t* __restrict__ probes, int32_t* __restrict__ nprobe) {
  const int lane = threadIdx.x & 63;
  const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (q >= m) return;   // whole wavefront
  const int LF = L * l;
  const float* Aq = la + (size_t)q * LF * D;
  const uint16_t* Cq = lc + (size_t)q * LF * D;
  const uint64_t total = (uint64_t)L * (l == 1 ? (uint64_t)D : (uint64_t)D * D);
  int64_t want = qp_arr ? qp_arr[q] : qp_uniform;
  uint64_t qP = want < 1 ? 0 : ((uint64_t)want < total ? (uint64_t)want : total);
  if (qP > (uint64_t)qcap) qP = (uint64_t)qcap;
  if (qP == 0) {
    if (lane == 0) nprobe[q] = 0;
    return;
  }

  float mx = 0.0f;
  for (int t = lane; t < L; t += 64) {
    const float* A = Aq + (size_t)t * l * D;
    const float s = l == 1 ? A[0] : A[0] + A[D];
    mx = fmaxf(mx, s);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
  uint32_t lo = 0u, hi = __float_as_uint(mx) + 1u;   // count_ge(lo) >= qP > count_ge(hi)
  uint64_t c_hi = 0;
  bool exact = false;
  while (hi - lo > 1u) {
    const uint32_t mid = lo + (hi - lo) / 2u;
    const float tau = __uint_as_float(mid);
    uint64_t c = 0;
    for (int t = lane; t < L; t += 64) {
      const float* A = Aq + (size_t)t * l * D;
      c += count_table(A, A + D, l, D, tau);
    }
    c = wave_sum_u64(c);
    if (c == qP) {
      lo = mid;
      exact = true;
      break;
    }
    if (c > qP) {
      lo = mid;
    } else {
      hi = mid;
      c_hi = c;
    }
  }
  // take every pair with s >= thr_gt, then `need` ties at s == tau_eq in (t, i, j) order
  const float thr_gt = __uint_as_float(exact ? lo : hi);
  const float tau_eq = __uint_as_float(lo);
  const uint64_t c_gt = exact ? qP : c_hi;
  const uint64_t need = qP - c_gt;
  uint32_t* out = probes + (size_t)q * qcap;
  const int64_t stride = NB + 1;
  const int twoD = 2 * D;

  uint64_t run_gt = 0, run_eq = 0;
  for (int tb = 0; tb < L; tb += 64) {
    const int t = tb + lane;
    const float* A = Aq + (size_t)t * l * D;
    const float* B = A + D;
    uint64_t n_gt = 0, n_eq = 0;
    if (t < L) {
      n_gt = count_table(A, B, l, D, thr_gt);
      if (need) n_eq = count_table(A, B, l, D, tau_eq) - n_gt;
    }
    uint64_t tot_gt, tot_eq;
    const uint64_t pos_gt0 = run_gt + wave_excl_scan_u64(n_gt, tot_gt);
    const uint64_t tie0 = run_eq + wave_excl_scan_u64(n_eq, tot_eq);
    run_gt += tot_gt;
    run_eq += tot_eq;
    if (t >= L) continue;
    const uint16_t* C1 = Cq + (size_t)t * l * D;
    const uint16_t* C2 = C1 + D;
    const uint32_t tbase = (uint32_t)((int64_t)t * stride);
    uint64_t pg = pos_gt0, te = tie0;
    if (l == 1) {
      for (uint64_t i = 0; i < n_gt; ++i) out[pg++] = tbase + C1[i];
      for (uint64_t i = n_gt; i < n_gt + n_eq && te < need; ++i, ++te)
        out[c_gt + te] = tbase + C1[i];
      continue;
    }
    // two thresholds walked together: jg for s >= thr_gt, je for s >= tau_eq (je >= jg)
    int jg = 0, je = 0;
    const float a0 = A[0];
    while (jg < D && a0 + B[jg] >= thr_gt) ++jg;
    if (need) {
      je = jg;
      while (je < D && a0 + B[je] >= tau_eq) ++je;
    }
    for (int i = 0; i < D && (jg > 0 || je > 0); ++i) {
      const float ai = A[i];
      while (jg > 0 && !(ai + B[jg - 1] >= thr_gt)) --jg;
      if (need)
        while (je > 0 && !(ai + B[je - 1] >= tau_eq)) --je;
      const uint32_t rowb = tbase + (uint32_t)C1[i] * twoD;
      for (int j = 0; j < jg; ++j) out[pg++] = rowb + C2[j];
      for (int j = jg; j < je && te < need; ++j, ++te) out[c_gt + te] = rowb + C2[j];
    }
  }
  if (lane == 0) nprobe[q] = (int32_t)qP;
}

}  // namespace

hipError_t launch_probe_select(const fpp_index* ix, const float* la, const uint16_t* lc, int64_t m,
                               const int32_t* qp_arr, int32_t qp_uniform, int32_t qcap,
                               uint32_t* probes, int32_t* nprobe, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(probe_kernel, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, s, la, lc, m,
                     ix->L, ix->l, ix->D, ix->NB, qp_arr, qp_uniform, qcap, probes, nprobe);
  return hipGetLastError();
}

}  // namespace fpp
