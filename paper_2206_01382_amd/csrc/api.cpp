// Host runtime and C ABI of libfpp: validation, index build orchestration, the query
// pipeline (hash -> probe selection -> gather/score/top-k -> optional FP32 rerank), index
// inspection. Every step of the path runs in the HIP kernels of this library.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>

#include "fpp_internal.hpp"

namespace fpp {

static thread_local std::string g_error;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
}

int hip_fail(hipError_t e, const char* what, const char* file, int line) {
  set_error("HIP error %d (%s) in %s at %s:%d", (int)e, hipGetErrorString(e), what, file, line);
  return e == hipErrorOutOfMemory ? FPP_ENOMEM : FPP_EHIP;
}

// SplitMix64 (S. Vigna): output c of the stream whose state starts at `seed` mixes the state
// seed + (c + 1) * 0x9E3779B97F4A7C15.
static inline uint64_t splitmix64_at(uint64_t seed, uint64_t c) {
  uint64_t z = seed + (c + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Sign of element j of diagonal r of function (t, f) is negative iff bit 63 of the output at
// counter ((t * l + f) * 3 + r) * P + j is set. Stored as XOR masks of the float sign bit.
std::vector<uint32_t> make_sign_masks(uint64_t seed, int L, int l, int P) {
  std::vector<uint32_t> m((size_t)L * l * 3 * P);
  for (size_t c = 0; c < m.size(); ++c) m[c] = (splitmix64_at(seed, c) >> 63) ? 0x80000000u : 0u;
  return m;
}

std::vector<uint32_t> pack_sign_bits(const std::vector<uint32_t>& masks, int L, int l, int P) {
  const int wpr = std::max(1, P / 32);
  std::vector<uint32_t> w((size_t)L * l * 3 * wpr, 0u);
  for (size_t fr = 0; fr < (size_t)L * l * 3; ++fr)
    for (int j = 0; j < P; ++j)
      if (masks[fr * P + j]) w[fr * wpr + j / 32] |= 1u << (j % 32);
  return w;
}

int64_t keep_count_host(int64_t B, int64_t A, int K, int rounding) {
  const uint64_t den = (uint64_t)K * 1000000ull, num = (uint64_t)B * (uint64_t)A;
  return (int64_t)(rounding == 0 ? (num + den - 1) / den : num / den);
}

// Standard normal quantile by Wichura's algorithm AS 241 (PPND16, Applied Statistics 37(3),
// 1988): rational approximations in three ranges, relative accuracy about 1e-16.
double normal_quantile(double p) {
  if (!(p > 0.0 && p < 1.0)) return std::nan("");
  const double q = p - 0.5;
  if (std::fabs(q) <= 0.425) {
    const double r = 0.180625 - q * q;
    const double num = (((((((2.5090809287301226727e+3 * r + 3.3430575583588128105e+4) * r +
                             6.7265770927008700853e+4) * r + 4.5921953931549871457e+4) * r +
                           1.3731693765509461125e+4) * r + 1.9715909503065514427e+3) * r +
                         1.3314166789178437745e+2) * r + 3.3871328727963666080e+0);
    const double den = (((((((5.2264952788528545610e+3 * r + 2.8729085735721942674e+4) * r +
                             3.9307895800092710610e+4) * r + 2.1213794301586595867e+4) * r +
                           5.3941960214247511077e+3) * r + 6.8718700749205790830e+2) * r +
                         4.2313330701600911252e+1) * r + 1.0);
    return q * num / den;
  }
  double r = q < 0.0 ? p : 1.0 - p;
  r = std::sqrt(-std::log(r));
  double val;
  if (r <= 5.0) {
    r -= 1.6;
    const double num = (((((((7.74545014278341407640e-4 * r + 2.27238449892691845833e-2) * r +
                             2.41780725177450611770e-1) * r + 1.27045825245236838258e+0) * r +
                           3.64784832476320460504e+0) * r + 5.76949722146069140550e+0) * r +
                         4.63033784615654529590e+0) * r + 1.42343711074968357734e+0);
    const double den = (((((((1.05075007164441684324e-9 * r + 5.47593808499534494600e-4) * r +
                             1.51986665636164571966e-2) * r + 1.48103976427480074590e-1) * r +
                           6.89767334985100004550e-1) * r + 1.67638483018380384940e+0) * r +
                         2.05319162663775882187e+0) * r + 1.0);
    val = num / den;
  } else {
    r -= 5.0;
    const double num = (((((((2.01033439929228813265e-7 * r + 2.71155556874348757815e-5) * r +
                             1.24266094738807843860e-3) * r + 2.65321895265761230930e-2) * r +
                           2.96560571828504891230e-1) * r + 1.78482653991729133580e+0) * r +
                         5.46378491116411436990e+0) * r + 6.65790464350110377720e+0);
    const double den = (((((((2.04426310338993978564e-15 * r + 1.42151175831644588870e-7) * r +
                             1.84631831751005468180e-5) * r + 7.86869131145613259100e-4) * r +
                           1.48753612908506148525e-2) * r + 1.36929880922735805310e-1) * r +
                         5.99832206555887937690e-1) * r + 1.0);
    val = num / den;
  }
  return q < 0.0 ? -val : val;
}

// Centring vector: per coordinate the float64 sum of the n values in row order, divided by n in
// float64 and rounded to float32. X is read back in chunks of rows.
static int compute_center(const float* X, int64_t n, int32_t d, hipStream_t s, std::vector<float>* c) {
  std::vector<double> acc((size_t)d, 0.0);
  const int64_t rows = std::max<int64_t>(1, ((int64_t)64 << 20) / ((int64_t)d * 4));
  std::vector<float> buf((size_t)std::min(rows, n) * d);
  for (int64_t r0 = 0; r0 < n; r0 += rows) {
    const int64_t nr = std::min(rows, n - r0);
    FPP_HIP(hipMemcpyAsync(buf.data(), X + r0 * d, (size_t)nr * d * 4, hipMemcpyDeviceToHost, s));
    FPP_HIP(hipStreamSynchronize(s));
    for (int64_t i = 0; i < nr; ++i) {
      const float* row = buf.data() + (size_t)i * d;
      for (int32_t j = 0; j < d; ++j) acc[j] += (double)row[j];
    }
  }
  c->resize((size_t)d);
  for (int32_t j = 0; j < d; ++j) (*c)[j] = (float)(acc[j] / (double)n);
  return FPP_OK;
}

static int next_pow2(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

static bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

// Device allocation tracked for the index footprint.
template <typename T>
static int dalloc(T** p, size_t count, int64_t* acc) {
  *p = nullptr;
  if (count == 0) count = 1;
  FPP_HIP(hipMalloc((void**)p, count * sizeof(T)));
  if (acc) *acc += (int64_t)(count * sizeof(T));
  return FPP_OK;
}

static void free_index_memory(fpp_index* ix) {
  if (!ix) return;
  void* ptrs[] = {ix->X, ix->Xbf16, ix->Xfp8, ix->fp8_scale, ix->sign_mask, ix->sign_bits,
                  ix->offsets, ix->ids, ix->center_vec, ix->Xsig};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  for (int i = 0; i < fpp_index::kGbmSets; ++i) {
    if (ix->gbm[i]) (void)hipFree(ix->gbm[i]);
    if (ix->gbm_free[i]) (void)hipEventDestroy(ix->gbm_free[i]);
    ix->gbm[i] = nullptr;
    ix->gbm_free[i] = nullptr;
  }
}

// Serialises the hand-over of an index's overflow bitmaps between calls (host side only).
static std::mutex g_gbm_mu;

// A scoped set of device buffers released on every exit path.
struct DeviceScratch {
  std::vector<void*> ptrs;
  ~DeviceScratch() {
    for (void* p : ptrs) (void)hipFree(p);
  }
  template <typename T>
  int get(T** p, size_t count) {
    FPP_TRY(dalloc(p, count, nullptr));
    ptrs.push_back((void*)*p);
    return FPP_OK;
  }
};

// Stream-ordered scratch for queries: the default pool keeps freed blocks cached.
static std::once_flag g_pool_once;
static void configure_pool() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return;
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, dev) != hipSuccess) return;
  uint64_t thr = UINT64_MAX;
  (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
}

// ------------------------------------------------------------------------------------------
// Build
// ------------------------------------------------------------------------------------------
static int validate_build(const float* X, int64_t n, int32_t d, int32_t L, int32_t D, float alpha,
                          int32_t iProbes, int l) {
  if (!X) return set_error("X is NULL"), FPP_EINVAL;
  if (n < 1 || n >= (int64_t)1 << 31) return set_error("n=%lld out of [1, 2^31)", (long long)n), FPP_EINVAL;
  if (d < 1 || d > kMaxD) return set_error("d=%d out of [1, %d]", d, kMaxD), FPP_EINVAL;
  if (L < 1 || L > 4096) return set_error("L=%d out of [1, 4096]", L), FPP_EINVAL;
  if (!is_pow2(D) || D < 2 || D > 2048) return set_error("D=%d is not a power of two in [2, 2048]", D), FPP_EINVAL;
  if (l != 1 && l != 2) return set_error("l=%d must be 1 or 2", l), FPP_EINVAL;
  const int P = std::max(D, next_pow2(d));
  if (P > kMaxP) return set_error("rotation length P=%d exceeds %d", P, kMaxP), FPP_EINVAL;
  if (!(alpha > 0.0f) || !(alpha <= 1.0f)) return set_error("alpha=%g out of (0, 1]", (double)alpha), FPP_EINVAL;
  const int64_t pairs = l == 1 ? (int64_t)D : (int64_t)D * D;
  if (iProbes < 1 || iProbes > kMaxIProbes || iProbes > pairs)
    return set_error("iProbes=%d out of [1, min(%d, D^l=%lld)]", iProbes, kMaxIProbes, (long long)pairs), FPP_EINVAL;
  if (n * (int64_t)iProbes >= (int64_t)1 << 31)
    return set_error("n * iProbes must stay below 2^31"), FPP_EINVAL;
  const int64_t NB = l == 1 ? 2LL * D : 4LL * D * D;
  if ((int64_t)L * (NB + 1) >= (int64_t)1 << 32)
    return set_error("L * ((2D)^l + 1) must stay below 2^32"), FPP_ECAPACITY;
  return FPP_OK;
}

static int build_impl(const float* X, int64_t n, int32_t d, int32_t L, int32_t D, float alpha,
                      int32_t iProbes, uint64_t seed, const fpp_build_opts& o, hipStream_t s,
                      fpp_index** out) {
  const auto t_start = std::chrono::steady_clock::now();
  FPP_TRY(validate_build(X, n, d, L, D, alpha, iProbes, o.l));
  if (!out) return set_error("out is NULL"), FPP_EINVAL;
  if (o.keep_rounding != 0 && o.keep_rounding != 1) return set_error("keep_rounding must be 0 or 1"), FPP_EINVAL;
  if (o.stores & ~((1 << FPP_STORE_BF16) | (1 << FPP_STORE_FP8) | (1 << FPP_STORE_SIMHASH)))
    return set_error("unknown store bits 0x%x", o.stores), FPP_EINVAL;
  int32_t sigF = 0;
  if (o.stores & (1 << FPP_STORE_SIMHASH)) {
    sigF = o.simhash_functions;
    if (sigF == 0) sigF = std::max(o.l, (256 / D) / o.l * o.l);
    if (sigF < 1 || sigF % o.l != 0 || sigF > L * o.l || (int64_t)sigF * D > 1024)
      return set_error("simhash_functions=%d: need a multiple of l, at most L*l, with F*D <= 1024", sigF),
             FPP_EINVAL;
  }
  if (o.kappa < 0) return set_error("kappa=%d < 0", o.kappa), FPP_EINVAL;
  if (o.center != 0 && o.center != 1) return set_error("center must be 0 or 1"), FPP_EINVAL;
  if (o.filter != FPP_FILTER_FRACTION && o.filter != FPP_FILTER_THRESHOLD)
    return set_error("unknown filter %d", o.filter), FPP_EINVAL;
  if (!(o.threshold == o.threshold) || std::isinf(o.threshold))
    return set_error("threshold is not finite"), FPP_EINVAL;

  std::unique_ptr<fpp_index> ix(new (std::nothrow) fpp_index());
  if (!ix) return set_error("host allocation failed"), FPP_ENOMEM;
  struct Guard {
    fpp_index* p;
    bool armed = true;
    ~Guard() {
      if (armed) free_index_memory(p);
    }
  } guard{ix.get()};

  FPP_HIP(hipGetDevice(&ix->device));
  ix->n = n;
  ix->d = d;
  ix->L = L;
  ix->D = D;
  ix->l = o.l;
  ix->P = std::max(D, next_pow2(d));
  ix->iProbes = iProbes;
  ix->alpha = alpha;
  ix->alpha_micro = (int64_t)std::floor((double)alpha * 1e6 + 0.5);
  ix->seed = seed;
  ix->keep_rounding = o.keep_rounding;
  ix->kappa = o.filter == FPP_FILTER_FRACTION ? o.kappa : 0;
  ix->centered = o.center;
  ix->filter = o.filter;
  ix->stores = o.stores;
  ix->NB = o.l == 1 ? 2LL * D : 4LL * D * D;
  ix->ldx = (d + 3) / 4 * 4;
  ix->ld16 = (d + 7) / 8 * 8;
  {
    // FP8 rows: the codes padded to 16 bytes; where that leaves room in the row's last 128-byte
    // line, the row's scale follows in a 16-byte chunk of its own and rows are laid out so that
    // none straddles more lines than its bytes need (a power of two up to 128 bytes, else whole
    // lines): the gather then fetches a row and its scale together
    const int codes = (d + 15) / 16 * 16;
    if (codes % 128 == 0) {
      ix->ld8 = codes;
      ix->fp8_sc_off = -1;
    } else {
      const int need = codes + 16;
      int ld = 16;
      if (need <= 128) {
        while (ld < need) ld <<= 1;
      } else {
        ld = (need + 127) / 128 * 128;
      }
      ix->ld8 = ld;
      ix->fp8_sc_off = codes;
    }
  }
  const int64_t NB = ix->NB;
  const int K = iProbes;
  const int64_t nK = n * K;

  if (ix->filter == FPP_FILTER_THRESHOLD) {
    // t from alpha: a point reaches a given bucket with probability alpha / (2D)^l when each of
    // its l projections, divided by P (the scale of the unnormalised rotation), is >= t
    const double pa = (o.l == 1 ? (double)alpha : std::sqrt((double)alpha)) / (2.0 * D);
    const double t = o.threshold > 0.f ? (double)o.threshold : -normal_quantile(pa);
    ix->thr = (float)((double)ix->P * t);
    if (!(ix->thr >= 0.f)) ix->thr = 0.f;
  }
  // upper bound of the stored ids: sum over buckets of keep(B) <= alpha * n + #non-empty buckets
  // (plus kappa per non-empty bucket under limit scaling; every record under the threshold)
  int64_t per_table = keep_count_host(nK, ix->alpha_micro, K, 0) +
                      (int64_t)(1 + ix->kappa) * std::min<int64_t>(NB, nK) + 1;
  if (ix->filter == FPP_FILTER_THRESHOLD || per_table > nK + 1) per_table = nK + 1;
  const int64_t id_cap = per_table * L;
  if (id_cap >= (int64_t)1 << 32) return set_error("more than 2^32 - 1 stored ids"), FPP_ECAPACITY;

  int64_t bytes = 0;
  FPP_TRY(dalloc(&ix->X, (size_t)n * ix->ldx, &bytes));
  FPP_HIP(hipMemsetAsync(ix->X, 0, (size_t)n * ix->ldx * 4, s));
  FPP_HIP(hipMemcpy2DAsync(ix->X, (size_t)ix->ldx * 4, X, (size_t)d * 4, (size_t)d * 4, (size_t)n,
                           hipMemcpyDeviceToDevice, s));
  DeviceScratch centred;
  ix->Xh = ix->X;
  if (ix->centered) {
    std::vector<float> c;
    FPP_TRY(compute_center(X, n, d, s, &c));
    FPP_TRY(dalloc(&ix->center_vec, (size_t)d, &bytes));
    FPP_HIP(hipMemcpyAsync(ix->center_vec, c.data(), (size_t)d * 4, hipMemcpyHostToDevice, s));
    float* Xc = nullptr;
    FPP_TRY(centred.get(&Xc, (size_t)n * ix->ldx));
    FPP_HIP(launch_center(ix.get(), Xc, s));
    ix->Xh = Xc;
  }
  const std::vector<uint32_t> masks = make_sign_masks(seed, L, o.l, ix->P);
  FPP_TRY(dalloc(&ix->sign_mask, masks.size(), &bytes));
  FPP_HIP(hipMemcpyAsync(ix->sign_mask, masks.data(), masks.size() * 4, hipMemcpyHostToDevice, s));
  const std::vector<uint32_t> bits = pack_sign_bits(masks, L, o.l, ix->P);
  FPP_TRY(dalloc(&ix->sign_bits, bits.size(), &bytes));
  FPP_HIP(hipMemcpyAsync(ix->sign_bits, bits.data(), bits.size() * 4, hipMemcpyHostToDevice, s));
  FPP_TRY(dalloc(&ix->offsets, (size_t)L * (NB + 1), &bytes));
  FPP_TRY(dalloc(&ix->ids, (size_t)id_cap, &bytes));

  // tables per pass from free memory (at most a quarter of it, at most 4 GiB of scratch)
  size_t free_b = 0, total_b = 0;
  FPP_HIP(hipMemGetInfo(&free_b, &total_b));
  const int64_t per_tab_scratch = nK * 16 + NB * 20 + (NB + 1) * 4 + 64;
  const int64_t budget = std::min<int64_t>((int64_t)free_b / 4, (int64_t)4 << 30);
  int Tc = o.tables_per_pass > 0 ? o.tables_per_pass : (int)std::max<int64_t>(1, budget / per_tab_scratch);
  Tc = std::min(Tc, L);

  {
    DeviceScratch sc;
    BuildScratch bs{};
    FPP_TRY(sc.get(&bs.rec_bucket, (size_t)Tc * nK));
    FPP_TRY(sc.get(&bs.rec_key, (size_t)Tc * nK));
    FPP_TRY(sc.get(&bs.srt_key, (size_t)Tc * nK));
    FPP_TRY(sc.get(&bs.srt_id, (size_t)Tc * nK));
    FPP_TRY(sc.get(&bs.cnt, (size_t)Tc * NB));
    FPP_TRY(sc.get(&bs.start, (size_t)Tc * (NB + 1)));
    FPP_TRY(sc.get(&bs.fill, (size_t)Tc * NB));
    FPP_TRY(sc.get(&bs.meta, (size_t)(2 + Tc)));
    FPP_TRY(sc.get(&bs.tbase, (size_t)(L + 1)));
    FPP_TRY(sc.get(&bs.large, (size_t)Tc * NB));
    FPP_TRY(sc.get(&bs.n_large, (size_t)1));
    FPP_HIP(hipMemsetAsync(bs.meta, 0, sizeof(uint64_t) * (2 + Tc), s));
    for (int t0 = 0; t0 < L; t0 += Tc) {
      const int tc = std::min(Tc, L - t0);
      FPP_HIP(launch_hash_build(ix.get(), t0, tc, bs.rec_bucket, bs.rec_key, s));
      FPP_HIP(launch_build_tables(ix.get(), t0, tc, bs, s));
    }
    std::vector<uint64_t> tb((size_t)L + 1), meta(2);
    FPP_HIP(hipMemcpyAsync(tb.data(), bs.tbase, sizeof(uint64_t) * (L + 1), hipMemcpyDeviceToHost, s));
    FPP_HIP(hipMemcpyAsync(meta.data(), bs.meta, sizeof(uint64_t) * 2, hipMemcpyDeviceToHost, s));
    FPP_HIP(hipStreamSynchronize(s));
    ix->table_base.assign(tb.begin(), tb.end());
    ix->total_ids = (int64_t)tb[L];
    ix->max_bucket = (int64_t)meta[1];
  }

  if (o.stores & (1 << FPP_STORE_BF16)) FPP_TRY(dalloc(&ix->Xbf16, (size_t)n * ix->ld16, &bytes));
  if (o.stores & (1 << FPP_STORE_FP8)) {
    FPP_TRY(dalloc(&ix->Xfp8, (size_t)n * ix->ld8, &bytes));
    FPP_TRY(dalloc(&ix->fp8_scale, (size_t)n, &bytes));
  }
  if (o.stores & ((1 << FPP_STORE_BF16) | (1 << FPP_STORE_FP8))) FPP_HIP(launch_quantize(ix.get(), s));
  if (ix->Xbf16) {
    // an upper bound of the rows' norms, for the rerank's bound on the BF16 score error
    uint32_t* nb = nullptr;
    DeviceScratch nsc;
    FPP_TRY(nsc.get(&nb, 1));
    FPP_HIP(hipMemsetAsync(nb, 0, sizeof(uint32_t), s));
    FPP_HIP(launch_row_norm_max(ix.get(), nb, s));
    uint32_t bits = 0;
    FPP_HIP(hipMemcpyAsync(&bits, nb, sizeof(bits), hipMemcpyDeviceToHost, s));
    FPP_HIP(hipStreamSynchronize(s));
    float v;
    std::memcpy(&v, &bits, sizeof(v));
    ix->xnorm_max = std::isfinite(v) ? v : -1.0f;
  }
  if (sigF) {
    // signatures: the sorted lists of the first F functions of every point, packed to bits
    ix->sigF = sigF;
    ix->ldsig = (int32_t)(((int64_t)sigF * D + 127) / 128 * 4);
    FPP_TRY(dalloc(&ix->Xsig, (size_t)n * ix->ldsig, &bytes));
    fpp_index view = *ix;
    view.L = sigF / o.l;        // the first F functions, in (table, function) order
    const int64_t rows = std::max<int64_t>(1, ((int64_t)256 << 20) / ((int64_t)sigF * D * 6));
    DeviceScratch sg;
    float* la = nullptr;
    uint16_t* lc = nullptr;
    FPP_TRY(sg.get(&la, (size_t)std::min(rows, n) * sigF * D));
    FPP_TRY(sg.get(&lc, (size_t)std::min(rows, n) * sigF * D));
    for (int64_t r0 = 0; r0 < n; r0 += rows) {
      const int64_t nr = std::min(rows, n - r0);
      FPP_HIP(launch_hash_query(&view, ix->X + r0 * ix->ldx, nr, ix->ldx, la, lc, view.D, s));
      FPP_HIP(launch_pack_signs(lc, nr, sigF, D, sigF, ix->ldsig, ix->Xsig + r0 * ix->ldsig, s));
    }
    FPP_HIP(hipStreamSynchronize(s));
  }
  FPP_HIP(hipStreamSynchronize(s));
  ix->device_bytes = bytes;
  ix->Xh = nullptr;   // the centred copy is released with this call's scratch
  ix->build_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  guard.armed = false;
  *out = ix.release();
  return FPP_OK;
}

// ------------------------------------------------------------------------------------------
// Query pipeline
// ------------------------------------------------------------------------------------------
int64_t total_pairs(const fpp_index* ix) {
  return (int64_t)ix->L * (ix->l == 1 ? (int64_t)ix->D : (int64_t)ix->D * ix->D);
}

// Short-list length of a query with k results in a low-precision pass.
int32_t short_list_len(int32_t R_opt, int32_t k) {
  int32_t R = R_opt > 0 ? R_opt : std::max(100, 2 * k);
  R = std::min(R, kMaxK);
  return std::max(R, k);
}

size_t a256(size_t v) { return (v + 255) / 256 * 256; }

size_t overflow_bitmap_bytes(const fpp_index* ix) {
  // the bitmaps of the workgroups, then 256 bytes for the gather's work counters (words 0-1)
  // and 16 bytes that stay zero (words 4-7)
  return (size_t)score_grid_blocks(ix) * (size_t)overflow_bitmap_words(ix) * 4 + 256;
}

Layout plan_layout(const fpp_index* ix, int64_t m, int32_t qp_max, int32_t k_max,
                          int32_t store, int32_t R_opt, int64_t budget, bool gbm_in_scratch) {
  Layout ly;
  ly.qcap = (int32_t)std::min<int64_t>(std::max(qp_max, 1), total_pairs(ix));
  ly.short_ld = (store == FPP_STORE_FP32 || R_opt < 0) ? 0 : short_list_len(R_opt, k_max);
  const int64_t LF = (int64_t)ix->L * ix->l;
  const int64_t sigw = store == FPP_STORE_SIMHASH ? ix->ldsig : 0;
  const int64_t per_q = LF * ix->D * 6 + (int64_t)ly.qcap * 4 + 4 + (int64_t)ly.short_ld * 8 + sigw * 4 + 64;
  ly.mc = std::max<int64_t>(1, std::min<int64_t>(m, budget / per_q));
  ly.gbm = gbm_in_scratch;
  ly.grid = score_grid_blocks(ix);
  size_t o = 0;
  ly.off_la = o;
  o = a256(o + (size_t)ly.mc * LF * ix->D * 4);
  ly.off_lc = o;
  o = a256(o + (size_t)ly.mc * LF * ix->D * 2);
  ly.off_probes = o;
  o = a256(o + (size_t)ly.mc * ly.qcap * 4);
  ly.off_np = o;
  o = a256(o + (size_t)ly.mc * 4);
  ly.off_short = o;   // ids, then their approximate scores
  o = a256(o + (size_t)ly.mc * ly.short_ld * 8);
  ly.off_qsig = o;
  o = a256(o + (size_t)ly.mc * sigw * 4);
  ly.off_gbm = o;
  if (ly.gbm) o = a256(o + overflow_bitmap_bytes(ix));
  ly.total = o;
  return ly;
}

int check_store(const fpp_index* ix, int32_t store) {
  if (store == FPP_STORE_FP32) return FPP_OK;
  if (store == FPP_STORE_BF16 && ix->Xbf16) return FPP_OK;
  if (store == FPP_STORE_FP8 && ix->Xfp8) return FPP_OK;
  if (store == FPP_STORE_SIMHASH && ix->Xsig) return FPP_OK;
  if (store == FPP_STORE_BF16 || store == FPP_STORE_FP8 || store == FPP_STORE_SIMHASH)
    return set_error("store %d was not built for this index", store), FPP_ESTATE;
  return set_error("unknown store %d", store), FPP_EINVAL;
}

// Runs the query pipeline over [0, m) in chunks, with scratch `ws` (device) laid out by `ly`.
int run_queries(const fpp_index* ix, const QuerySpec& qs, const Layout& ly,
                       unsigned char* ws, hipStream_t s, std::vector<hipEvent_t>* ev) {
  auto mark = [&]() -> int {
    if (!ev) return FPP_OK;
    hipEvent_t e;
    FPP_HIP(hipEventCreate(&e));
    ev->push_back(e);
    FPP_HIP(hipEventRecord(e, s));
    return FPP_OK;
  };
  float* la = (float*)(ws + ly.off_la);
  uint16_t* lc = (uint16_t*)(ws + ly.off_lc);
  uint32_t* probes = (uint32_t*)(ws + ly.off_probes);
  int32_t* np = (int32_t*)(ws + ly.off_np);
  int32_t* shortl = (int32_t*)(ws + ly.off_short);
  float* shortsc = (float*)(ws + ly.off_short) + (size_t)ly.mc * ly.short_ld;
  const float bound_c = qs.store == FPP_STORE_BF16 && ix->rerank_cut ? bf16_rerank_bound(ix) : -1.0f;
  uint32_t* gbm = ly.gbm ? (uint32_t*)(ws + ly.off_gbm) : qs.gbm_ext;
  const int d = ix->d;
  for (int64_t c0 = 0; c0 < qs.m; c0 += ly.mc) {
    const int64_t mc = std::min<int64_t>(ly.mc, qs.m - c0);
    const float* Qc = qs.Q + c0 * d;
    FPP_TRY(mark());
    // the SimHash signature reads every code; probe selection only a prefix of each list
    const int W = qs.store == FPP_STORE_SIMHASH ? ix->D : probe_list_len(ix, ly.qcap);
    const int32_t* qp_c = qs.qp_dev ? qs.qp_dev + c0 : nullptr;
    if (hash_probe_applies(ix, ly.qcap, qs.probe_score, qs.store)) {
      // hashing and selection in one kernel; the list-based kernels finish only the queries it
      // leaves (nprobe < 0)
      FPP_HIP(launch_hash_probe(ix, Qc, mc, d, qp_c, qs.qp_uniform, ly.qcap, probes, np, s));
      FPP_HIP(launch_hash_query(ix, Qc, mc, d, la, lc, W, s, np));
      FPP_TRY(mark());
      FPP_HIP(launch_probe_select(ix, la, lc, mc, qp_c, qs.qp_uniform, ly.qcap, qs.probe_score, probes,
                                  np, s, true));
    } else {
      FPP_HIP(launch_hash_query(ix, Qc, mc, d, la, lc, W, s));
      FPP_TRY(mark());
      FPP_HIP(launch_probe_select(ix, la, lc, mc, qp_c, qs.qp_uniform, ly.qcap, qs.probe_score, probes,
                                  np, s));
    }
    FPP_TRY(mark());
    ScoreArgs a{};
    a.Q = Qc;
    a.ldq = d;
    if (qs.store == FPP_STORE_SIMHASH) {
      // the query's signature from its sorted lists; the gather scores against it
      uint32_t* qsig = (uint32_t*)(ws + ly.off_qsig);
      FPP_HIP(launch_pack_signs(lc, mc, ix->L * ix->l, ix->D, ix->sigF, ix->ldsig, qsig, s));
      a.Q = reinterpret_cast<const float*>(qsig);
      a.ldq = ix->ldsig;
    }
    a.m = mc;
    a.probes = probes;
    a.nprobe = np;
    a.qcap = ly.qcap;
    a.k_arr = qs.k_dev ? qs.k_dev + c0 : nullptr;
    a.k_uniform = qs.k_uniform;
    a.store = qs.store;
    a.rerank_R = qs.R_opt;
    a.stats = qs.stats ? qs.stats + c0 * 3 : nullptr;
    a.gbitmap = gbm;
    a.grid = ly.grid;
    a.short_ids = shortl;
    a.short_sc = shortsc;
    a.short_ld = ly.short_ld;
    a.cut_c = qs.R_opt >= 0 ? bound_c : -1.0f;
    int32_t* ids_c = qs.ids_out;
    float* sc_c = qs.scores_out;
    const int64_t* off_c = nullptr;
    if (qs.off_dev) {
      off_c = qs.off_dev + c0;
    } else {
      ids_c += c0 * qs.k_uniform;
      sc_c += c0 * qs.k_uniform;
    }
    a.out_off = off_c;
    a.ids_out = ids_c;
    a.scores_out = sc_c;
    FPP_HIP(launch_score(ix, a, s));
    FPP_TRY(mark());
    if (qs.store != FPP_STORE_FP32 && qs.R_opt >= 0) {
      FPP_HIP(launch_rerank(ix, Qc, d, mc, shortl, shortsc, ly.short_ld, bound_c, a.k_arr,
                            qs.k_uniform, qs.R_opt, off_c, ids_c, sc_c, s));
    }
    FPP_TRY(mark());
  }
  return FPP_OK;
}

static int query_common(const fpp_index* ix, QuerySpec& qs, hipStream_t s) {
  if (!ix) return set_error("index is NULL"), FPP_EINVAL;
  if (qs.m < 0) return set_error("m < 0"), FPP_EINVAL;
  if (qs.m == 0) return FPP_OK;
  if (!qs.Q || !qs.ids_out || !qs.scores_out) return set_error("Q, ids_out and scores_out must be non-NULL"), FPP_EINVAL;
  FPP_TRY(check_store(ix, qs.store));
  if (qs.R_opt < -1 || qs.R_opt > kMaxK) return set_error("rerank_R=%d out of [-1, %d]", qs.R_opt, kMaxK), FPP_EINVAL;
  if (qs.probe_score != FPP_PROBE_SUM && qs.probe_score != FPP_PROBE_GAP)
    return set_error("unknown probe_score %d", qs.probe_score), FPP_EINVAL;

  DeviceScratch host_arrays_unused;
  unsigned char* arrays = nullptr;
  if (qs.k_host) {
    int32_t kmax = 0, qpmax = 0;
    for (int64_t i = 0; i < qs.m; ++i) {
      const int32_t k = qs.k_host[i], qp = qs.qp_host[i];
      if (k < 1 || k > kMaxK) return set_error("k[%lld]=%d out of [1, %d]", (long long)i, k, kMaxK), FPP_EINVAL;
      if (qp < 1) return set_error("qProbes[%lld]=%d < 1", (long long)i, qp), FPP_EINVAL;
      if (qs.R_opt > 0 && qs.store != FPP_STORE_FP32 && qs.R_opt < k)
        return set_error("rerank_R=%d < k[%lld]=%d", qs.R_opt, (long long)i, k), FPP_EINVAL;
      kmax = std::max(kmax, k);
      qpmax = std::max(qpmax, qp);
    }
    qs.k_max = kmax;
    qs.qp_max = qpmax;
  } else {
    if (qs.k_uniform < 1 || qs.k_uniform > kMaxK) return set_error("k=%d out of [1, %d]", qs.k_uniform, kMaxK), FPP_EINVAL;
    if (qs.qp_uniform < 1) return set_error("qProbes=%d < 1", qs.qp_uniform), FPP_EINVAL;
    if (qs.R_opt > 0 && qs.store != FPP_STORE_FP32 && qs.R_opt < qs.k_uniform)
      return set_error("rerank_R=%d < k=%d", qs.R_opt, qs.k_uniform), FPP_EINVAL;
    qs.k_max = qs.k_uniform;
    qs.qp_max = qs.qp_uniform;
  }
  std::call_once(g_pool_once, configure_pool);
  const Layout ly = plan_layout(ix, qs.m, qs.qp_max, qs.k_max, qs.store, qs.R_opt, (int64_t)4 << 30, false);
  // a set of overflow bitmaps for this call: one last used on this stream (stream order frees
  // it), else one whose last user has finished, else a new one, else the one taken longest ago
  // (this call's stream then waits for its last user)
  // The lock is held while this call's kernels are enqueued (host side only), so that the set's
  // event records this call before another call can take the set.
  int set = -1;
  std::unique_lock<std::mutex> gbm_lock(g_gbm_mu);
  {
    for (int i = 0; i < fpp_index::kGbmSets && set < 0; ++i)
      if (ix->gbm[i] && ix->gbm_stream[i] == s) set = i;
    for (int i = 0; i < fpp_index::kGbmSets && set < 0; ++i)
      if (ix->gbm[i] && hipEventQuery(ix->gbm_free[i]) == hipSuccess) set = i;
    for (int i = 0; i < fpp_index::kGbmSets && set < 0; ++i) {
      if (ix->gbm[i]) continue;
      const size_t b = overflow_bitmap_bytes(ix);
      FPP_HIP(hipMalloc((void**)&ix->gbm[i], b));
      hipError_t e = hipMemset(ix->gbm[i], 0, b);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&ix->gbm_free[i], hipEventDisableTiming);
      if (e != hipSuccess) {
        (void)hipFree(ix->gbm[i]);
        ix->gbm[i] = nullptr;
        ix->gbm_free[i] = nullptr;
        return hip_fail(e, "overflow bitmaps", __FILE__, __LINE__);
      }
      set = i;
    }
    if (set < 0) {
      set = 0;
      for (int i = 1; i < fpp_index::kGbmSets; ++i)
        if (ix->gbm_stamp[i] < ix->gbm_stamp[set]) set = i;
    }
    ix->gbm_stamp[set] = ++ix->gbm_calls;
    ix->gbm_stream[set] = s;
    // the set's previous user (if any) finishes before this call's kernels start
    FPP_HIP(hipStreamWaitEvent(s, ix->gbm_free[set], 0));
    qs.gbm_ext = ix->gbm[set];
  }
  size_t arr_bytes = 0;
  if (qs.k_host) arr_bytes = a256((size_t)qs.m * 16);
  unsigned char* ws = nullptr;
  FPP_HIP(hipMallocAsync((void**)&ws, ly.total + arr_bytes, s));
  int rc = FPP_OK;
  do {
    if (qs.k_host) {
      arrays = ws + ly.total;
      std::vector<int64_t> off((size_t)qs.m);
      std::vector<int32_t> kq((size_t)qs.m * 2);
      int64_t run = 0;
      for (int64_t i = 0; i < qs.m; ++i) {
        off[i] = run;
        run += qs.k_host[i];
        kq[i] = qs.k_host[i];
        kq[qs.m + i] = qs.qp_host[i];
      }
      hipError_t e = hipMemcpyAsync(arrays, off.data(), (size_t)qs.m * 8, hipMemcpyHostToDevice, s);
      if (e == hipSuccess)
        e = hipMemcpyAsync(arrays + (size_t)qs.m * 8, kq.data(), (size_t)qs.m * 8, hipMemcpyHostToDevice, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);   // host vectors go out of scope
      if (e != hipSuccess) { rc = hip_fail(e, "hipMemcpyAsync", __FILE__, __LINE__); break; }
      qs.off_dev = (const int64_t*)arrays;
      qs.k_dev = (const int32_t*)(arrays + (size_t)qs.m * 8);
      qs.qp_dev = qs.k_dev + qs.m;
    }
    std::vector<hipEvent_t> ev;
    rc = run_queries(ix, qs, ly, ws, s, qs.stage_ms ? &ev : nullptr);
    {
      const hipError_t e = hipEventRecord(ix->gbm_free[set], s);
      if (rc == FPP_OK && e != hipSuccess) rc = hip_fail(e, "hipEventRecord", __FILE__, __LINE__);
    }
    gbm_lock.unlock();
    if (qs.stage_ms) {
      for (int i = 0; i < 4; ++i) qs.stage_ms[i] = 0.0;
      if (rc == FPP_OK) {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) rc = hip_fail(e, "hipStreamSynchronize", __FILE__, __LINE__);
      }
      for (size_t c = 0; rc == FPP_OK && c + 4 < ev.size(); c += 5) {
        for (int i = 0; i < 4; ++i) {
          float ms = 0.f;
          if (hipEventElapsedTime(&ms, ev[c + i], ev[c + i + 1]) == hipSuccess) qs.stage_ms[i] += ms;
        }
      }
      for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
  } while (0);
  hipError_t fe = hipFreeAsync(ws, s);
  if (rc == FPP_OK && fe != hipSuccess) rc = hip_fail(fe, "hipFreeAsync", __FILE__, __LINE__);
  return rc;
}

}  // namespace fpp

using namespace fpp;

// ------------------------------------------------------------------------------------------
// C ABI
// ------------------------------------------------------------------------------------------
extern "C" {

const char* fpp_last_error(void) { return g_error.c_str(); }
const char* fpp_version(void) { return "fpp 0.1 (gfx950)"; }

void fpp_default_build_opts(fpp_build_opts* o) {
  if (!o) return;
  o->l = 2;
  o->stores = 0;
  o->keep_rounding = 0;
  o->tables_per_pass = 0;
  o->kappa = 0;
  o->center = 0;
  o->filter = FPP_FILTER_FRACTION;
  o->threshold = 0.f;
  o->simhash_functions = 0;
}

void fpp_default_query_opts(fpp_query_opts* o) {
  if (!o) return;
  o->store = FPP_STORE_FP32;
  o->rerank_R = 0;
  o->stats = nullptr;
  o->stage_ms = nullptr;
  o->probe_score = FPP_PROBE_SUM;
}

int fpp_build_index(const float* X, int64_t n, int32_t d, int32_t L, int32_t D, float alpha,
                    int32_t iProbes, uint64_t seed, fpp_index** out) {
  fpp_build_opts o;
  fpp_default_build_opts(&o);
  return build_impl(X, n, d, L, D, alpha, iProbes, seed, o, nullptr, out);
}

int fpp_build_index_ex(const float* X, int64_t n, int32_t d, int32_t L, int32_t D, float alpha,
                       int32_t iProbes, uint64_t seed, const fpp_build_opts* opts, void* stream,
                       fpp_index** out) {
  fpp_build_opts o;
  fpp_default_build_opts(&o);
  if (opts) o = *opts;
  return build_impl(X, n, d, L, D, alpha, iProbes, seed, o, (hipStream_t)stream, out);
}

void fpp_free_index(fpp_index* index) {
  if (!index) return;
  free_index_memory(index);
  delete index;
}

int fpp_query(const fpp_index* index, const float* Q, int64_t m, int32_t k, int32_t qProbes,
              int32_t* ids_out, float* scores_out, void* stream) {
  return fpp_query_ex(index, Q, m, k, qProbes, nullptr, ids_out, scores_out, stream);
}

int fpp_query_ex(const fpp_index* index, const float* Q, int64_t m, int32_t k, int32_t qProbes,
                 const fpp_query_opts* opts, int32_t* ids_out, float* scores_out, void* stream) {
  QuerySpec qs;
  qs.Q = Q;
  qs.m = m;
  qs.k_uniform = k;
  qs.qp_uniform = qProbes;
  qs.ids_out = ids_out;
  qs.scores_out = scores_out;
  if (opts) {
    qs.store = opts->store;
    qs.R_opt = opts->rerank_R;
    qs.probe_score = opts->probe_score;
    qs.stats = opts->stats;
    qs.stage_ms = opts->stage_ms;
  }
  return query_common(index, qs, (hipStream_t)stream);
}

int fpp_query_batch(const fpp_index* index, const float* Q, int64_t m, const int32_t* k,
                    const int32_t* qProbes, const fpp_query_opts* opts, int32_t* ids_out,
                    float* scores_out, void* stream) {
  if (m > 0 && (!k || !qProbes)) return set_error("k and qProbes arrays must be non-NULL"), FPP_EINVAL;
  QuerySpec qs;
  qs.Q = Q;
  qs.m = m;
  qs.k_host = k;
  qs.qp_host = qProbes;
  qs.ids_out = ids_out;
  qs.scores_out = scores_out;
  if (opts) {
    qs.store = opts->store;
    qs.R_opt = opts->rerank_R;
    qs.probe_score = opts->probe_score;
    qs.stats = opts->stats;
    qs.stage_ms = opts->stage_ms;
  }
  return query_common(index, qs, (hipStream_t)stream);
}

int64_t fpp_query_workspace_bytes(const fpp_index* index, int64_t m, int32_t k_max,
                                  int32_t qprobes_max, const fpp_query_opts* opts) {
  if (!index || m < 0) return -1;
  const int32_t store = opts ? opts->store : FPP_STORE_FP32;
  const int32_t R = opts ? opts->rerank_R : 0;
  const Layout ly = plan_layout(index, std::max<int64_t>(m, 1), qprobes_max, k_max, store, R,
                                (int64_t)4 << 30, false);
  return (int64_t)(ly.total + a256((size_t)m * 16));
}

int fpp_index_get_info(const fpp_index* ix, fpp_index_info* info) {
  if (!ix || !info) return set_error("NULL argument"), FPP_EINVAL;
  info->n = ix->n;
  info->d = ix->d;
  info->L = ix->L;
  info->D = ix->D;
  info->l = ix->l;
  info->P = ix->P;
  info->iProbes = ix->iProbes;
  info->stores = ix->stores;
  info->alpha = ix->alpha;
  info->seed = ix->seed;
  info->buckets_per_table = ix->NB;
  info->total_ids = ix->total_ids;
  info->max_bucket = ix->max_bucket;
  info->device_bytes = ix->device_bytes;
  info->build_ms = ix->build_ms;
  info->kappa = ix->kappa;
  info->centered = ix->centered;
  info->filter = ix->filter;
  info->threshold = ix->filter == FPP_FILTER_THRESHOLD ? ix->thr : 0.f;
  info->simhash_bits = ix->sigF * ix->D;
  {
    std::lock_guard<std::mutex> lk(g_gbm_mu);
    info->overflow_sets = 0;
    for (int i = 0; i < fpp_index::kGbmSets; ++i) info->overflow_sets += ix->gbm[i] ? 1 : 0;
  }
  return FPP_OK;
}

int fpp_index_table_sizes(const fpp_index* ix, int64_t* sizes_out) {
  if (!ix || !sizes_out) return set_error("NULL argument"), FPP_EINVAL;
  for (int t = 0; t < ix->L; ++t) sizes_out[t] = ix->table_base[t + 1] - ix->table_base[t];
  return FPP_OK;
}

int fpp_debug_signs(const fpp_index* ix, int8_t* out) {
  if (!ix || !out) return set_error("NULL argument"), FPP_EINVAL;
  const std::vector<uint32_t> m = make_sign_masks(ix->seed, ix->L, ix->l, ix->P);
  for (size_t i = 0; i < m.size(); ++i) out[i] = m[i] ? -1 : 1;
  return FPP_OK;
}

int fpp_debug_query_lists(const fpp_index* ix, const float* V, int64_t m, float* abs_out,
                          int32_t* code_out, void* stream) {
  if (!ix) return set_error("NULL argument"), FPP_EINVAL;
  return fpp_debug_query_list_prefix(ix, V, m, ix->D, abs_out, code_out, stream);
}

int fpp_debug_query_list_prefix(const fpp_index* ix, const float* V, int64_t m, int32_t W,
                                float* abs_out, int32_t* code_out, void* stream) {
  if (!ix || (m > 0 && (!V || !abs_out || !code_out))) return set_error("NULL argument"), FPP_EINVAL;
  if (W < 1 || W > ix->D) return set_error("prefix %d outside [1, D = %d]", W, ix->D), FPP_EINVAL;
  if (m <= 0) return FPP_OK;
  hipStream_t s = (hipStream_t)stream;
  const size_t cnt = (size_t)m * ix->L * ix->l * ix->D;
  DeviceScratch sc;
  uint16_t* lc = nullptr;
  FPP_TRY(sc.get(&lc, cnt));
  FPP_HIP(hipMemsetAsync(lc, 0, cnt * 2, s));
  FPP_HIP(launch_hash_query(ix, V, m, ix->d, abs_out, lc, W, s));
  std::vector<uint16_t> h(cnt);
  FPP_HIP(hipMemcpyAsync(h.data(), lc, cnt * 2, hipMemcpyDeviceToHost, s));
  FPP_HIP(hipStreamSynchronize(s));
  std::vector<int32_t> c(cnt);
  for (size_t i = 0; i < cnt; ++i) c[i] = h[i];
  FPP_HIP(hipMemcpyAsync(code_out, c.data(), cnt * 4, hipMemcpyHostToDevice, s));
  FPP_HIP(hipStreamSynchronize(s));
  return FPP_OK;
}

int fpp_debug_build_records(const fpp_index* ix, int32_t t, uint32_t* bucket_out, float* key_out,
                            void* stream) {
  if (!ix || !bucket_out || !key_out) return set_error("NULL argument"), FPP_EINVAL;
  if (t < 0 || t >= ix->L) return set_error("table %d out of range", t), FPP_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (!ix->centered) {
    FPP_HIP(launch_hash_build(ix, t, 1, bucket_out, key_out, s));
    return FPP_OK;
  }
  // a centred index hashed X - c: rebuild that copy for the call
  DeviceScratch sc;
  float* Xc = nullptr;
  FPP_TRY(sc.get(&Xc, (size_t)ix->n * ix->ldx));
  FPP_HIP(launch_center(ix, Xc, s));
  fpp_index view = *ix;
  view.Xh = Xc;
  FPP_HIP(launch_hash_build(&view, t, 1, bucket_out, key_out, s));
  FPP_HIP(hipStreamSynchronize(s));
  view.table_base.clear();
  return FPP_OK;
}

int fpp_debug_center(const fpp_index* ix, float* c_out) {
  if (!ix || !c_out) return set_error("NULL argument"), FPP_EINVAL;
  if (!ix->center_vec) {
    std::fill(c_out, c_out + ix->d, 0.f);
    return FPP_OK;
  }
  FPP_HIP(hipMemcpy(c_out, ix->center_vec, (size_t)ix->d * 4, hipMemcpyDeviceToHost));
  return FPP_OK;
}

double fpp_normal_quantile(double p) { return normal_quantile(p); }

int fpp_debug_set_partition_threshold(fpp_index* ix, int64_t min_entries, int32_t range_bits) {
  if (!ix) return set_error("index is NULL"), FPP_EINVAL;
  if (range_bits >= 0 && (range_bits < 5 || range_bits > fpp_index::kPartShiftDefault))
    return set_error("range_bits=%d out of [5, %d]", range_bits, fpp_index::kPartShiftDefault), FPP_EINVAL;
  ix->part_min = min_entries < 0 ? fpp_index::kPartMinDefault : min_entries;
  ix->part_shift = range_bits < 0 ? fpp_index::kPartShiftDefault : range_bits;
  return FPP_OK;
}

int fpp_debug_set_rerank_cut(fpp_index* ix, int32_t enabled) {
  if (!ix) return set_error("index is NULL"), FPP_EINVAL;
  if (enabled != 0 && enabled != 1) return set_error("enabled=%d: 0 or 1", enabled), FPP_EINVAL;
  ix->rerank_cut = enabled == 1;
  return FPP_OK;
}

int fpp_debug_export_table(const fpp_index* ix, int32_t t, uint32_t* offsets_out, int32_t* ids_out) {
  if (!ix || !offsets_out || !ids_out) return set_error("NULL argument"), FPP_EINVAL;
  if (t < 0 || t >= ix->L) return set_error("table %d out of range", t), FPP_EINVAL;
  const int64_t NB = ix->NB;
  FPP_HIP(hipMemcpy(offsets_out, ix->offsets + (size_t)t * (NB + 1), (NB + 1) * 4, hipMemcpyDeviceToHost));
  const uint32_t base = offsets_out[0];
  for (int64_t b = 0; b <= NB; ++b) offsets_out[b] -= base;
  const int64_t sz = ix->table_base[t + 1] - ix->table_base[t];
  if (sz > 0) FPP_HIP(hipMemcpy(ids_out, ix->ids + ix->table_base[t], sz * 4, hipMemcpyDeviceToHost));
  return FPP_OK;
}

int fpp_debug_probes(const fpp_index* ix, const float* Q, int64_t m, int32_t qProbes,
                     int32_t probe_score, int64_t* probes_out, void* stream) {
  if (!ix || (m > 0 && (!Q || !probes_out))) return set_error("NULL argument"), FPP_EINVAL;
  if (qProbes < 1) return set_error("qProbes < 1"), FPP_EINVAL;
  if (probe_score != FPP_PROBE_SUM && probe_score != FPP_PROBE_GAP)
    return set_error("unknown probe_score %d", probe_score), FPP_EINVAL;
  if (m <= 0) return FPP_OK;
  hipStream_t s = (hipStream_t)stream;
  const int32_t qcap = (int32_t)std::min<int64_t>(qProbes, total_pairs(ix));
  const size_t LFD = (size_t)ix->L * ix->l * ix->D;
  DeviceScratch sc;
  float* la = nullptr;
  uint16_t* lc = nullptr;
  uint32_t* pr = nullptr;
  int32_t* np = nullptr;
  FPP_TRY(sc.get(&la, (size_t)m * LFD));
  FPP_TRY(sc.get(&lc, (size_t)m * LFD));
  FPP_TRY(sc.get(&pr, (size_t)m * qcap));
  FPP_TRY(sc.get(&np, (size_t)m));
  // the same kernels as the query path
  if (hash_probe_applies(ix, qcap, probe_score, FPP_STORE_FP32)) {
    FPP_HIP(launch_hash_probe(ix, Q, m, ix->d, nullptr, qProbes, qcap, pr, np, s));
    FPP_HIP(launch_hash_query(ix, Q, m, ix->d, la, lc, probe_list_len(ix, qcap), s, np));
    FPP_HIP(launch_probe_select(ix, la, lc, m, nullptr, qProbes, qcap, probe_score, pr, np, s, true));
  } else {
    FPP_HIP(launch_hash_query(ix, Q, m, ix->d, la, lc, probe_list_len(ix, qcap), s));
    FPP_HIP(launch_probe_select(ix, la, lc, m, nullptr, qProbes, qcap, probe_score, pr, np, s));
  }
  std::vector<uint32_t> h((size_t)m * qcap);
  std::vector<int32_t> hn((size_t)m);
  FPP_HIP(hipMemcpyAsync(h.data(), pr, h.size() * 4, hipMemcpyDeviceToHost, s));
  FPP_HIP(hipMemcpyAsync(hn.data(), np, hn.size() * 4, hipMemcpyDeviceToHost, s));
  FPP_HIP(hipStreamSynchronize(s));
  std::vector<int64_t> out(h.size(), -1);
  const int64_t NB = ix->NB;
  for (int64_t q = 0; q < m; ++q)
    for (int32_t i = 0; i < hn[q]; ++i) {
      const int64_t gb = h[(size_t)q * qcap + i];
      out[(size_t)q * qcap + i] = (gb / (NB + 1)) * NB + gb % (NB + 1);
    }
  FPP_HIP(hipMemcpyAsync(probes_out, out.data(), out.size() * 8, hipMemcpyHostToDevice, s));
  FPP_HIP(hipStreamSynchronize(s));
  return FPP_OK;
}

int fpp_debug_export_store(const fpp_index* ix, int32_t store, void* codes_out, float* scales_out,
                           void* stream) {
  if (!ix || !codes_out) return set_error("NULL argument"), FPP_EINVAL;
  FPP_TRY(check_store(ix, store));
  hipStream_t s = (hipStream_t)stream;
  if (store == FPP_STORE_BF16) {
    FPP_HIP(hipMemcpy2DAsync(codes_out, (size_t)ix->d * 2, ix->Xbf16, (size_t)ix->ld16 * 2,
                             (size_t)ix->d * 2, (size_t)ix->n, hipMemcpyDeviceToDevice, s));
  } else if (store == FPP_STORE_FP8) {
    if (!scales_out) return set_error("scales_out is NULL"), FPP_EINVAL;
    FPP_HIP(hipMemcpy2DAsync(codes_out, (size_t)ix->d, ix->Xfp8, (size_t)ix->ld8, (size_t)ix->d,
                             (size_t)ix->n, hipMemcpyDeviceToDevice, s));
    FPP_HIP(hipMemcpyAsync(scales_out, ix->fp8_scale, (size_t)ix->n * 4, hipMemcpyDeviceToDevice, s));
  } else if (store == FPP_STORE_SIMHASH) {
    const size_t words = ((size_t)ix->sigF * ix->D + 31) / 32;
    FPP_HIP(hipMemcpy2DAsync(codes_out, words * 4, ix->Xsig, (size_t)ix->ldsig * 4, words * 4,
                             (size_t)ix->n, hipMemcpyDeviceToDevice, s));
  } else {
    return set_error("store %d has no low-precision copy", store), FPP_EINVAL;
  }
  FPP_HIP(hipStreamSynchronize(s));
  return FPP_OK;
}

}  // extern "C"
