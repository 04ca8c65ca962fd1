// fpp_query_ex_noalloc: the query pipeline of fpp_query_ex with every per-call buffer taken from
// one static device array instead of the stream-ordered allocator, for callers that cannot
// allocate (code under HIP graph capture, tight serving loops, harnesses that forbid it).
//
// The array (`scratch`, kScratchBytes) exists once per device that loads the library and lives
// until the process ends. Host code never passes the array's name to a kernel: on the first call
// on a device the library looks up that device's address of the array with hipGetSymbolAddress
// and uses only that address afterwards. Layout per call:
//   [ overflow dedup bitmaps of the gather, one per workgroup of its (reduced) grid ]
//   [ 256 bytes: the gather's work counters and a zero line ]
//   [ sorted lists, probes, counts and short lists of one chunk of queries ]
// The bitmaps and counters must be zero when the gather starts; a fill kernel on the caller's
// stream clears them at the start of every call (no hipMemsetAsync, so the call can be captured
// into a graph). Calls that overlap on one device share the array and therefore race.
#include <mutex>

#include "fpp_internal.hpp"

namespace fpp {
namespace {

constexpr size_t kScratchBytes = (size_t)128 << 20;   // 128 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};

// This device's address of `scratch` (looked up once per device, with the device current).
int device_scratch(unsigned char** out) {
  int dev = 0;
  FPP_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return set_error("device %d out of range", dev), FPP_EINVAL;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                               "hipGetSymbolAddress(scratch)", __FILE__, __LINE__);
    g_scratch_ptr[dev] = static_cast<unsigned char*>(p);
  }
  *out = g_scratch_ptr[dev];
  return FPP_OK;
}

__global__ __launch_bounds__(256) void zero_fill_kernel(uint4* __restrict__ p, int64_t n16) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += (int64_t)gridDim.x * 256)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
}

}  // namespace
}  // namespace fpp

using namespace fpp;

extern "C" int fpp_query_ex_noalloc(const fpp_index* ix, const float* Q, int64_t m, int32_t k,
                                    int32_t qProbes, const fpp_query_opts* opts, int32_t* ids_out,
                                    float* scores_out, void* stream) {
  if (!ix) return set_error("index is NULL"), FPP_EINVAL;
  if (m < 0) return set_error("m < 0"), FPP_EINVAL;
  if (m == 0) return FPP_OK;
  if (!Q || !ids_out || !scores_out) return set_error("Q, ids_out and scores_out must be non-NULL"), FPP_EINVAL;
  QuerySpec qs;
  qs.Q = Q;
  qs.m = m;
  qs.k_uniform = qs.k_max = k;
  qs.qp_uniform = qs.qp_max = qProbes;
  qs.ids_out = ids_out;
  qs.scores_out = scores_out;
  if (opts) {
    if (opts->stage_ms) return set_error("stage_ms is not available without allocation"), FPP_EINVAL;
    qs.store = opts->store;
    qs.R_opt = opts->rerank_R;
    qs.probe_score = opts->probe_score;
    qs.stats = opts->stats;
  }
  if (k < 1 || k > kMaxK) return set_error("k=%d out of [1, %d]", k, kMaxK), FPP_EINVAL;
  if (qProbes < 1) return set_error("qProbes=%d < 1", qProbes), FPP_EINVAL;
  FPP_TRY(check_store(ix, qs.store));
  if (qs.R_opt < -1 || qs.R_opt > kMaxK) return set_error("rerank_R=%d out of [-1, %d]", qs.R_opt, kMaxK), FPP_EINVAL;
  if (qs.R_opt > 0 && qs.store != FPP_STORE_FP32 && qs.R_opt < k)
    return set_error("rerank_R=%d < k=%d", qs.R_opt, k), FPP_EINVAL;
  if (qs.probe_score != FPP_PROBE_SUM && qs.probe_score != FPP_PROBE_GAP)
    return set_error("unknown probe_score %d", qs.probe_score), FPP_EINVAL;

  // the gather's grid: as many workgroups as have their n-bit bitmap within a quarter of the
  // array (at most the usual grid)
  const size_t bm_bytes = (size_t)overflow_bitmap_words(ix) * 4;
  const int grid = (int)std::min<size_t>((size_t)score_grid_blocks(ix), (kScratchBytes / 4) / bm_bytes);
  if (grid < 1)
    return set_error("an overflow bitmap of %zu bytes (n=%lld) exceeds the %zu-byte static scratch",
                     bm_bytes, (long long)ix->n, kScratchBytes), FPP_ECAPACITY;
  const size_t head = a256((size_t)grid * bm_bytes + 256);   // bitmaps, counters, zero line
  // queries per chunk: the largest layout that fits after the head
  int64_t budget = (int64_t)(kScratchBytes - head);
  Layout ly;
  for (int tries = 0; tries < 8; ++tries) {
    ly = plan_layout(ix, m, qs.qp_max, qs.k_max, qs.store, qs.R_opt, budget, false);
    if ((int64_t)ly.total <= (int64_t)(kScratchBytes - head)) break;
    budget -= (int64_t)ly.total - (int64_t)(kScratchBytes - head) + 4096;
  }
  if (ly.mc < 1 || ly.total > kScratchBytes - head)
    return set_error("one query needs %zu scratch bytes; the static scratch holds %zu after the %zu "
                     "bytes of dedup bitmaps", ly.total, kScratchBytes - head, head), FPP_ECAPACITY;
  ly.grid = grid;

  unsigned char* base = nullptr;
  FPP_TRY(device_scratch(&base));
  const hipStream_t s = (hipStream_t)stream;
  const int64_t n16 = (int64_t)(head / 16);
  hipLaunchKernelGGL(zero_fill_kernel, dim3((unsigned)std::min<int64_t>((n16 + 255) / 256, 1024)),
                     dim3(256), 0, s, reinterpret_cast<uint4*>(base), n16);
  FPP_HIP(hipGetLastError());
  qs.gbm_ext = reinterpret_cast<uint32_t*>(base);
  return run_queries(ix, qs, ly, base + head, s);
}
