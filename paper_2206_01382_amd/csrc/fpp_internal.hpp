// Internal declarations shared by the HIP sources of libfpp (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/fpp.h"

namespace fpp {

// ----------------------------------------------------------------------------------------------
// Errors: a thread-local message plus FPP_E* codes; no exception leaves the library.
// ----------------------------------------------------------------------------------------------
void set_error(const char* fmt, ...);
int hip_fail(hipError_t e, const char* what, const char* file, int line);

#define FPP_HIP(call)                                                               \
  do {                                                                              \
    hipError_t _e = (call);                                                         \
    if (_e != hipSuccess) return ::fpp::hip_fail(_e, #call, __FILE__, __LINE__);    \
  } while (0)

#define FPP_TRY(call)                   \
  do {                                          \
    int _rc = (call);                            \
    if (_rc != FPP_OK) return _rc;               \
  } while (0)

constexpr int kMaxIProbes = 16;      // build kernel keeps at most this many buckets per point
constexpr int kMaxK = 512;           // results / short list per query
constexpr int kMaxD = 1024;          // dimension of stored vectors
constexpr int kMaxP = 4096;          // rotation length
constexpr uint32_t kDropped = 0xffffffffu;   // bucket of a build record the threshold filter drops

// ----------------------------------------------------------------------------------------------
// The index object (opaque in the ABI).
// ----------------------------------------------------------------------------------------------
}  // namespace fpp

struct fpp_index {
  int64_t n = 0;
  int32_t d = 0, L = 0, D = 0, l = 0, P = 0, iProbes = 0;
  float alpha = 0.f;
  int64_t alpha_micro = 0;   // alpha in millionths
  uint64_t seed = 0;
  int32_t keep_rounding = 0;
  int32_t kappa = 0;         // limit scaling: keep min(B, max(kappa, keep(B)))
  int32_t centered = 0;
  int32_t filter = 0;        // FPP_FILTER_*
  float thr = 0.f;           // FPP_FILTER_THRESHOLD: keep a record when every |y| >= thr
  int32_t stores = 0;        // bit mask of low-precision stores
  int64_t NB = 0;            // buckets per table, (2D)^l
  int32_t ldx = 0;           // FP32 row stride in floats (multiple of 4)
  int32_t ld16 = 0;          // BF16 row stride in elements (multiple of 8)
  int32_t ld8 = 0;           // FP8 row stride in bytes (multiple of 16)
  int32_t fp8_sc_off = -1;   // byte offset of the row's scale inside an FP8 row, or -1 (separate)
  int device = 0;

  float* X = nullptr;             // device [n][ldx]
  uint16_t* Xbf16 = nullptr;      // device [n][ld16]
  uint8_t* Xfp8 = nullptr;        // device [n][ld8]
  float* fp8_scale = nullptr;     // device [n]
  float xnorm_max = -1.0f;        // an upper bound of the rows' L2 norms (BF16 builds), else -1
  bool rerank_cut = true;         // the BF16 rerank's cut (fpp_debug_set_rerank_cut)
  float* center_vec = nullptr;    // device [d] centring vector (centred builds only)
  uint32_t* Xsig = nullptr;       // device [n][ldsig] SimHash signatures
  int32_t sigF = 0;               // hash functions in a signature
  int32_t ldsig = 0;              // signature row stride in 32-bit words (multiple of 4)
  const float* Xh = nullptr;      // hashing input of the build kernels ([n][ldx]): X, or X - c
  uint32_t* sign_mask = nullptr;  // device [L][l][3][P]: 0 or 0x80000000 (xor mask of the sign)
  uint32_t* sign_bits = nullptr;  // device [L][l][3][max(1, P / 32)]: bit j % 32 of word j / 32 set
                                  // when element j of the diagonal is -1
  uint32_t* offsets = nullptr;    // device [L][NB + 1], absolute positions into ids
  int32_t* ids = nullptr;         // device [total_ids]

  // Overflow bitmaps and work counters of the gather kernel for fpp_query / fpp_query_ex /
  // fpp_query_batch: up to kGbmSets sets, each allocated zeroed when a call finds every existing
  // set still in use, and kept zero by the kernel. A call takes the set last used on its own
  // stream, else a set whose last user has finished (its event has completed), else allocates
  // one, else waits (on its stream) for the set used longest ago; so calls on different streams
  // overlap up to kGbmSets deep, and calls on one stream share one set.
  // the gather deduplicates a query by id range when it has more probed entries than this
  int64_t part_min = kPartMinDefault;
  int32_t part_shift = kPartShiftDefault;   // ids per range: 2^part_shift (at most 2^18)
  static constexpr int64_t kPartMinDefault = 16384;
  static constexpr int32_t kPartShiftDefault = 18;
  static constexpr int kGbmSets = 4;
  mutable uint32_t* gbm[kGbmSets] = {};
  mutable hipEvent_t gbm_free[kGbmSets] = {};
  mutable hipStream_t gbm_stream[kGbmSets] = {};   // stream of the set's last user
  mutable uint64_t gbm_stamp[kGbmSets] = {};   // call counter when the set was last taken
  mutable uint64_t gbm_calls = 0;

  std::vector<int64_t> table_base;   // host [L + 1]
  int64_t total_ids = 0;
  int64_t max_bucket = 0;
  int64_t device_bytes = 0;
  double build_ms = 0.0;
};

namespace fpp {

// ----------------------------------------------------------------------------------------------
// Host-side helpers
// ----------------------------------------------------------------------------------------------
std::vector<uint32_t> make_sign_masks(uint64_t seed, int L, int l, int P);
// The same signs packed 32 to a word (layout of fpp_index::sign_bits).
std::vector<uint32_t> pack_sign_bits(const std::vector<uint32_t>& masks, int L, int l, int P);
int64_t keep_count_host(int64_t B, int64_t alpha_micro, int iProbes, int rounding);

// ----------------------------------------------------------------------------------------------
// Kernel launchers (each enqueues on `s`, returns hipError_t of the launch)
// ----------------------------------------------------------------------------------------------

// Build-side hash: records of tables [t0, t0 + Tc) for all n points.
//   rec_bucket / rec_key: [Tc][n * K] (slot r of point p at p * K + r).
hipError_t launch_hash_build(const fpp_index* ix, int t0, int Tc, uint32_t* rec_bucket,
                             float* rec_key, hipStream_t s);

// Query-side hash: sorted lists for m vectors (row stride ldv floats) and all L*l functions.
//   la: [m][L*l][D] float32, lc: [m][L*l][D] uint16 codes. Entries [0, W) of every list are
//   written (1 <= W <= D; the kernel may write up to a multiple of its per-lane run past W).
//   skip (optional, device [m]): vectors with skip[q] >= 0 are left out.
hipError_t launch_hash_query(const fpp_index* ix, const float* V, int64_t m, int ldv, float* la,
                             uint16_t* lc, int W, hipStream_t s, const int32_t* skip = nullptr);

// Fused query hashing and probe selection (probe budgets up to 2L, D == P <= 256, probe score
// FPP_PROBE_SUM): probes [m][qcap] and nprobe [m] as launch_probe_select writes them; a query the
// kernel cannot finish gets nprobe = -1 and is left to the list-based kernels.
bool hash_probe_applies(const fpp_index* ix, int32_t qp_max, int32_t probe_score, int32_t store);
hipError_t launch_hash_probe(const fpp_index* ix, const float* V, int64_t m, int ldv,
                             const int32_t* qp_arr, int32_t qp_uniform, int32_t qcap,
                             uint32_t* probes, int32_t* nprobe, hipStream_t s);

// Per-table build passes over a chunk of Tc tables.
struct BuildScratch {
  uint32_t* rec_bucket;   // [Tc][nK]
  float* rec_key;         // [Tc][nK]
  float* srt_key;         // [Tc][nK] records grouped by bucket
  int32_t* srt_id;        // [Tc][nK]
  uint32_t* cnt;          // [Tc][NB]
  uint32_t* start;        // [Tc][NB + 1]
  uint32_t* fill;         // [Tc][NB]
  uint64_t* meta;         // [2 + Tc]: running base, max bucket, per-table sizes
  uint64_t* tbase;        // [L + 1]: start of each table in the ids array
  uint64_t* large;        // [Tc][NB]: (table in chunk << 32 | bucket) of buckets > 64 records
  uint32_t* n_large;      // [1]
};
hipError_t launch_build_tables(const fpp_index* ix, int t0, int Tc, const BuildScratch& b,
                               hipStream_t s);

// Quantised stores.
hipError_t launch_quantize(const fpp_index* ix, hipStream_t s);
// SimHash signature words of m vectors from their sorted lists lc [m][lf][D] (the first F
// functions): out [m][ldsig], padding words zero.
hipError_t launch_pack_signs(const uint16_t* lc, int64_t m, int lf, int D, int F, int ldsig,
                             uint32_t* out, hipStream_t s);
// Centred copy of X (ix->center_vec must be set): Xc [n][ldx].
hipError_t launch_center(const fpp_index* ix, float* Xc, hipStream_t s);
// Standard normal quantile (Wichura's algorithm AS 241, PPND16), 0 < p < 1.
double normal_quantile(double p);

// Probe selection: probes [m][qcap] as absolute offset-array positions t * (NB + 1) + bucket;
// nprobe[m] receives the count per query. It reads list entries [0, probe_list_len) only.
int probe_list_len(const fpp_index* ix, int32_t qcap);
// only_unfinished: select only for the queries whose nprobe is negative (after the fused kernel).
hipError_t launch_probe_select(const fpp_index* ix, const float* la, const uint16_t* lc,
                               int64_t m, const int32_t* qp_arr, int32_t qp_uniform, int32_t qcap,
                               int32_t probe_score, uint32_t* probes, int32_t* nprobe, hipStream_t s,
                               bool only_unfinished = false);

// Candidate gather, dedup, scoring and top-k (plus the FP32 rerank of a short list).
struct ScoreArgs {
  const float* Q;          // [m][ldq]
  int ldq;
  int64_t m;
  const uint32_t* probes;  // [m][qcap]
  const int32_t* nprobe;   // [m]
  int32_t qcap;
  const int32_t* k_arr;    // [m] or null -> k_uniform
  int32_t k_uniform;
  const int64_t* out_off;  // [m] or null -> q * k_uniform
  int32_t store;           // FPP_STORE_*
  int32_t rerank_R;        // short list length option (low-precision stores); 0 -> max(100, 2k)
  int32_t* ids_out;
  float* scores_out;
  int32_t* short_ids;      // [m][short_ld] short lists (low-precision stores)
  float* short_sc;         // [m][short_ld] their approximate scores (-inf past the list)
  int32_t short_ld;
  float cut_c;             // > 0: the rerank's bound constant (launch_rerank); the gather then
                           // also drops candidates that the rerank could not keep
  int64_t* stats;          // [m][3] or null
  uint32_t* gbitmap;       // overflow dedup bitmaps [grid][ceil(n/32)], zero on entry and exit
  int32_t grid;            // persistent blocks
};
hipError_t launch_score(const fpp_index* ix, const ScoreArgs& a, hipStream_t s);
// bound_c > 0: |approximate - FP32 score| <= bound_c * ||q|| for every stored row, and short_sc
// holds the approximate scores; the rerank then skips the tail of a short list that cannot reach
// the top k (the result is the same). bound_c <= 0: every listed row is rescored.
hipError_t launch_rerank(const fpp_index* ix, const float* Q, int ldq, int64_t m,
                         const int32_t* short_ids, const float* short_sc, int short_ld,
                         float bound_c, const int32_t* k_arr, int k_uniform, int R_opt,
                         const int64_t* out_off, int32_t* ids_out, float* scores_out,
                         hipStream_t s);
// An upper bound of max_i ||x_i||_2 over the stored rows, as float bits (atomic max into *out,
// which the caller zeroes).
hipError_t launch_row_norm_max(const fpp_index* ix, uint32_t* out, hipStream_t s);
// The rerank bound constant of the BF16 store (see launch_rerank), or -1 if unknown.
float bf16_rerank_bound(const fpp_index* ix);
int score_grid_blocks(const fpp_index* ix);
int64_t overflow_bitmap_words(const fpp_index* ix);   // per score workgroup
int32_t short_list_len(int32_t R_opt, int32_t k);

// ----------------------------------------------------------------------------------------------
// Query pipeline (api.cpp), shared with the serving loop
// ----------------------------------------------------------------------------------------------
struct QuerySpec {
  const float* Q = nullptr;
  int64_t m = 0;
  int32_t k_uniform = 0, qp_uniform = 0;
  const int32_t* k_host = nullptr;     // per-query (host) or null
  const int32_t* qp_host = nullptr;
  const int32_t* k_dev = nullptr;      // per-query (device) or null
  const int32_t* qp_dev = nullptr;
  const int64_t* off_dev = nullptr;    // packed output offsets (device) or null
  int32_t k_max = 0, qp_max = 0;
  int32_t store = FPP_STORE_FP32;
  int32_t R_opt = 0;                   // rerank short-list length (0 = max(100, 2k))
  int32_t probe_score = FPP_PROBE_SUM;  // FPP_PROBE_*
  int32_t* ids_out = nullptr;
  float* scores_out = nullptr;
  int64_t* stats = nullptr;
  double* stage_ms = nullptr;          // host [4] or null
  uint32_t* gbm_ext = nullptr;         // caller-owned zeroed overflow bitmaps, or null (scratch)
};

struct Layout {
  int64_t mc = 0;         // queries per chunk
  int32_t qcap = 0;       // probes per query
  int32_t short_ld = 0;   // short-list row length
  bool gbm = false;       // overflow bitmaps live in the scratch (else the caller provides them)
  int grid = 0;
  size_t off_la = 0, off_lc = 0, off_probes = 0, off_np = 0, off_short = 0, off_qsig = 0, off_gbm = 0,
         total = 0;
};

size_t a256(size_t v);
int64_t total_pairs(const fpp_index* ix);
int check_store(const fpp_index* ix, int32_t store);
// Scratch layout for m queries; queries are processed in chunks so that one chunk's lists and
// probes stay within `budget` bytes.
Layout plan_layout(const fpp_index* ix, int64_t m, int32_t qp_max, int32_t k_max, int32_t store,
                   int32_t R_opt, int64_t budget = (int64_t)4 << 30, bool gbm_in_scratch = true);
// Bytes of the overflow bitmaps of one score launch and its work counters.
size_t overflow_bitmap_bytes(const fpp_index* ix);
// Runs hash -> probe selection -> score (-> rerank) over [0, qs.m) with device scratch `ws`
// laid out by `ly`. Per-query arrays of qs must already be on the device.
// `ev` (optional) receives 5 events per chunk: before hashing, after hashing, after probe
// selection, after scoring, after the rerank.
int run_queries(const fpp_index* ix, const QuerySpec& qs, const Layout& ly, unsigned char* ws,
                hipStream_t s, std::vector<hipEvent_t>* ev = nullptr);

}  // namespace fpp
