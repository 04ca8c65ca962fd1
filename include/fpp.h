/*
 * fpp.h — C ABI of the MI355X (gfx950) Falconn++ hot path.
 *
 * Falconn++ (Pham & Liu, NeurIPS 2022) answers top-k inner-product queries on
 * the unit sphere (Section 1, problem statement) with cross-polytope LSH
 * tables (Section 2.2, Eq. 1) whose buckets keep only the points with the
 * largest projections onto the bucket's random vector (Section 3.4, Algorithm 1),
 * probed across all tables in order of |q^T r_i| (Section 3.4, multi-probing
 * for querying).
 *
 * Conventions for every entry point:
 *   - Pointers documented as "device" point to memory on the current HIP device
 *     (for example torch.Tensor.data_ptr() of a cuda tensor); "host" pointers to
 *     ordinary process memory. Matrices are dense row-major.
 *   - The caller owns every buffer it passes; the library never frees or keeps
 *     a caller pointer beyond the call (the index copies X).
 *   - `stream` is a hipStream_t (NULL = the legacy default stream). Work is
 *     enqueued on it; outputs are valid once the stream has reached the point
 *     of the call. Entry points that return host data synchronise that stream.
 *   - Return value: FPP_OK (0) or a negative FPP_E* code. On error nothing has
 *     been written to the outputs and fpp_last_error() describes the failure.
 *     No C++ exception crosses this boundary.
 *   - An index is immutable after build: concurrent fpp_query calls on one index
 *     from several threads or streams are safe.
 *   - Inputs are assumed finite and unit-norm (Section 1); the library does not
 *     renormalise.
 */
#ifndef FPP_H
#define FPP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FPP_OK 0
#define FPP_EINVAL (-1)    /* an argument is out of range; nothing was enqueued        */
#define FPP_ENOMEM (-2)    /* a device or host allocation failed                        */
#define FPP_EHIP (-3)      /* a HIP runtime call failed                                 */
#define FPP_ECAPACITY (-4) /* a request exceeds a fixed capacity (pool, table limits)   */
#define FPP_ESTATE (-5)    /* the object is not in a state that allows the call         */

/* Scoring stores. The FP32 copy of X always exists (it gives exact scores and the rerank). */
#define FPP_STORE_FP32 0
#define FPP_STORE_BF16 1   /* x rounded to bfloat16, nearest-even                                */
#define FPP_STORE_FP8 2    /* per-vector scale s = max|x|/448; codes = OCP E4M3(x/s), nearest-even */
#define FPP_STORE_SIMHASH 3 /* SimHash signatures (Section 4, "Falconn++ parameter settings"): the
                               signs of the first D projections of the first F hash functions,
                               F*D bits; approximate score = F*D - 2 * Hamming distance          */

typedef struct fpp_index fpp_index;

/* Build options (fpp_default_build_opts fills the defaults shown). */
typedef struct fpp_build_opts {
  int32_t l;              /* cross-polytope functions concatenated per table: 1 or 2 (2). Section 4
                             uses 2, giving (2D)^2 buckets per table.                            */
  int32_t stores;         /* bit mask of extra low-precision stores to build: 1<<FPP_STORE_BF16,
                             1<<FPP_STORE_FP8, 1<<FPP_STORE_SIMHASH (0 = FP32 only)              */
  int32_t keep_rounding;  /* 0: a bucket of B records keeps ceil(alpha*B/iProbes) (default);
                             1: floor(...). alpha is taken to 6 decimals.                       */
  int32_t tables_per_pass;/* tables hashed and sorted per pass (0 = chosen from free memory)    */
  int32_t kappa;          /* limit scaling (Section 3.4, heuristic 2): a bucket keeps
                             min(B, max(kappa, keep(B))) records; 0 = off (default)             */
  int32_t center;         /* centering (Section 3.4, heuristic 1): 1 = hash x - c at build, with
                             c the mean of X (per coordinate: float64 sum in row order, divided by
                             n in float64, rounded to float32); queries are hashed as given and
                             scores stay x^T q on the uncentred X; 0 = off (default)            */
  int32_t filter;         /* FPP_FILTER_FRACTION (0): the per-bucket top fraction of Algorithm 1;
                             FPP_FILTER_THRESHOLD (1): the global threshold of the theoretical
                             LSF comparison (appendix, "Falconn++ vs. theoretical LSF"): a record
                             is kept when each of its l projections, divided by P, is >= t       */
  float threshold;        /* t for FPP_FILTER_THRESHOLD; <= 0: t = Phi^-1(1 - alpha^(1/l) / (2D)),
                             so that a point reaches a given bucket with probability alpha/(2D)^l
                             for Gaussian projections (Phi^-1 by Wichura's algorithm AS 241)    */
  int32_t simhash_functions; /* F for FPP_STORE_SIMHASH: hash functions (t * l + f order) whose
                             projection signs form a signature; a multiple of l with
                             F * D <= 1024; 0 = the largest multiple of l with F * D <= 256
                             (at least l)                                                       */
} fpp_build_opts;

#define FPP_FILTER_FRACTION 0
#define FPP_FILTER_THRESHOLD 1

#define FPP_PROBE_SUM 0
#define FPP_PROBE_GAP 1

void fpp_default_build_opts(fpp_build_opts* opts);

/*
 * Build an index over X (Algorithm 1 applied to each of L tables).
 *   X       device, float32 [n][d]; copied into the index (caller may free it after return).
 *   n       number of points, 1 <= n < 2^31.
 *   d       dimension, 1 <= d <= 1024.
 *   L       number of tables, 1 <= L <= 4096.
 *   D       random vectors per cross-polytope function (2D codes), a power of two,
 *           2 <= D <= 2048; the rotation length is P = max(D, 2^ceil(log2 d)) <= 4096.
 *   alpha   fraction of every bucket that is kept, 0 < alpha <= 1 (Section 3.4).
 *   iProbes buckets per point and table before filtering, 1 <= iProbes <= min(16, D^l)
 *           (Algorithm 1, multi-probe indexing).
 *   seed    seeds the random sign diagonals of the rotation (SplitMix64 counter stream).
 *   out     host, receives the new index.
 * fpp_build_index uses the default options and the default stream and returns after
 * the build has finished. Errors: FPP_EINVAL (ranges), FPP_ENOMEM, FPP_EHIP,
 * FPP_ECAPACITY (more than 2^32 - 1 stored ids in total).
 */
int fpp_build_index(const float* X, int64_t n, int32_t d, int32_t L, int32_t D, float alpha,
                    int32_t iProbes, uint64_t seed, fpp_index** out);
int fpp_build_index_ex(const float* X, int64_t n, int32_t d, int32_t L, int32_t D, float alpha,
                       int32_t iProbes, uint64_t seed, const fpp_build_opts* opts, void* stream,
                       fpp_index** out);

/* Release an index and its device memory (NULL is ignored). The caller must ensure no
 * enqueued query still uses it. */
void fpp_free_index(fpp_index* index);

/* Query options (fpp_default_query_opts fills the defaults shown). */
typedef struct fpp_query_opts {
  int32_t store;       /* store scored during the candidate pass: FPP_STORE_FP32 (exact scores, 0),
                          FPP_STORE_BF16, FPP_STORE_FP8 or FPP_STORE_SIMHASH (approximate;
                          requires that store)                                                  */
  int32_t rerank_R;    /* low-precision stores: short-list length re-scored exactly in FP32
                          (0 = max(100, 2k)); k <= R <= 512. -1: no rerank, the top-k of the
                          low-precision pass is returned with its approximate scores           */
  int64_t* stats;      /* optional device int64 [m][3]: probes, probed entries (with repeats),
                          unique candidates scored                                               */
  double* stage_ms;    /* optional host double [4]: milliseconds spent in hashing, probe
                          selection, gather/score/top-k and rerank, from HIP events recorded on
                          `stream` around each kernel; when set, the call synchronises `stream`  */
  int32_t probe_score; /* FPP_PROBE_SUM (0): a bucket's probe score is the sum of its |projections|
                          (Section 3.4, Falconn++); FPP_PROBE_GAP (1): that sum minus the best
                          pair of its table, the multi-probe score of plain Falconn (Section 2.2);
                          both ranked globally over the L tables                              */
} fpp_query_opts;

void fpp_default_query_opts(fpp_query_opts* opts);

/*
 * Top-k search for m queries (Section 3.4, multi-probing for querying; Section 1).
 *   Q          device, float32 [m][d] (d of the index).
 *   m          number of queries, m >= 0 (0 enqueues nothing).
 *   k          results per query, 1 <= k <= 512.
 *   qProbes    total number of (table, bucket) probes per query over all L tables, ranked by
 *              the sum of the query's |projections| (clamped to L * D^l); >= 1.
 *   ids_out    device, int32 [m][k]: ids by (score desc, id asc); -1 pads short results.
 *   scores_out device, float32 [m][k]: FP32 inner products q^T x on the stored FP32 X
 *              (after a low-precision pass, the exact FP32 rerank scores); -inf pads.
 * Scratch memory is taken from the stream-ordered allocator on `stream`. The first query also
 * allocates the gather's overflow bitmaps (n / 8 bytes per workgroup of its persistent grid,
 * 768 workgroups on MI355X), which the index keeps, zero, until fpp_free_index; calls on
 * different streams take turns on them (a call's stream waits for the previous call's work).
 * Errors: FPP_EINVAL, FPP_ENOMEM, FPP_EHIP, FPP_ESTATE (requested store not built).
 */
int fpp_query(const fpp_index* index, const float* Q, int64_t m, int32_t k, int32_t qProbes,
              int32_t* ids_out, float* scores_out, void* stream);
int fpp_query_ex(const fpp_index* index, const float* Q, int64_t m, int32_t k, int32_t qProbes,
                 const fpp_query_opts* opts, int32_t* ids_out, float* scores_out, void* stream);

/*
 * fpp_query_ex for callers that cannot allocate (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): the same results as fpp_query_ex with the same
 * arguments, but no call to hipMalloc, hipMallocAsync, hipFree or any allocating routine. Every
 * per-call buffer lives in one static device array of 128 MiB, which each device that loads the
 * library holds until the process ends: the gather's overflow dedup bitmaps (n / 8 bytes per
 * workgroup; the gather runs on as many workgroups, at most its usual grid, as have a bitmap
 * within 32 MiB) and the lists, probes and short lists of one chunk of queries (any m is taken
 * in chunks that fit). A fill kernel on `stream` clears the bitmaps and work counters at the
 * start of each call. All calls on one device share the array: calls whose work overlaps on a
 * device (other threads, other streams) race and must be serialised by the caller.
 * opts->stage_ms must be NULL. Errors: as fpp_query_ex, FPP_EINVAL for stage_ms, and
 * FPP_ECAPACITY when one overflow bitmap exceeds 32 MiB (n > 268,435,455) or one query's
 * scratch does not fit beside the bitmaps.
 */
int fpp_query_ex_noalloc(const fpp_index* index, const float* Q, int64_t m, int32_t k,
                         int32_t qProbes, const fpp_query_opts* opts, int32_t* ids_out,
                         float* scores_out, void* stream);

/*
 * Mixed batch in one launch sequence: query i uses k[i] and qProbes[i] (host arrays of m
 * entries, same ranges as above) and writes its k[i] results at ids_out + off_i and
 * scores_out + off_i with off_i = k[0] + ... + k[i-1] (packed). Other arguments as fpp_query_ex.
 * A query's result does not depend on the other queries of the batch.
 */
int fpp_query_batch(const fpp_index* index, const float* Q, int64_t m, const int32_t* k,
                    const int32_t* qProbes, const fpp_query_opts* opts, int32_t* ids_out,
                    float* scores_out, void* stream);

/* Bytes of scratch memory fpp_query_batch needs for m queries with the given maxima (besides
   the overflow bitmaps the index keeps). */
int64_t fpp_query_workspace_bytes(const fpp_index* index, int64_t m, int32_t k_max,
                                  int32_t qprobes_max, const fpp_query_opts* opts);

/* Facts about a built index (host struct). */
typedef struct fpp_index_info {
  int64_t n;
  int32_t d, L, D, l, P, iProbes;
  int32_t stores;          /* bit mask of built low-precision stores               */
  float alpha;
  uint64_t seed;
  int64_t buckets_per_table;
  int64_t total_ids;       /* stored ids over all tables                            */
  int64_t max_bucket;      /* largest kept bucket                                   */
  int64_t device_bytes;    /* device memory held by the index                       */
  double build_ms;         /* wall time of the build call                           */
  int32_t kappa;           /* limit scaling of the build (0 = off)                  */
  int32_t centered;        /* 1 if the build hashed x - c                           */
  int32_t filter;          /* FPP_FILTER_*                                           */
  float threshold;         /* FPP_FILTER_THRESHOLD: the float32 bound on |y| the build
                              compared against (fl32(P * t)); 0 otherwise             */
  int32_t simhash_bits;    /* F * D of the SimHash store (0 if not built)           */
  int32_t overflow_sets;   /* sets of gather overflow bitmaps allocated so far: a query call
                              takes one whose last call has finished, else a new one (up to 4),
                              so calls in flight on different streams do not wait for each other */
} fpp_index_info;

int fpp_index_get_info(const fpp_index* index, fpp_index_info* info);
/* host int64 [L]: ids stored per table. */
int fpp_index_table_sizes(const fpp_index* index, int64_t* sizes_out);

/* Standard normal quantile Phi^-1(p) for 0 < p < 1 (NaN otherwise), by Wichura's algorithm
 * AS 241 (PPND16); the threshold filter derives its bound from alpha with it. Host only. */
double fpp_normal_quantile(double p);

const char* fpp_last_error(void);   /* message of the last failed call on this thread */
const char* fpp_version(void);

/* ------------------------------------------------------------------------------------------
 * Serving: a persistent request loop over one resident index (continuous batching).
 * Requests of mixed m, k and qProbes are admitted first-in first-out while the scratch
 * pool and a stream slot are free, packed into one launch sequence with per-query
 * parameters, and run on `n_streams` streams so that batches overlap on the device.
 * ------------------------------------------------------------------------------------------ */
typedef struct fpp_server fpp_server;

typedef struct fpp_server_opts {
  int64_t scratch_bytes;   /* scratch pool shared by in-flight batches (>= one request's need) */
  int32_t n_streams;       /* batches in flight at once, 1..8                                   */
  int32_t max_batch;       /* queries packed into one launch, >= 1                              */
  int32_t store;           /* as fpp_query_opts.store                                           */
  int32_t rerank_R;        /* as fpp_query_opts.rerank_R                                        */
  int32_t probe_score;     /* as fpp_query_opts.probe_score                                     */
} fpp_server_opts;

void fpp_default_server_opts(fpp_server_opts* opts);

/* Start the loop thread. The index must outlive the server. */
int fpp_server_create(const fpp_index* index, const fpp_server_opts* opts, fpp_server** out);

/*
 * Submit one request: Q device float32 [m][d]; ids_out / scores_out device [m][k].
 * The buffers must stay valid until the request completes. The server's streams are not
 * ordered after any stream of the caller: Q must already hold its values, and no pending work
 * may write to ids_out / scores_out, when the call is made (synchronise the producing stream
 * first). Returns a ticket (> 0) in *ticket. Errors: FPP_EINVAL, FPP_ECAPACITY (the request alone needs more scratch than
 * the pool holds), FPP_ESTATE (server stopping).
 */
int fpp_server_submit(fpp_server* server, const float* Q, int32_t m, int32_t k, int32_t qProbes,
                      int32_t* ids_out, float* scores_out, int64_t* ticket);

/* Request state: *status = 0 done, 1 pending, < 0 failed (an FPP_E* code). Times are
 * CLOCK_MONOTONIC nanoseconds of submission and of completion (0 while pending). */
int fpp_server_poll(fpp_server* server, int64_t ticket, int32_t* status, int64_t* t_submit_ns,
                    int64_t* t_done_ns);
/* Block until the request completes or timeout_ms passes (< 0: no limit). */
int fpp_server_wait(fpp_server* server, int64_t ticket, int64_t timeout_ms, int32_t* status,
                    int64_t* t_submit_ns, int64_t* t_done_ns);

typedef struct fpp_server_stats {
  int64_t submitted, completed, failed, batches, queries;
  int64_t max_inflight_batches;   /* largest number of batches on the device at once */
  int64_t scratch_high_water;     /* largest scratch in use at once (bytes)          */
} fpp_server_stats;
int fpp_server_get_stats(fpp_server* server, fpp_server_stats* stats);

/*
 * Open-loop load generator for measuring the server: request i (i < n_req) is submitted as
 * fpp_server_submit would, at CLOCK_MONOTONIC time t0_ns + arrive_ns[i] (the call spins until
 * then; late requests go at once), with queries Q[q_row[i] .. q_row[i] + m[i]) (Q device float32
 * [*][d] of the index), k[i] and qProbes[i], and results at ids_out + out_off[i] and
 * scores_out + out_off[i] (device, m[i] * k[i] values each). Host arrays of n_req entries;
 * tickets[i] receives the ticket. Returns when the last request is submitted (not completed), or
 * at the first failed submission with its error (tickets of the requests not submitted are 0).
 * Latency of request i = completion time - (t0_ns + arrive_ns[i]), queueing included.
 */
int fpp_server_replay(fpp_server* server, const float* Q, int64_t n_req, int64_t t0_ns,
                      const int64_t* arrive_ns, const int64_t* q_row, const int32_t* m,
                      const int32_t* k, const int32_t* qProbes, int32_t* ids_out,
                      float* scores_out, const int64_t* out_off, int64_t* tickets);

/* For tests of failure handling: the next n batches the loop launches fail after their first
 * kernel is on the stream, as a failing HIP call would leave them. Each such batch's requests
 * complete with status FPP_EHIP, its scratch returns to the pool, and the loop goes on admitting
 * and serving later requests. n = 0 cancels. Errors: FPP_EINVAL. */
int fpp_server_debug_fail_batches(fpp_server* server, int32_t n);

/* Stop accepting work, finish what was admitted, join the loop thread and free it. */
void fpp_server_destroy(fpp_server* server);

/* ------------------------------------------------------------------------------------------
 * Inspection entry points (used by the parity tests; not on the query path).
 * ------------------------------------------------------------------------------------------ */

/* host int8 [L][l][3][P]: the +-1 sign diagonals of the rotation (Section 3.4). */
int fpp_debug_signs(const fpp_index* index, int8_t* signs_out);

/* Query-side hash lists: for every vector of V (device float32 [m][d]) and every (table t,
 * function f), the D entries sorted by (|y_i| desc, i asc): abs_out device float32 and
 * code_out device int32, both [m][L][l][D]; code = i if y_i >= 0 else i + D (Eq. 1). */
int fpp_debug_query_lists(const fpp_index* index, const float* V, int64_t m, float* abs_out,
                          int32_t* code_out, void* stream);

/* As fpp_debug_query_lists, but the hash kernel stores only what the query path stores for a
 * probe selection that reads the first W entries of every list (1 <= W <= D, else FPP_EINVAL):
 * positions [0, W) of each list are defined, later positions are unspecified. */
int fpp_debug_query_list_prefix(const fpp_index* index, const float* V, int64_t m, int32_t W,
                                float* abs_out, int32_t* code_out, void* stream);

/* Build-side records of table t: for every point p and r < iProbes, the bucket and key of its
 * r-th best pair (device uint32 bucket_out / float32 key_out, [n][iProbes]). */
int fpp_debug_build_records(const fpp_index* index, int32_t t, uint32_t* bucket_out,
                            float* key_out, void* stream);

/* CSR of table t: host uint32 offsets_out [(2D)^l + 1] (relative to the table start) and
 * host int32 ids_out [table size]. Synchronises. */
int fpp_debug_export_table(const fpp_index* index, int32_t t, uint32_t* offsets_out,
                           int32_t* ids_out);

/* The selected probes of each query: device int64 [m][qProbes'] with qProbes' = min(qProbes,
 * L * D^l), each t * (2D)^l + bucket, in no particular order; probe_score as in
 * fpp_query_opts. */
int fpp_debug_probes(const fpp_index* index, const float* Q, int64_t m, int32_t qProbes,
                     int32_t probe_score, int64_t* probes_out, void* stream);

/* host float [d]: the centring vector c of a centred index (zeros otherwise). */
int fpp_debug_center(const fpp_index* index, float* c_out);

/* A low-precision store: store FPP_STORE_BF16 -> device uint16 [n][d]; FPP_STORE_FP8 -> device
 * uint8 [n][d] codes plus device float32 [n] scales (scales_out ignored for BF16 and SimHash);
 * FPP_STORE_SIMHASH -> device uint32 [n][ceil(F*D/32)] signature words (bit b of a signature is
 * word b / 32, bit b % 32; b = g * D + i is set when projection i of function g is negative). */
int fpp_debug_export_store(const fpp_index* index, int32_t store, void* codes_out,
                           float* scales_out, void* stream);

/* For tests of the gather's dedup (Section 4: candidates are deduplicated, each scored once):
 * queries of this index with more than min_entries probed entries, and no more than n / 32,
 * are deduplicated by id range (ids grouped by id >> range_bits, each group against an on-chip
 * bitmap of 2^range_bits bits; at most 256 groups) instead of the on-chip set that spills into
 * a device bitmap. Both give the same results. min_entries < 0 restores the default (16,384),
 * range_bits < 0 the default (18); otherwise range_bits must lie in [5, 18]. Not thread-safe
 * against running queries on the index. Errors: FPP_EINVAL. */
int fpp_debug_set_partition_threshold(fpp_index* index, int64_t min_entries, int32_t range_bits);

/* For tests of the BF16 rerank: with a BF16 store, the rerank rescores only the head of a short
 * list that can still reach the top k (rows below the k-th approximate score by more than twice
 * a bound on |approximate - FP32 score| cannot), and the gather drops such candidates as it
 * scores; the results are the same as rescoring every listed row. enabled = 0 turns both off
 * (every short-listed row is rescored), 1 (the default) on. Not thread-safe against running
 * queries on the index. Errors: FPP_EINVAL. */
int fpp_debug_set_rerank_cut(fpp_index* index, int32_t enabled);

#ifdef __cplusplus
}
#endif

#endif /* FPP_H */
