// Serving: a persistent request loop over one resident index (continuous batching).
//
// Requests (m queries each, with their own k and qProbes) wait in a FIFO. The loop thread
// admits requests from the head while a stream slot is free and the batch's scratch fits in
// the remaining part of a fixed device pool; the admitted requests are packed into one launch
// sequence with per-query k / qProbes / output offsets:
//   pack kernel (request rows -> one query matrix) -> hash -> probe selection -> score
//   (-> FP32 rerank) -> scatter kernel (packed results -> each request's buffers) -> event.
// Batches run on `n_streams` streams, so a batch admitted while others are on the device
// overlaps with them. When a batch's event completes, its requests are stamped and its scratch
// returns to the pool. A query's result does not depend on its batch (per-query kernels with
// fixed reduction trees and total orders).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <time.h>

#include "fpp_internal.hpp"
#include "server_pool.hpp"

namespace fpp {
namespace {

int64_t now_ns() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (int64_t)ts.tv_sec * 1000000000LL + ts.tv_nsec;
}

struct QueryDesc {
  const float* src;   // query row in the request's buffer
  int32_t* ids;       // destination of this query's k ids
  float* scores;
};

__global__ __launch_bounds__(256) void pack_kernel(const QueryDesc* __restrict__ desc, int64_t m,
                                                   int d, float* __restrict__ Qp) {
  const int64_t q = blockIdx.x;
  if (q >= m) return;
  const float* src = desc[q].src;
  for (int j = threadIdx.x; j < d; j += 256) Qp[q * d + j] = src[j];
}

__global__ __launch_bounds__(256) void scatter_kernel(const QueryDesc* __restrict__ desc,
                                                      const int64_t* __restrict__ off,
                                                      const int32_t* __restrict__ karr, int64_t m,
                                                      const int32_t* __restrict__ ids_p,
                                                      const float* __restrict__ sc_p) {
  const int64_t q = blockIdx.x;
  if (q >= m) return;
  const int64_t o = off[q];
  const int k = karr[q];
  for (int r = threadIdx.x; r < k; r += 256) {
    desc[q].ids[r] = ids_p[o + r];
    desc[q].scores[r] = sc_p[o + r];
  }
}

struct Request {
  int64_t ticket = 0;
  const float* Q = nullptr;
  int32_t m = 0, k = 0, qp = 0;
  int32_t* ids = nullptr;
  float* scores = nullptr;
  int64_t t_submit = 0, t_done = 0;
  int32_t status = 1;   // 1 pending, 0 done, < 0 error
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  bool busy = false;
  // per-slot buffers sized for max_batch queries
  QueryDesc* h_desc = nullptr;    // pinned
  int64_t* h_off = nullptr;       // pinned [m]
  int32_t* h_kq = nullptr;        // pinned [2m]: k then qProbes
  QueryDesc* d_desc = nullptr;
  int64_t* d_off = nullptr;
  int32_t* d_kq = nullptr;
  float* d_Q = nullptr;           // [max_batch][d]
  int32_t* d_ids = nullptr;       // [max_batch * kMaxK]
  float* d_sc = nullptr;
  uint32_t* d_gbm = nullptr;      // overflow dedup bitmaps of this slot's launches (kept zero)
  size_t ws_off = 0, ws_bytes = 0;
  std::vector<std::shared_ptr<Request>> reqs;
};

}  // namespace
}  // namespace fpp

struct fpp_server {
  const fpp_index* ix = nullptr;
  fpp_server_opts opts{};
  unsigned char* pool_mem = nullptr;
  fpp::Pool pool;
  std::vector<fpp::Slot> slots;
  std::mutex mu;
  std::condition_variable cv;       // new work / stop
  std::condition_variable done_cv;  // request completions
  std::deque<std::shared_ptr<fpp::Request>> queue;
  std::map<int64_t, std::shared_ptr<fpp::Request>> live;
  int64_t next_ticket = 1;
  bool stopping = false;
  std::thread loop;
  fpp_server_stats stats{};
  int device = 0;
  std::atomic<int32_t> fail_batches{0};   // batches still to fail on request (tests)
};

namespace fpp {
namespace {

size_t batch_bytes(const fpp_index* ix, const fpp_server_opts& o, int64_t m, int32_t kmax,
                   int32_t qpmax) {
  return plan_layout(ix, m, qpmax, kmax, o.store, o.rerank_R, INT64_MAX, false).total;
}

void release_slot_buffers(Slot& s) {
  if (s.h_desc) (void)hipHostFree(s.h_desc);
  if (s.h_off) (void)hipHostFree(s.h_off);
  if (s.h_kq) (void)hipHostFree(s.h_kq);
  void* d[] = {s.d_desc, s.d_off, s.d_kq, s.d_Q, s.d_ids, s.d_sc, s.d_gbm};
  for (void* p : d)
    if (p) (void)hipFree(p);
  if (s.done) (void)hipEventDestroy(s.done);
  if (s.stream) (void)hipStreamDestroy(s.stream);
  s = Slot{};
}

// Launch one admitted batch on slot `s` (called with the server lock released).
int launch_batch(fpp_server* sv, Slot& s) {
  const fpp_index* ix = sv->ix;
  int64_t m = 0, off = 0;
  int32_t kmax = 0, qpmax = 0;
  for (auto& r : s.reqs) {
    for (int32_t i = 0; i < r->m; ++i) {
      s.h_desc[m] = QueryDesc{r->Q + (size_t)i * ix->d, r->ids + (size_t)i * r->k,
                              r->scores + (size_t)i * r->k};
      s.h_off[m] = off;
      s.h_kq[m] = r->k;
      off += r->k;
      ++m;
    }
    kmax = std::max(kmax, r->k);
    qpmax = std::max(qpmax, r->qp);
  }
  int64_t j = 0;
  for (auto& r : s.reqs)
    for (int32_t i = 0; i < r->m; ++i) s.h_kq[m + j++] = r->qp;
  hipStream_t st = s.stream;
  FPP_HIP(hipMemcpyAsync(s.d_desc, s.h_desc, sizeof(QueryDesc) * m, hipMemcpyHostToDevice, st));
  FPP_HIP(hipMemcpyAsync(s.d_off, s.h_off, sizeof(int64_t) * m, hipMemcpyHostToDevice, st));
  FPP_HIP(hipMemcpyAsync(s.d_kq, s.h_kq, sizeof(int32_t) * 2 * m, hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(pack_kernel, dim3((unsigned)m), dim3(256), 0, st, s.d_desc, m, ix->d, s.d_Q);
  FPP_HIP(hipGetLastError());
  {
    // a failure requested by fpp_server_debug_fail_batches, at the point where a failing HIP call
    // would leave the batch: part of its work is already on the stream
    int32_t f = sv->fail_batches.load();
    while (f > 0 && !sv->fail_batches.compare_exchange_weak(f, f - 1)) {
    }
    if (f > 0) return set_error("batch failed on request"), FPP_EHIP;
  }
  QuerySpec qs;
  qs.Q = s.d_Q;
  qs.m = m;
  qs.k_dev = s.d_kq;
  qs.qp_dev = s.d_kq + m;
  qs.off_dev = s.d_off;
  qs.k_max = kmax;
  qs.qp_max = qpmax;
  qs.store = sv->opts.store;
  qs.R_opt = sv->opts.rerank_R;
  qs.probe_score = sv->opts.probe_score;
  qs.ids_out = s.d_ids;
  qs.scores_out = s.d_sc;
  const Layout ly = plan_layout(ix, m, qpmax, kmax, qs.store, qs.R_opt, INT64_MAX, false);
  qs.gbm_ext = s.d_gbm;
  unsigned char* ws = sv->pool_mem + s.ws_off;
  FPP_TRY(run_queries(ix, qs, ly, ws, st));
  hipLaunchKernelGGL(scatter_kernel, dim3((unsigned)m), dim3(256), 0, st, s.d_desc, s.d_off, s.d_kq,
                     m, s.d_ids, s.d_sc);
  FPP_HIP(hipGetLastError());
  FPP_HIP(hipEventRecord(s.done, st));
  return FPP_OK;
}

void server_loop(fpp_server* sv) {
  (void)hipSetDevice(sv->device);
  std::unique_lock<std::mutex> lk(sv->mu);
  for (;;) {
    // 1. retire finished batches
    int inflight = 0;
    for (auto& s : sv->slots) {
      if (!s.busy) continue;
      const hipError_t q = hipEventQuery(s.done);
      if (q == hipErrorNotReady) {
        ++inflight;
        continue;
      }
      const int64_t t = now_ns();
      for (auto& r : s.reqs) {
        r->t_done = t;
        r->status = q == hipSuccess ? 0 : FPP_EHIP;
        if (q == hipSuccess) ++sv->stats.completed;
        else ++sv->stats.failed;
      }
      s.reqs.clear();
      sv->pool.release(s.ws_off, s.ws_bytes);
      s.busy = false;
      sv->done_cv.notify_all();
    }
    // 2. admit FIFO while a slot and scratch are free
    for (auto& s : sv->slots) {
      if (s.busy || sv->queue.empty()) continue;
      const Admitted a = admit_fifo(
          sv->queue.begin(), sv->queue.end(), sv->opts.max_batch, sv->pool,
          [](const std::shared_ptr<Request>& r) { return AdmitShape{r->m, r->k, r->qp}; },
          [sv](int64_t m, int32_t k, int32_t qp) { return batch_bytes(sv->ix, sv->opts, m, k, qp); });
      if (a.taken == 0) break;   // the head waits for scratch
      s.reqs.assign(sv->queue.begin(), sv->queue.begin() + (std::ptrdiff_t)a.taken);
      sv->queue.erase(sv->queue.begin(), sv->queue.begin() + (std::ptrdiff_t)a.taken);
      s.ws_off = a.offset;
      s.ws_bytes = a.bytes;
      s.busy = true;
      ++sv->stats.batches;
      sv->stats.queries += a.m;
      lk.unlock();
      const int rc = launch_batch(sv, s);
      lk.lock();
      if (rc != FPP_OK) {
        // the stream may hold part of the batch: wait for it, then fail the requests
        lk.unlock();
        (void)hipStreamSynchronize(s.stream);
        lk.lock();
        const int64_t t = now_ns();
        for (auto& r : s.reqs) {
          r->t_done = t;
          r->status = rc;
          ++sv->stats.failed;
        }
        s.reqs.clear();
        sv->pool.release(s.ws_off, s.ws_bytes);
        s.busy = false;
        sv->done_cv.notify_all();
      } else {
        ++inflight;
      }
    }
    sv->stats.max_inflight_batches = std::max<int64_t>(sv->stats.max_inflight_batches, inflight);
    sv->stats.scratch_high_water = (int64_t)sv->pool.high_water();
    if (sv->stopping && sv->queue.empty() && inflight == 0) break;
    if (inflight > 0) {
      // poll the device for completions
      sv->cv.wait_for(lk, std::chrono::microseconds(20));
    } else {
      sv->cv.wait(lk, [sv] { return sv->stopping || !sv->queue.empty(); });
    }
  }
}

}  // namespace
}  // namespace fpp

using namespace fpp;

extern "C" {

void fpp_default_server_opts(fpp_server_opts* o) {
  if (!o) return;
  o->scratch_bytes = (int64_t)2 << 30;
  o->n_streams = 2;
  o->max_batch = 1024;
  o->store = FPP_STORE_FP32;
  o->rerank_R = 0;
  o->probe_score = FPP_PROBE_SUM;
}

int fpp_server_create(const fpp_index* ix, const fpp_server_opts* opts, fpp_server** out) {
  if (!ix || !out) return set_error("NULL argument"), FPP_EINVAL;
  fpp_server_opts o;
  fpp_default_server_opts(&o);
  if (opts) o = *opts;
  if (o.n_streams < 1 || o.n_streams > 8) return set_error("n_streams=%d out of [1, 8]", o.n_streams), FPP_EINVAL;
  if (o.max_batch < 1) return set_error("max_batch=%d < 1", o.max_batch), FPP_EINVAL;
  if (o.scratch_bytes < 1) return set_error("scratch_bytes < 1"), FPP_EINVAL;
  if (o.rerank_R < -1 || o.rerank_R > kMaxK) return set_error("rerank_R out of range"), FPP_EINVAL;
  if (o.probe_score != FPP_PROBE_SUM && o.probe_score != FPP_PROBE_GAP)
    return set_error("unknown probe_score %d", o.probe_score), FPP_EINVAL;
  FPP_TRY(check_store(ix, o.store));
  std::unique_ptr<fpp_server> sv(new fpp_server());
  sv->ix = ix;
  sv->opts = o;
  FPP_HIP(hipGetDevice(&sv->device));
  sv->slots.resize(o.n_streams);
  auto fail = [&](int rc) {
    for (auto& s : sv->slots) release_slot_buffers(s);
    if (sv->pool_mem) (void)hipFree(sv->pool_mem);
    return rc;
  };
  hipError_t e = hipMalloc((void**)&sv->pool_mem, (size_t)o.scratch_bytes);
  if (e != hipSuccess) return fail(hip_fail(e, "hipMalloc(pool)", __FILE__, __LINE__));
  sv->pool.init((size_t)o.scratch_bytes);
  const size_t mb = (size_t)o.max_batch;
  for (auto& s : sv->slots) {
    // default priority (no priority streams)
    if ((e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming)) != hipSuccess ||
        (e = hipHostMalloc((void**)&s.h_desc, sizeof(QueryDesc) * mb, hipHostMallocDefault)) != hipSuccess ||
        (e = hipHostMalloc((void**)&s.h_off, sizeof(int64_t) * mb, hipHostMallocDefault)) != hipSuccess ||
        (e = hipHostMalloc((void**)&s.h_kq, sizeof(int32_t) * 2 * mb, hipHostMallocDefault)) != hipSuccess ||
        (e = hipMalloc((void**)&s.d_desc, sizeof(QueryDesc) * mb)) != hipSuccess ||
        (e = hipMalloc((void**)&s.d_off, sizeof(int64_t) * mb)) != hipSuccess ||
        (e = hipMalloc((void**)&s.d_kq, sizeof(int32_t) * 2 * mb)) != hipSuccess ||
        (e = hipMalloc((void**)&s.d_Q, sizeof(float) * mb * ix->d)) != hipSuccess ||
        (e = hipMalloc((void**)&s.d_ids, sizeof(int32_t) * mb * kMaxK)) != hipSuccess ||
        (e = hipMalloc((void**)&s.d_sc, sizeof(float) * mb * kMaxK)) != hipSuccess ||
        (e = hipMalloc((void**)&s.d_gbm, overflow_bitmap_bytes(ix))) != hipSuccess ||
        (e = hipMemset(s.d_gbm, 0, overflow_bitmap_bytes(ix))) != hipSuccess)
      return fail(hip_fail(e, "server slot allocation", __FILE__, __LINE__));
  }
  fpp_server* raw = sv.get();
  raw->loop = std::thread(server_loop, raw);
  *out = sv.release();
  return FPP_OK;
}

int fpp_server_submit(fpp_server* sv, const float* Q, int32_t m, int32_t k, int32_t qProbes,
                      int32_t* ids_out, float* scores_out, int64_t* ticket) {
  if (!sv || !ticket) return set_error("NULL argument"), FPP_EINVAL;
  if (m < 1 || !Q || !ids_out || !scores_out) return set_error("empty request or NULL buffer"), FPP_EINVAL;
  if (m > sv->opts.max_batch) return set_error("m=%d exceeds max_batch=%d", m, sv->opts.max_batch), FPP_ECAPACITY;
  if (k < 1 || k > kMaxK) return set_error("k=%d out of [1, %d]", k, kMaxK), FPP_EINVAL;
  if (qProbes < 1) return set_error("qProbes < 1"), FPP_EINVAL;
  if (sv->opts.store != FPP_STORE_FP32 && sv->opts.rerank_R > 0 && sv->opts.rerank_R < k)
    return set_error("rerank_R < k"), FPP_EINVAL;
  const size_t need = batch_bytes(sv->ix, sv->opts, m, k, qProbes);
  if (a256(need) > sv->pool.capacity())
    return set_error("request needs %zu scratch bytes, pool holds %zu", need, sv->pool.capacity()), FPP_ECAPACITY;
  auto r = std::make_shared<Request>();
  r->Q = Q;
  r->m = m;
  r->k = k;
  r->qp = qProbes;
  r->ids = ids_out;
  r->scores = scores_out;
  {
    std::lock_guard<std::mutex> g(sv->mu);
    if (sv->stopping) return set_error("server is stopping"), FPP_ESTATE;
    r->ticket = sv->next_ticket++;
    r->t_submit = now_ns();
    sv->live[r->ticket] = r;
    sv->queue.push_back(r);
    ++sv->stats.submitted;
    *ticket = r->ticket;
  }
  sv->cv.notify_all();
  return FPP_OK;
}

static int report(fpp_server* sv, std::map<int64_t, std::shared_ptr<Request>>::iterator it,
                  int32_t* status, int64_t* ts, int64_t* td) {
  Request& r = *it->second;
  if (status) *status = r.status;
  if (ts) *ts = r.t_submit;
  if (td) *td = r.t_done;
  if (r.status != 1) sv->live.erase(it);   // a completed ticket is reported once
  return FPP_OK;
}

int fpp_server_poll(fpp_server* sv, int64_t ticket, int32_t* status, int64_t* t_submit_ns,
                    int64_t* t_done_ns) {
  if (!sv) return set_error("NULL argument"), FPP_EINVAL;
  std::lock_guard<std::mutex> g(sv->mu);
  auto it = sv->live.find(ticket);
  if (it == sv->live.end()) return set_error("unknown or already reported ticket %lld", (long long)ticket), FPP_EINVAL;
  return report(sv, it, status, t_submit_ns, t_done_ns);
}

int fpp_server_wait(fpp_server* sv, int64_t ticket, int64_t timeout_ms, int32_t* status,
                    int64_t* t_submit_ns, int64_t* t_done_ns) {
  if (!sv) return set_error("NULL argument"), FPP_EINVAL;
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->live.find(ticket);
  if (it == sv->live.end()) return set_error("unknown or already reported ticket %lld", (long long)ticket), FPP_EINVAL;
  std::shared_ptr<Request> r = it->second;
  auto pred = [&] { return r->status != 1; };
  if (timeout_ms < 0) sv->done_cv.wait(lk, pred);
  else sv->done_cv.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred);
  it = sv->live.find(ticket);
  if (it != sv->live.end()) return report(sv, it, status, t_submit_ns, t_done_ns);
  if (status) *status = r->status;   // reported meanwhile by another caller
  if (t_submit_ns) *t_submit_ns = r->t_submit;
  if (t_done_ns) *t_done_ns = r->t_done;
  return FPP_OK;
}

int fpp_server_replay(fpp_server* sv, const float* Q, int64_t n_req, int64_t t0_ns,
                      const int64_t* arrive_ns, const int64_t* q_row, const int32_t* m,
                      const int32_t* k, const int32_t* qProbes, int32_t* ids_out,
                      float* scores_out, const int64_t* out_off, int64_t* tickets) {
  if (!sv || n_req < 0) return set_error("NULL server or n_req < 0"), FPP_EINVAL;
  if (n_req == 0) return FPP_OK;
  if (!Q || !arrive_ns || !q_row || !m || !k || !qProbes || !ids_out || !scores_out || !out_off ||
      !tickets)
    return set_error("NULL argument"), FPP_EINVAL;
  for (int64_t i = 0; i < n_req; ++i) tickets[i] = 0;
  const int64_t d = sv->ix->d;
  for (int64_t i = 0; i < n_req; ++i) {
    const int64_t t = t0_ns + arrive_ns[i];
    while (now_ns() < t) {
    }
    const int rc = fpp_server_submit(sv, Q + q_row[i] * d, m[i], k[i], qProbes[i], ids_out + out_off[i],
                                     scores_out + out_off[i], &tickets[i]);
    if (rc != FPP_OK) return rc;
  }
  return FPP_OK;
}

int fpp_server_debug_fail_batches(fpp_server* sv, int32_t n) {
  if (!sv || n < 0) return set_error("NULL server or n < 0"), FPP_EINVAL;
  sv->fail_batches.store(n);
  return FPP_OK;
}

int fpp_server_get_stats(fpp_server* sv, fpp_server_stats* out) {
  if (!sv || !out) return set_error("NULL argument"), FPP_EINVAL;
  std::lock_guard<std::mutex> g(sv->mu);
  *out = sv->stats;
  return FPP_OK;
}

void fpp_server_destroy(fpp_server* sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> g(sv->mu);
    sv->stopping = true;
  }
  sv->cv.notify_all();
  if (sv->loop.joinable()) sv->loop.join();
  for (auto& s : sv->slots) {
    if (s.stream) (void)hipStreamSynchronize(s.stream);
    release_slot_buffers(s);
  }
  if (sv->pool_mem) (void)hipFree(sv->pool_mem);
  delete sv;
}

}  // extern "C"
