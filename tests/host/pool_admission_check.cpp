// Randomised check of the serving loop's scratch pool and FIFO admission (host code only), built
// with AddressSanitizer and UndefinedBehaviorSanitizer by the test suite. It drives
// fpp::Pool / fpp::admit_fifo the way the loop does: a FIFO of requests, a few stream slots,
// batches admitted while a slot and scratch are free, completions in random order.
// Checked after every step: allocated blocks lie inside the pool and never overlap, the pool's
// bookkeeping adds up, requests leave the queue in submission order, a batch holds at most
// max_batch queries unless it is a single request, and a drained pool is one free block again.
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <random>
#include <vector>

#include "../../paper_2206_01382_amd/csrc/server_pool.hpp"

namespace {

struct Req {
  long id;
  int64_t m;
  int32_t k, qp;
};

struct Batch {
  bool busy = false;
  size_t off = 0, bytes = 0;
  std::vector<Req> reqs;
};

int failures = 0;
#define CHECK(c, ...)                              \
  do {                                             \
    if (!(c)) {                                    \
      std::fprintf(stderr, "FAILED %s: ", #c);     \
      std::fprintf(stderr, __VA_ARGS__);           \
      std::fprintf(stderr, "\n");                  \
      if (++failures > 20) std::exit(1);           \
    }                                              \
  } while (0)

// scratch of a batch: per query a few hundred bytes plus terms in k and qProbes (the shape of
// the real layout: linear in m with per-query costs growing with k and qProbes)
size_t bytes_of(int64_t m, int32_t k, int32_t qp) {
  return (size_t)m * (64 + 8 * (size_t)k + 4 * (size_t)qp) + 300;
}

void run(unsigned seed, size_t capacity, int n_slots, int64_t max_batch, int steps) {
  std::mt19937_64 rng(seed);
  fpp::Pool pool;
  pool.init(capacity);
  std::deque<Req> queue;
  std::vector<Batch> slots(n_slots);
  long next_id = 0, next_out = 0;
  for (int step = 0; step < steps; ++step) {
    // arrivals (requests that could never fit are rejected at submission, as the server does)
    const int arrivals = (int)(rng() % 4);
    for (int a = 0; a < arrivals; ++a) {
      Req r{next_id, 1 + (int64_t)(rng() % (uint64_t)std::max<int64_t>(1, max_batch)),
            (int32_t)(1 + rng() % 512), (int32_t)(1 + rng() % 20000)};
      if (fpp::pool_round(bytes_of(r.m, r.k, r.qp)) > pool.capacity()) continue;
      ++next_id;
      queue.push_back(r);
    }
    // completions in random order
    for (auto& s : slots) {
      if (!s.busy || rng() % 3) continue;
      pool.release(s.off, s.bytes);
      s.busy = false;
      s.reqs.clear();
    }
    // admission, as the loop does it
    for (auto& s : slots) {
      if (s.busy || queue.empty()) continue;
      const fpp::Admitted a = fpp::admit_fifo(
          queue.begin(), queue.end(), max_batch, pool,
          [](const Req& r) { return fpp::AdmitShape{r.m, r.k, r.qp}; }, bytes_of);
      if (a.taken == 0) break;
      CHECK(a.taken <= queue.size(), "taken %zu of %zu", a.taken, queue.size());
      int64_t m = 0;
      int32_t kmax = 0, qpmax = 0;
      for (size_t i = 0; i < a.taken; ++i) {
        const Req& r = queue[i];
        CHECK(r.id == next_out, "request %ld left the queue before %ld", r.id, next_out);
        ++next_out;
        m += r.m;
        kmax = std::max(kmax, r.k);
        qpmax = std::max(qpmax, r.qp);
      }
      CHECK(m == a.m && kmax == a.kmax && qpmax == a.qpmax, "batch shape");
      CHECK(a.taken == 1 || m <= max_batch, "batch of %lld queries", (long long)m);
      CHECK(a.bytes == bytes_of(m, kmax, qpmax), "batch bytes");
      CHECK(a.offset + fpp::pool_round(a.bytes) <= capacity, "block past the pool end");
      s.busy = true;
      s.off = a.offset;
      s.bytes = a.bytes;
      s.reqs.assign(queue.begin(), queue.begin() + (std::ptrdiff_t)a.taken);
      queue.erase(queue.begin(), queue.begin() + (std::ptrdiff_t)a.taken);
    }
    // allocated blocks are disjoint and the bookkeeping adds up
    size_t used = 0;
    for (size_t i = 0; i < slots.size(); ++i) {
      if (!slots[i].busy) continue;
      used += fpp::pool_round(slots[i].bytes);
      for (size_t j = i + 1; j < slots.size(); ++j) {
        if (!slots[j].busy) continue;
        const size_t a0 = slots[i].off, a1 = a0 + fpp::pool_round(slots[i].bytes);
        const size_t b0 = slots[j].off, b1 = b0 + fpp::pool_round(slots[j].bytes);
        CHECK(a1 <= b0 || b1 <= a0, "blocks [%zu,%zu) and [%zu,%zu) overlap", a0, a1, b0, b1);
      }
    }
    CHECK(used == pool.used(), "used %zu, pool says %zu", used, pool.used());
    CHECK(pool.high_water() <= capacity, "high water");
    CHECK(pool.largest_free() <= capacity - used, "largest free block");
  }
  // drain
  for (auto& s : slots)
    if (s.busy) pool.release(s.off, s.bytes);
  CHECK(pool.used() == 0 && pool.free_blocks() == 1 && pool.largest_free() == capacity,
        "drained pool: used %zu, %zu free blocks", pool.used(), pool.free_blocks());
}

}  // namespace

int main() {
  const size_t caps[] = {4096, 100000, 1u << 20, 12345679, 64u << 20};
  unsigned seed = 1;
  for (size_t cap : caps)
    for (int slots : {1, 2, 4, 8})
      for (int64_t mb : {1, 16, 1024}) run(seed++, cap, slots, mb, 3000);
  if (failures) {
    std::fprintf(stderr, "%d failures\n", failures);
    return 1;
  }
  std::printf("pool/admission check passed\n");
  return 0;
}
