// Host-side scratch pool and first-in first-out admission of the serving loop. Plain C++ with no
// HIP dependency, so the same code also builds for the CPU alone (the sanitizer check of the
// tests compiles it with AddressSanitizer and UndefinedBehaviorSanitizer).
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <map>

namespace fpp {

inline size_t pool_round(size_t v) { return (v + 255) / 256 * 256; }

// First-fit allocator over one buffer of `capacity` bytes; blocks are multiples of 256 bytes,
// and adjacent free blocks are merged on release.
class Pool {
 public:
  void init(size_t bytes) {
    cap_ = bytes;
    used_ = high_ = 0;
    free_.clear();
    if (bytes) free_[0] = bytes;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = pool_round(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rem = it->second - bytes, start = it->first + bytes;
        free_.erase(it);
        if (rem) free_[start] = rem;
        used_ += bytes;
        high_ = std::max(high_, used_);
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = pool_round(bytes);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t largest_free() const {
    size_t b = 0;
    for (auto& kv : free_) b = std::max(b, kv.second);
    return b;
  }
  size_t capacity() const { return cap_; }
  size_t used() const { return used_; }
  size_t high_water() const { return high_; }
  size_t free_blocks() const { return free_.size(); }

 private:
  std::map<size_t, size_t> free_;   // offset -> bytes
  size_t cap_ = 0, used_ = 0, high_ = 0;
};

// What admission needs to know of a request.
struct AdmitShape {
  int64_t m;
  int32_t k, qp;
};

// One admitted batch: the first `taken` requests of the queue, `m` queries with the largest k
// and qProbes of its requests, and `bytes` of scratch at `offset` in the pool.
struct Admitted {
  size_t taken = 0;
  int64_t m = 0;
  int32_t kmax = 0, qpmax = 0;
  size_t bytes = 0, offset = 0;
};

// Takes requests from the head of [first, last) in order while the batch stays within max_batch
// queries (a single request may fill a batch alone) and its scratch, bytes_of(m, kmax, qpmax)
// rounded up to the pool's 256-byte blocks, fits in the pool's largest free block, then
// allocates that scratch. `shape` maps a queue element to its AdmitShape. Returns taken = 0
// when the head request has to wait for scratch.
template <class It, class Shape, class BytesOf>
Admitted admit_fifo(It first, It last, int64_t max_batch, Pool& pool, Shape shape, BytesOf bytes_of) {
  Admitted a;
  const size_t avail = pool.largest_free();
  for (It it = first; it != last; ++it) {
    const AdmitShape r = shape(*it);
    const int64_t m2 = a.m + r.m;
    if (m2 > max_batch && a.m > 0) break;
    const int32_t k2 = std::max(a.kmax, r.k), q2 = std::max(a.qpmax, r.qp);
    const size_t need2 = bytes_of(m2, k2, q2);
    if (pool_round(need2) > avail) break;
    a.m = m2;
    a.kmax = k2;
    a.qpmax = q2;
    a.bytes = need2;
    ++a.taken;
  }
  if (a.taken && !pool.alloc(a.bytes, &a.offset)) a = Admitted{};
  return a;
}

}  // namespace fpp
