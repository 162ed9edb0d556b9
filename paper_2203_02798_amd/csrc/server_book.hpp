// Host-side bookkeeping of the request server: the first-fit pool
// allocator that admits requests by workspace footprint, and the ticket
// board that hands each finished request back exactly once.  Plain C++ (no
// HIP), so that it can be built and tested on a host alone.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <condition_variable>
#include <iterator>
#include <map>
#include <mutex>

namespace psk {

constexpr size_t kAlign = 256;

// First-fit allocator over [0, cap) with coalescing of free ranges.
class PoolAlloc {
 public:
  explicit PoolAlloc(size_t cap) : cap_(cap) {
    if (cap_ > 0) free_[0] = cap_;
  }
  // offset of a block of `bytes`, or SIZE_MAX if none fits
  size_t alloc(size_t bytes) {
    bytes = (bytes + kAlign - 1) / kAlign * kAlign;
    if (bytes == 0) bytes = kAlign;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const size_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > bytes) free_[off + bytes] = len - bytes;
        used_ += bytes;
        if (used_ > peak_) peak_ = used_;
        sizes_[off] = bytes;
        return off;
      }
    }
    return SIZE_MAX;
  }
  void release(size_t off) {
    auto s = sizes_.find(off);
    if (s == sizes_.end()) return;
    size_t start = off, len = s->second;
    sizes_.erase(s);
    used_ -= len;
    auto next = free_.find(start + len);  // merge with the following free range
    if (next != free_.end()) {
      len += next->second;
      free_.erase(next);
    }
    auto it = free_.lower_bound(start);  // and with the preceding one
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == start) {
        start = prev->first;
        len += prev->second;
        free_.erase(prev);
      }
    }
    free_[start] = len;
  }
  size_t peak() const { return peak_; }
  size_t used() const { return used_; }

 private:
  size_t cap_, used_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_;   // offset -> length
  std::map<size_t, size_t> sizes_;  // allocated offset -> length
};

// Tickets of submitted jobs (Job needs a `bool done`).  Every member is
// called with the server's mutex held (wait releases it while it blocks).
// A ticket is claimed by the first wait on it; a second wait or a poll on a
// claimed ticket is refused (kClaimed) instead of sharing the job, which
// the claiming waiter deletes when it returns.
template <typename Job>
class TicketBoard {
 public:
  enum { kOk = 0, kPending = 1, kUnknown = -1, kClaimed = -2 };

  int64_t add(Job *j) {
    const int64_t t = next_++;
    slots_[t] = Slot{j, false};
    return t;
  }
  // after a job's `done` was set: wake its waiter
  void completed() { cv_.notify_all(); }
  // block until ticket t is done, fill(job), forget it
  template <typename F>
  int wait(std::unique_lock<std::mutex> &lk, int64_t t, F &&fill) {
    auto it = slots_.find(t);
    if (it == slots_.end()) return kUnknown;
    if (it->second.claimed) return kClaimed;
    it->second.claimed = true;
    Job *j = it->second.job;
    cv_.wait(lk, [&] { return j->done; });
    fill(*j);
    slots_.erase(t);
    delete j;
    return kOk;
  }
  // fill(job) and forget it if done; kPending if not
  template <typename F>
  int poll(int64_t t, F &&fill) {
    auto it = slots_.find(t);
    if (it == slots_.end()) return kUnknown;
    if (it->second.claimed) return kClaimed;
    Job *j = it->second.job;
    if (!j->done) return kPending;
    fill(*j);
    slots_.erase(it);
    delete j;
    return kOk;
  }
  // delete every job still held (the server is being destroyed)
  void clear() {
    for (auto &kv : slots_) delete kv.second.job;
    slots_.clear();
  }
  size_t size() const { return slots_.size(); }

 private:
  struct Slot {
    Job *job;
    bool claimed;
  };
  std::map<int64_t, Slot> slots_;
  int64_t next_ = 1;
  std::condition_variable cv_;
};

}  // namespace psk
