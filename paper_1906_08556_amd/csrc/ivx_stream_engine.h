// Ordered producer/consumer ring of the streaming host pipeline (the data
// loaders of Sec. 4.2, Fig. 1): loader threads fill batches into a ring of
// host slots in any order, the consumer takes them strictly in batch order.
//
// Batch b always goes to slot b % nslots.  A loader that takes batch b waits
// until the slot has been released by batch b - nslots; the consumer releases
// a batch's slot once its upload has finished.  With nslots >= 2 and the
// consumer releasing batch b - 1 after it has issued batch b, no wait depends
// on a later action of the thread that waits, so the ring cannot deadlock.
// Plain C++ (no HIP): the loaders only touch host memory.
#pragma once

#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <mutex>
#include <thread>
#include <vector>

namespace ivx {

class BatchRing {
 public:
  BatchRing(int nslots, int64_t nbatches)
      : nslots_(nslots), nb_(nbatches), owner_(nslots), ready_(nslots, 0) {
    for (int s = 0; s < nslots; ++s) owner_[s] = s;
  }

  int slot_of(int64_t b) const { return (int)(b % nslots_); }

  // Loader side: fill(b, slot) -> bool writes batch b into the slot.
  template <class Fill>
  void loader_loop(Fill fill) {
    for (;;) {
      const int64_t b = next_.fetch_add(1);
      if (b >= nb_) return;
      const int s = slot_of(b);
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return abort_ || (owner_[s] == b && !ready_[s]); });
        if (abort_) return;
      }
      const bool ok = fill(b, s);
      {
        std::lock_guard<std::mutex> lk(mu_);
        if (ok)
          ready_[s] = 1;
        else
          abort_ = failed_ = true;
      }
      cv_.notify_all();
    }
  }

  // Consumer side: blocks until batch b is in its slot; false once aborted.
  bool wait_ready(int64_t b) {
    const int s = slot_of(b);
    std::unique_lock<std::mutex> lk(mu_);
    cv_.wait(lk, [&] { return abort_ || (owner_[s] == b && ready_[s]); });
    return !abort_;
  }

  // Consumer side: batch b no longer needs its slot.
  void release(int64_t b) {
    const int s = slot_of(b);
    {
      std::lock_guard<std::mutex> lk(mu_);
      ready_[s] = 0;
      owner_[s] = b + nslots_;
    }
    cv_.notify_all();
  }

  // Stops every loader (they return at their next wait).
  void stop() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      abort_ = true;
    }
    cv_.notify_all();
  }

  // True if a fill reported failure.
  bool failed() {
    std::lock_guard<std::mutex> lk(mu_);
    return failed_;
  }

 private:
  const int nslots_;
  const int64_t nb_;
  std::mutex mu_;
  std::condition_variable cv_;
  std::vector<int64_t> owner_;  // the batch allowed into each slot next
  std::vector<int> ready_;      // slot holds owner_'s batch, filled
  bool abort_ = false;
  bool failed_ = false;
  std::atomic<int64_t> next_{0};
};

// Greedy split of utterances [0, U) into runs of consecutive utterances with
// at most max_utts utterances and max_frames frames each.  starts receives the
// first utterance of every batch followed by U.  Returns the number of
// batches, or -1 - u if utterance u alone exceeds max_frames (or offsets
// decrease there).
inline int64_t plan_batches(const int64_t* off, int64_t U, int64_t max_utts, int64_t max_frames,
                            std::vector<int64_t>& starts) {
  starts.clear();
  int64_t u = 0;
  while (u < U) {
    starts.push_back(u);
    const int64_t u0 = u;
    while (u < U && u - u0 < max_utts) {
      const int64_t len = off[u + 1] - off[u];
      if (len < 0 || len > max_frames) return -1 - u;
      if (off[u + 1] - off[u0] > max_frames) break;
      ++u;
    }
  }
  starts.push_back(U);
  return (int64_t)starts.size() - 1;
}

}  // namespace ivx
