// Scheduling core of the query server: device-memory pool, request queue,
// continuous batching and slot management.  Plain C++17 with no HIP: the
// server drives it with a HIP executor, the tests with a fake one.
//
// Policy:
//   * requests wait in arrival order;
//   * when a slot is free, a launch is formed from the head of the queue: the
//     head plus the requests right behind it, up to max_batch_queries query
//     rows in all; it computes the top-k for the largest k among them, and
//     each request keeps the first k of its rows' lists (the order -- |tau|
//     descending, then row -- makes a shorter list a prefix of a longer one);
//   * the launch is admitted only if its device bytes can be carved from the
//     pool (first fit); otherwise it waits until running launches free
//     memory -- so requests that arrive while others run are admitted as
//     slots and memory free up, and their work overlaps on the device;
//   * a request flagged for a forced failure always runs alone;
//   * a launch whose start fails part-way is drained (the executor waits for
//     what it already enqueued) before its memory returns to the pool;
//   * while paused, nothing new is admitted (running launches still finish and
//     requests still queue).
#pragma once

#include <stdint.h>

#include <chrono>
#include <deque>
#include <map>
#include <memory>
#include <vector>

namespace ktau {
namespace sched {

using Clock = std::chrono::steady_clock;

// First-fit allocator over [0, capacity) in 256-byte units.
class Pool {
 public:
  explicit Pool(size_t capacity) : cap_(capacity & ~(size_t)255) {
    if (cap_) free_[0] = cap_;
  }
  static size_t round(size_t b) { return (b + 255) & ~(size_t)255; }
  bool alloc(size_t bytes, size_t* off) {
    bytes = round(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes, at = it->first + bytes;
        free_.erase(it);
        if (rest) free_[at] = rest;
        used_ += bytes;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = round(bytes);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }
  size_t capacity() const { return cap_; }

 private:
  size_t cap_;
  size_t used_ = 0;
  std::map<size_t, size_t> free_;
};

enum State : int { kQueued = 1, kRunning = 2, kDone = 0 };

struct Request {
  int64_t ticket = 0;
  int64_t nq = 0, k = 0;
  std::vector<float> q;            // host copy of the query rows
  Clock::time_point t_submit, t_start, t_done;
  int state = kQueued;
  int status = 0;                  // result status once done
  bool force_fail = false;
  int64_t batch_queries = 0, batch_requests = 0;
  std::vector<int64_t> idx;
  std::vector<double> tau;
  std::vector<int64_t> nd;
};

struct Launch {
  std::vector<Request*> reqs;
  int64_t nq = 0, k = 0;
  size_t bytes = 0, off = 0;
  int slot = -1;
  bool fail = false;
};

// What runs a launch.  All calls come from the scheduler's thread.
class Executor {
 public:
  virtual ~Executor() = default;
  virtual size_t bytes_for(int64_t nq, int64_t k) const = 0;
  // enqueue the launch's work; non-zero = it could not be started
  virtual int start(Launch& l) = 0;
  // after start() failed: returns only once nothing that start() may already
  // have enqueued can still touch the launch's pool region or staging
  virtual void abandon(Launch& l) = 0;
  // has the launch finished (results ready to collect)?
  virtual bool finished(const Launch& l) = 0;
  // copy results into the requests; returns the launch status
  virtual int collect(Launch& l) = 0;
};

struct Config {
  int slots = 4;
  int64_t max_batch_queries = 64;
  size_t budget = (size_t)1 << 30;
};

struct Stats {
  int64_t launches = 0, merged = 0, completed = 0, failed = 0;
  size_t peak_bytes = 0;
  int64_t peak_running = 0;
};

class Scheduler {
 public:
  Scheduler(const Config& c, Executor* ex) : cfg_(c), ex_(ex), pool_(c.budget), slots_(c.slots) {}

  // Largest launch that can ever be admitted.
  bool fits_ever(int64_t nq, int64_t k) const { return ex_->bytes_for(nq, k) <= pool_.capacity(); }

  void enqueue(Request* r) { queue_.push_back(r); }

  void set_paused(bool p) { paused_ = p; }
  bool paused() const { return paused_; }

  // Removes a queued request; false if it is not waiting.
  bool cancel(Request* r) {
    for (auto it = queue_.begin(); it != queue_.end(); ++it)
      if (*it == r) {
        queue_.erase(it);
        return true;
      }
    return false;
  }

  // One pass: collect finished launches, then admit what fits.  Returns the
  // requests completed in this pass.
  std::vector<Request*> step() {
    std::vector<Request*> done;
    for (int s = 0; s < (int)slots_.size(); ++s) {
      auto& l = slots_[s];
      if (!l || !(l->fail || ex_->finished(*l))) continue;
      const int st = l->fail ? -7 : ex_->collect(*l);
      const auto now = Clock::now();
      for (Request* r : l->reqs) {
        r->state = kDone;
        r->status = st;
        r->t_done = now;
        done.push_back(r);
        if (st == 0) stats_.completed++;
        else stats_.failed++;
      }
      pool_.release(l->off, l->bytes);
      l.reset();
      --running_;
    }
    for (;;) {
      if (queue_.empty() || paused_) break;
      int free_slot = -1;
      for (int s = 0; s < (int)slots_.size(); ++s)
        if (!slots_[s]) {
          free_slot = s;
          break;
        }
      if (free_slot < 0) break;
      auto l = std::make_unique<Launch>();
      Request* head = queue_.front();
      l->fail = head->force_fail;
      size_t take = 0;
      int64_t nq = 0;
      for (size_t i = 0; i < queue_.size(); ++i) {
        Request* r = queue_[i];
        if (i > 0 && (r->force_fail || l->fail)) break;
        if (i > 0 && nq + r->nq > cfg_.max_batch_queries) break;
        nq += r->nq;
        take = i + 1;
      }
      // shrink the launch until it fits the free pool (the head alone at least)
      while (take > 0) {
        int64_t q = 0, k = 0;
        for (size_t i = 0; i < take; ++i) {
          q += queue_[i]->nq;
          k = queue_[i]->k > k ? queue_[i]->k : k;
        }
        size_t off = 0;
        const size_t bytes = ex_->bytes_for(q, k);
        if (pool_.alloc(bytes, &off)) {
          l->nq = q;
          l->k = k;
          l->bytes = bytes;
          l->off = off;
          break;
        }
        --take;
      }
      if (take == 0) break;   // the head waits for memory
      const auto now = Clock::now();
      for (size_t i = 0; i < take; ++i) {
        Request* r = queue_.front();
        queue_.pop_front();
        r->state = kRunning;
        r->t_start = now;
        r->batch_queries = l->nq;
        r->batch_requests = (int64_t)take;
        l->reqs.push_back(r);
      }
      l->slot = free_slot;
      stats_.launches++;
      stats_.merged += (int64_t)take - 1;
      const int st = l->fail ? 0 : ex_->start(*l);
      if (st != 0) {
        // work already enqueued may still write the region: drain it before
        // the failure is collected and the region goes back to the pool
        ex_->abandon(*l);
        l->fail = true;   // collected as a failure on the next pass
      }
      ++running_;
      if (running_ > stats_.peak_running) stats_.peak_running = running_;
      if (pool_.used() > stats_.peak_bytes) stats_.peak_bytes = pool_.used();
      slots_[free_slot] = std::move(l);
    }
    return done;
  }

  bool idle() const { return queue_.empty() && running_ == 0; }
  int64_t running() const { return running_; }
  size_t queued() const { return queue_.size(); }
  size_t pool_used() const { return pool_.used(); }
  const Stats& stats() const { return stats_; }
  const Config& config() const { return cfg_; }

 private:
  Config cfg_;
  Executor* ex_;
  Pool pool_;
  std::deque<Request*> queue_;
  std::vector<std::unique_ptr<Launch>> slots_;
  int64_t running_ = 0;
  bool paused_ = false;
  Stats stats_;
};

}  // namespace sched
}  // namespace ktau
