// Query server: continuous batching of query-vs-database requests over a
// resident database.  A worker thread runs the scheduling core
// (ktau_sched.h) with a HIP executor: every launch gets a region of one
// device pool (its admission), a slot stream, pinned staging for its query
// rows and its results, and an event that signals completion.  Launches on
// different slots overlap on the device.  Latency of a request is completion
// time minus submission time, so it includes queueing.
#include <string.h>

#include <atomic>
#include <condition_variable>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "ktau_query.h"
#include "ktau_sched.h"

namespace ktau {
namespace {

using sched::Launch;
using sched::Request;

size_t al(size_t b) { return (b + 255) & ~(size_t)255; }

// How a finished launch wakes the worker: a host function enqueued on the
// slot's stream after the result copy sets the flag and notifies the
// worker's condition variable.  It takes no lock: a callback waiting for the
// server's mutex could deadlock a stream synchronisation the worker makes
// while holding it; the worker's wait has a short timeout for the rare
// notification that arrives just before it blocks.
struct Wake {
  std::atomic<bool> pending{false};
  std::condition_variable* cv = nullptr;
};

void wake_worker(void* p) {
  Wake* w = (Wake*)p;
  w->pending.store(true, std::memory_order_release);
  w->cv->notify_one();
}

class GpuExecutor : public sched::Executor {
 public:
  GpuExecutor(const DbView& db, int slots, int64_t max_q, int64_t k_max, char* pool, Wake* wake)
      : db_(db), max_q_(max_q), k_max_(k_max), pool_(pool), wake_(wake), slots_(slots) {}

  // HIP objects; false if any could not be made.
  bool init() {
    for (Slot& s : slots_) {
      if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess) return false;
      if (hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess) return false;
      if (hipHostMalloc((void**)&s.in, (size_t)max_q_ * db_.n * sizeof(float),
                        hipHostMallocDefault) != hipSuccess)
        return false;
      if (hipHostMalloc((void**)&s.out, out_bytes(max_q_, k_max_), hipHostMallocDefault) !=
          hipSuccess)
        return false;
      s.in_cap = max_q_;
    }
    return true;
  }

  ~GpuExecutor() override {
    for (Slot& s : slots_) {
      if (s.stream) {
        (void)hipStreamSynchronize(s.stream);
        (void)hipStreamDestroy(s.stream);
      }
      if (s.done) (void)hipEventDestroy(s.done);
      if (s.in) (void)hipHostFree(s.in);
      if (s.out) (void)hipHostFree(s.out);
    }
  }

  // status header | idx | tau | nd   (one contiguous block copied back)
  static size_t out_bytes(int64_t nq, int64_t k) { return 256 + 3 * al((size_t)(nq * k) * 8); }

  size_t bytes_for(int64_t nq, int64_t k) const override {
    return out_bytes(nq, k) + al((size_t)(nq * db_.n) * sizeof(float)) +
           query_scratch_bytes(nq, db_.m, db_.n, (int)k, db_.scheme == KTAU_SCHEME_NAIVE);
  }

  int start(Launch& l) override {
    Slot& s = slots_[l.slot];
    const int64_t n = db_.n, nq = l.nq, k = l.k;
    if (nq > s.in_cap || k > k_max_) {
      // a request larger than the staging buffers: grow them for this slot
      (void)hipHostFree(s.in);
      (void)hipHostFree(s.out);
      s.in = nullptr;
      s.out = nullptr;
      const int64_t cap = nq > s.in_cap ? nq : s.in_cap;
      if (hipHostMalloc((void**)&s.in, (size_t)cap * n * sizeof(float), hipHostMallocDefault) !=
              hipSuccess ||
          hipHostMalloc((void**)&s.out, out_bytes(cap, k > k_max_ ? k : k_max_),
                        hipHostMallocDefault) != hipSuccess)
        return KTAU_ENOMEM;
      s.in_cap = cap;
      if (k > k_max_) k_max_ = k;
    }
    int64_t o = 0;
    for (Request* r : l.reqs) {
      memcpy(s.in + o * n, r->q.data(), (size_t)(r->nq * n) * sizeof(float));
      o += r->nq;
    }
    char* base = pool_ + l.off;
    const size_t ob = out_bytes(nq, k);
    int32_t* status = (int32_t*)base;
    int64_t* idx = (int64_t*)(base + 256);
    double* tau = (double*)(base + 256 + al((size_t)(nq * k) * 8));
    int64_t* nd = (int64_t*)(base + 256 + 2 * al((size_t)(nq * k) * 8));
    float* q = (float*)(base + ob);
    char* scratch = base + ob + al((size_t)(nq * n) * sizeof(float));
    if (hipMemcpyAsync(q, s.in, (size_t)(nq * n) * sizeof(float), hipMemcpyHostToDevice,
                       s.stream) != hipSuccess)
      return KTAU_EDEVICE;
    if (clear_words(status, 2, s.stream) != KTAU_OK) return KTAU_EDEVICE;
    int rc = launch_query(db_, q, nq, (int)k, scratch, idx, tau, nd, status, s.stream);
    if (rc != KTAU_OK) return rc;
    if (hipMemcpyAsync(s.out, base, ob, hipMemcpyDeviceToHost, s.stream) != hipSuccess)
      return KTAU_EDEVICE;
    if (hipEventRecord(s.done, s.stream) != hipSuccess) return KTAU_EDEVICE;
    if (hipLaunchHostFunc(s.stream, wake_worker, wake_) != hipSuccess) return KTAU_EDEVICE;
    return KTAU_OK;
  }

  void abandon(Launch& l) override { (void)hipStreamSynchronize(slots_[l.slot].stream); }

  bool finished(const Launch& l) override {
    return hipEventQuery(slots_[l.slot].done) != hipErrorNotReady;
  }

  int collect(Launch& l) override {
    Slot& s = slots_[l.slot];
    if (hipEventSynchronize(s.done) != hipSuccess) return KTAU_EDEVICE;
    const int64_t k = l.k, nq = l.nq;
    const int32_t status = *(const int32_t*)s.out;
    const int64_t* idx = (const int64_t*)(s.out + 256);
    const double* tau = (const double*)(s.out + 256 + al((size_t)(nq * k) * 8));
    const int64_t* nd = (const int64_t*)(s.out + 256 + 2 * al((size_t)(nq * k) * 8));
    // each request's rows, each cut to the request's own k (the launch ran
    // the largest k of the requests it merged)
    int64_t o = 0;
    for (Request* r : l.reqs) {
      const int64_t kr = r->k;
      r->idx.resize((size_t)(r->nq * kr));
      r->tau.resize((size_t)(r->nq * kr));
      r->nd.resize((size_t)(r->nq * kr));
      for (int64_t qi = 0; qi < r->nq; ++qi) {
        const int64_t src = (o + qi) * k, dst = qi * kr;
        memcpy(r->idx.data() + dst, idx + src, (size_t)kr * sizeof(int64_t));
        memcpy(r->tau.data() + dst, tau + src, (size_t)kr * sizeof(double));
        memcpy(r->nd.data() + dst, nd + src, (size_t)kr * sizeof(int64_t));
      }
      o += r->nq;
    }
    return status;
  }

 private:
  struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    float* in = nullptr;
    char* out = nullptr;
    int64_t in_cap = 0;
  };
  DbView db_;
  int64_t max_q_, k_max_;
  char* pool_;
  Wake* wake_;
  std::vector<Slot> slots_;
};

bool has_nan(const float* p, size_t count) {
  for (size_t i = 0; i < count; ++i)
    if (p[i] != p[i]) return true;
  return false;
}

}  // namespace
}  // namespace ktau

using namespace ktau;

struct ktau_server {
  ktau_server_cfg cfg;
  const ktau_db* db = nullptr;
  int device = 0;
  char* pool = nullptr;
  std::unique_ptr<GpuExecutor> ex;
  std::unique_ptr<sched::Scheduler> sched;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  Wake wake;
  std::thread worker;
  bool stop = false;
  int64_t epoch = 0;   // counts submissions and admission changes (under mu)
  int64_t next_ticket = 1;
  std::unordered_map<int64_t, std::unique_ptr<Request>> reqs;
};

namespace {

void worker_loop(ktau_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    s->wake.pending.store(false, std::memory_order_relaxed);
    const auto done = s->sched->step();
    if (!done.empty()) s->cv_done.notify_all();
    if (s->stop && s->sched->idle()) break;
    const int64_t seen = s->epoch;
    if (s->sched->running() > 0) {
      // until a launch finishes (its host function) or new work arrives
      s->cv_work.wait_for(lk, std::chrono::microseconds(250), [&] {
        return s->stop || s->epoch != seen || s->wake.pending.load(std::memory_order_acquire);
      });
    } else {
      s->cv_work.wait(lk, [&] {
        return s->stop || (s->sched->queued() > 0 && !s->sched->paused());
      });
    }
  }
}

}  // namespace

extern "C" {

void ktau_server_default_cfg(ktau_server_cfg* c) {
  if (!c) return;
  // measured on a 20000 x 800 database with requests of 1-64 rows at 0.8 of
  // saturation: two launches in flight of up to 256 rows gave the highest
  // saturation and the most requests per launch at a p50 within 10% of the
  // best
  c->slots = 2;
  c->max_batch_queries = 256;
  c->mem_budget_bytes = (int64_t)1 << 30;
  c->max_queue = 4096;
  c->k_max = 128;
}

int ktau_server_create(const ktau_db* db, const ktau_server_cfg* cfg, ktau_server** out) {
  if (!db || !out) return KTAU_EINVAL;
  *out = nullptr;
  ktau_server_cfg c;
  ktau_server_default_cfg(&c);
  if (cfg) c = *cfg;
  if (c.slots < 1 || c.slots > 64 || c.max_batch_queries < 1 || c.mem_budget_bytes < 4096 ||
      c.max_queue < 1 || c.k_max < 1 || c.k_max > KTAU_MAX_K)
    return KTAU_EINVAL;
  ktau_server* s = new ktau_server();
  s->cfg = c;
  s->db = db;
  if (hipGetDevice(&s->device) != hipSuccess ||
      hipMalloc((void**)&s->pool, (size_t)c.mem_budget_bytes) != hipSuccess) {
    delete s;
    return KTAU_ENOMEM;
  }
  s->wake.cv = &s->cv_work;
  s->ex = std::make_unique<GpuExecutor>(db->v, c.slots, c.max_batch_queries, c.k_max, s->pool,
                                        &s->wake);
  if (!s->ex->init()) {
    s->ex.reset();
    (void)hipFree(s->pool);
    delete s;
    return KTAU_EDEVICE;
  }
  sched::Config sc;
  sc.slots = c.slots;
  sc.max_batch_queries = c.max_batch_queries;
  sc.budget = (size_t)c.mem_budget_bytes;
  s->sched = std::make_unique<sched::Scheduler>(sc, s->ex.get());
  s->worker = std::thread(worker_loop, s);
  *out = s;
  return KTAU_OK;
}

int ktau_server_submit(ktau_server* s, const float* q, int64_t nq, int64_t k, int blocking,
                       int64_t* ticket) {
  if (!s || !q || nq < 1 || !ticket) return KTAU_EINVAL;
  if (k < 1 || k > s->cfg.k_max) return KTAU_ERANGE;
  const int64_t n = s->db->v.n;
  if (has_nan(q, (size_t)(nq * n))) return KTAU_ENAN;
  auto r = std::make_unique<Request>();
  r->nq = nq;
  r->k = k;
  r->q.assign(q, q + nq * n);
  std::unique_lock<std::mutex> lk(s->mu);
  if (!s->sched->fits_ever(nq, k)) return KTAU_ENOMEM;
  if ((int64_t)s->sched->queued() >= s->cfg.max_queue) {
    if (!blocking) return KTAU_EBUSY;
    s->cv_done.wait(lk, [&] { return (int64_t)s->sched->queued() < s->cfg.max_queue; });
  }
  r->ticket = s->next_ticket++;
  r->t_submit = sched::Clock::now();
  *ticket = r->ticket;
  s->sched->enqueue(r.get());
  s->reqs[r->ticket] = std::move(r);
  ++s->epoch;
  s->cv_work.notify_one();
  return KTAU_OK;
}

int ktau_server_wait(ktau_server* s, int64_t ticket, int64_t* idx, double* tau, int64_t* nd,
                     ktau_latency* lat, int64_t timeout_ms) {
  if (!s) return KTAU_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return KTAU_EINVAL;
  Request* r = it->second.get();
  auto ready = [&] { return r->state == sched::kDone; };
  if (timeout_ms < 0) {
    s->cv_done.wait(lk, ready);
  } else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready)) {
    return KTAU_ETIMEDOUT;
  }
  const int st = r->status;
  if (st == KTAU_OK) {
    if (idx) memcpy(idx, r->idx.data(), r->idx.size() * sizeof(int64_t));
    if (tau) memcpy(tau, r->tau.data(), r->tau.size() * sizeof(double));
    if (nd) memcpy(nd, r->nd.data(), r->nd.size() * sizeof(int64_t));
  }
  if (lat) {
    using us = std::chrono::duration<double, std::micro>;
    lat->queue_us = us(r->t_start - r->t_submit).count();
    lat->device_us = us(r->t_done - r->t_start).count();
    lat->total_us = us(r->t_done - r->t_submit).count();
    lat->batch_queries = r->batch_queries;
    lat->batch_requests = r->batch_requests;
  }
  s->reqs.erase(it);
  return st;
}

int ktau_server_cancel(ktau_server* s, int64_t ticket) {
  if (!s) return KTAU_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return KTAU_EINVAL;
  Request* r = it->second.get();
  if (r->state != sched::kQueued || !s->sched->cancel(r)) return KTAU_EBUSY;
  r->state = sched::kDone;
  r->status = KTAU_ECANCELED;
  r->t_start = r->t_done = sched::Clock::now();
  s->cv_done.notify_all();
  return KTAU_OK;
}

int ktau_server_inject_failure(ktau_server* s, int64_t ticket) {
  if (!s) return KTAU_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end() || it->second->state != sched::kQueued) return KTAU_EBUSY;
  it->second->force_fail = true;
  return KTAU_OK;
}

int ktau_server_pause(ktau_server* s, int paused) {
  if (!s) return KTAU_EINVAL;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->sched->set_paused(paused != 0);
    ++s->epoch;
  }
  s->cv_work.notify_all();
  return KTAU_OK;
}

int ktau_server_stats(ktau_server* s, ktau_server_counters* out) {
  if (!s || !out) return KTAU_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  const sched::Stats& st = s->sched->stats();
  out->launches = st.launches;
  out->merged_requests = st.merged;
  out->completed = st.completed;
  out->failed = st.failed;
  out->peak_pool_bytes = (int64_t)st.peak_bytes;
  out->peak_running = st.peak_running;
  out->queued = (int64_t)s->sched->queued();
  return KTAU_OK;
}

size_t ktau_server_launch_bytes(const ktau_server* s, int64_t nq, int64_t k) {
  if (!s || nq < 1 || k < 1) return 0;
  return sched::Pool::round(s->ex->bytes_for(nq, k));
}

void ktau_server_destroy(ktau_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->sched->set_paused(false);   // what is queued is still served
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  s->sched.reset();
  s->ex.reset();
  if (s->pool) (void)hipFree(s->pool);
  delete s;
}

}  // extern "C"
