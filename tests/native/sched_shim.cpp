// Test shim: drives the server's scheduling core (ktau_sched.h) with a fake
// executor whose launches finish only when the test says so.  Host code only.
#include <memory>
#include <vector>

#include "ktau_sched.h"

using namespace ktau::sched;

namespace {

struct Fake : Executor {
  size_t per_query = 1000;
  std::vector<bool> done;          // per slot
  // regions with work still "in flight" (enqueued by a start that failed,
  // not yet drained), and tickets whose start fails after enqueueing
  std::vector<std::pair<size_t, size_t>> inflight;
  std::vector<int64_t> fail_start;
  int overlaps = 0, abandoned = 0;
  size_t bytes_for(int64_t nq, int64_t) const override { return (size_t)nq * per_query; }
  int start(Launch& l) override {
    done[l.slot] = false;
    for (auto& r : inflight)
      if (l.off < r.first + r.second && r.first < l.off + l.bytes) ++overlaps;
    for (int64_t t : fail_start)
      if (!l.reqs.empty() && l.reqs[0]->ticket == t) {
        inflight.push_back({l.off, l.bytes});   // work enqueued, then an error
        return -4;
      }
    return 0;
  }
  void abandon(Launch& l) override {
    ++abandoned;
    for (auto it = inflight.begin(); it != inflight.end(); ++it)
      if (it->first == l.off) {
        inflight.erase(it);
        break;
      }
  }
  bool finished(const Launch& l) override { return done[l.slot]; }
  int collect(Launch& l) override {
    for (Request* r : l.reqs) {
      r->idx.assign((size_t)(r->nq * r->k), r->ticket);
      r->nd.assign(1, l.k);   // the k the launch ran
    }
    return 0;
  }
};

struct World {
  Fake ex;
  std::unique_ptr<Scheduler> s;
  std::vector<std::unique_ptr<Request>> reqs;
  std::vector<int> slot_of;        // ticket -> slot while running
};

}  // namespace

extern "C" {

void* st_create(int slots, long long max_batch, long long budget, long long per_query) {
  World* w = new World();
  w->ex.per_query = (size_t)per_query;
  w->ex.done.assign(slots, false);
  Config c;
  c.slots = slots;
  c.max_batch_queries = max_batch;
  c.budget = (size_t)budget;
  w->s = std::make_unique<Scheduler>(c, &w->ex);
  return w;
}

void st_pause(void* p, int paused) { ((World*)p)->s->set_paused(paused != 0); }

long long st_launch_k(void* p, long long t) {
  const Request* r = ((World*)p)->reqs[(size_t)t].get();
  return r->nd.empty() ? -1 : r->nd[0];
}

long long st_submit(void* p, long long nq, long long k, int force_fail) {
  World* w = (World*)p;
  if (!w->s->fits_ever(nq, k)) return -1;
  auto r = std::make_unique<Request>();
  r->ticket = (int64_t)w->reqs.size();
  r->nq = nq;
  r->k = k;
  r->force_fail = force_fail != 0;
  r->t_submit = Clock::now();
  w->s->enqueue(r.get());
  w->reqs.push_back(std::move(r));
  return w->reqs.back()->ticket;
}

int st_step(void* p) { return (int)((World*)p)->s->step().size(); }

void st_finish_slot(void* p, int slot) { ((World*)p)->ex.done[slot] = true; }
void st_fail_start(void* p, long long t) { ((World*)p)->ex.fail_start.push_back(t); }
int st_overlaps(void* p) { return ((World*)p)->ex.overlaps; }
int st_abandoned(void* p) { return ((World*)p)->ex.abandoned; }
int st_inflight(void* p) { return (int)((World*)p)->ex.inflight.size(); }

int st_state(void* p, long long t) { return ((World*)p)->reqs[t]->state; }
int st_status(void* p, long long t) { return ((World*)p)->reqs[t]->status; }
long long st_batch_requests(void* p, long long t) { return ((World*)p)->reqs[t]->batch_requests; }
long long st_batch_queries(void* p, long long t) { return ((World*)p)->reqs[t]->batch_queries; }
long long st_result0(void* p, long long t) {
  auto& r = ((World*)p)->reqs[t];
  return r->idx.empty() ? -1 : r->idx[0];
}
long long st_pool_used(void* p) { return (long long)((World*)p)->s->pool_used(); }
long long st_running(void* p) { return ((World*)p)->s->running(); }
long long st_queued(void* p) { return (long long)((World*)p)->s->queued(); }
int st_cancel(void* p, long long t) {
  World* w = (World*)p;
  return w->s->cancel(w->reqs[t].get()) ? 1 : 0;
}
long long st_peak_running(void* p) { return ((World*)p)->s->stats().peak_running; }
void st_destroy(void* p) { delete (World*)p; }

// Pool allocator exercise: n random alloc/free rounds; returns 1 if every
// allocation stayed inside [0, cap) without overlap and all memory returned.
int st_pool_fuzz(long long cap, int rounds, unsigned seed) {
  Pool pool((size_t)cap);
  std::vector<std::pair<size_t, size_t>> live;
  unsigned x = seed;
  for (int i = 0; i < rounds; ++i) {
    x = x * 1664525u + 1013904223u;
    if ((x >> 16) % 3 != 0 || live.empty()) {
      const size_t b = 1 + (x % (unsigned)(cap / 8));
      size_t off;
      if (pool.alloc(b, &off)) {
        const size_t rb = Pool::round(b);
        if (off + rb > pool.capacity()) return 0;
        for (auto& l : live)
          if (off < l.first + l.second && l.first < off + rb) return 0;
        live.push_back({off, rb});
      }
    } else {
      const size_t j = (x >> 8) % live.size();
      pool.release(live[j].first, live[j].second);
      live.erase(live.begin() + (long)j);
    }
  }
  for (auto& l : live) pool.release(l.first, l.second);
  size_t off;
  return pool.used() == 0 && pool.alloc(pool.capacity(), &off) ? 1 : 0;
}

}  // extern "C"
