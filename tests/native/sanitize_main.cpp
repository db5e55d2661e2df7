// Host-side code under AddressSanitizer and UndefinedBehaviorSanitizer: the
// CPU oracle (linked from oracle/ktau_oracle.c), the query server's
// scheduling core with a fake executor (the test shim), and the plain
// launch's tile schedule.  Exits non-zero on the first failed check; the
// sanitizers abort on the first finding.  Host code only.
#include <stdint.h>
#include <stdio.h>

#include <random>
#include <set>
#include <vector>

#include "ktau_order.h"
#include "sched_shim.cpp"

extern "C" {
typedef struct {
  int64_t nc, nd, n1, n2, n3;
} ko_counts;
void ko_pair_brute(const float* u, const float* v, int64_t n, ko_counts* c);
int ko_pair_gse(const float* u, const float* v, int64_t n, ko_counts* c);
int ko_allpairs(const float* X, int64_t m, int64_t n, int method, int threads, int64_t* nc,
                int64_t* nd, int64_t* n3, double* tau_b, double* tau_a, int64_t* n1row);
int ko_rank_rows(const float* X, int64_t m, int64_t n, int32_t* order, int32_t* rank,
                 int64_t* n1);
int ko_query_topk(const float* db, int64_t m, int64_t n, const float* q, int64_t nq, int64_t k,
                  int threads, int64_t* idx_out, double* tau_out, int64_t* nd_out);
int ko_enumerate_pairs(int64_t m, int64_t* ys, int64_t* xs);
}

#define CHECK(c)                                            \
  do {                                                      \
    if (!(c)) {                                             \
      fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
      return 1;                                             \
    }                                                       \
  } while (0)

static int oracle_checks() {
  std::mt19937 rng(7);
  for (int n = 2; n <= 300; n += (n < 40 ? 1 : 37)) {
    for (int rep = 0; rep < 3; ++rep) {
      const int levels = 1 + (int)(rng() % (unsigned)n);
      std::vector<float> u(n), v(n);
      for (int i = 0; i < n; ++i) {
        u[i] = (float)(rng() % (unsigned)levels);
        v[i] = (float)(rng() % (unsigned)(1 + rng() % (unsigned)n));
      }
      ko_counts a, b;
      ko_pair_brute(u.data(), v.data(), n, &a);
      CHECK(ko_pair_gse(u.data(), v.data(), n, &b) == 0);
      CHECK(a.nc == b.nc && a.nd == b.nd && a.n1 == b.n1 && a.n2 == b.n2 && a.n3 == b.n3);
    }
  }
  const int64_t m = 17, n = 33, P = m * (m - 1) / 2;
  std::vector<float> X(m * n);
  for (auto& x : X) x = (float)(rng() % 5u);
  std::vector<int64_t> nc(P), nd(P), n3(P), n1(m), ys(P), xs(P);
  std::vector<double> tb(P), ta(P);
  for (int method = 0; method < 2; ++method)
    CHECK(ko_allpairs(X.data(), m, n, method, 1, nc.data(), nd.data(), n3.data(), tb.data(),
                      ta.data(), n1.data()) == 0);
  std::vector<int32_t> order(m * n), rank(m * n);
  CHECK(ko_rank_rows(X.data(), m, n, order.data(), rank.data(), n1.data()) == 0);
  CHECK(ko_enumerate_pairs(m, ys.data(), xs.data()) == 0);
  const int64_t k = 40;   // more than m: padded results
  std::vector<int64_t> idx(3 * k), ndo(3 * k);
  std::vector<double> tau(3 * k);
  CHECK(ko_query_topk(X.data(), m, n, X.data(), 3, k, 1, idx.data(), tau.data(), ndo.data()) ==
        0);
  return 0;
}

static int scheduler_checks() {
  for (unsigned seed = 1; seed <= 20; ++seed) CHECK(st_pool_fuzz(1 << 20, 400, seed) == 1);
  void* w = st_create(3, 64, 100000, 1000);
  std::mt19937 rng(11);
  std::vector<long long> tickets;
  for (int round = 0; round < 200; ++round) {
    const unsigned op = rng() % 4u;
    if (op == 0) {
      const long long t = st_submit(w, 1 + rng() % 64u, rng() % 2u ? 100 : 10, rng() % 17u == 0);
      if (t >= 0) tickets.push_back(t);
    } else if (op == 1) {
      st_step(w);
    } else if (op == 2) {
      st_finish_slot(w, (int)(rng() % 3u));
      st_step(w);
    } else if (!tickets.empty()) {
      st_cancel(w, tickets[rng() % tickets.size()]);
    }
    CHECK(st_pool_used(w) <= 100000);
    CHECK(st_running(w) <= 3);
  }
  for (int i = 0; i < 500 && (st_queued(w) > 0 || st_running(w) > 0); ++i) {
    for (int s = 0; s < 3; ++s) st_finish_slot(w, s);
    st_step(w);
  }
  CHECK(st_queued(w) == 0 && st_running(w) == 0 && st_pool_used(w) == 0);
  st_destroy(w);
  return 0;
}

static int order_checks() {
  for (int64_t w = 1; w <= 120; ++w) {
    const int64_t T = w * (w + 1) / 2;
    std::set<int64_t> seen;
    for (int64_t b = 0; b < T; ++b) {
      int64_t y, x;
      ktau::scheduled_tile(w, T, b, y, x);
      CHECK(0 <= y && y <= x && x < w);
      seen.insert(y * w + x);
    }
    CHECK((int64_t)seen.size() == T);
  }
  return 0;
}

int main() {
  if (oracle_checks()) return 1;
  if (scheduler_checks()) return 1;
  if (order_checks()) return 1;
  printf("sanitized host checks passed\n");
  return 0;
}
