/*
 * ktau_oracle.c -- plain, slow, obviously correct CPU oracle for exact
 * Kendall's tau over the strict upper triangle of an m x n float32 matrix.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no source, header, table or helper with the
 * HIP library.
 *
 * Paper: Liu, Pan, Green, Aluru, "Parallelized Kendall's Tau Coefficient
 * Computation via SIMD Vectorized Sorting on Many-Integrated-Core Processors".
 *
 * Two independent pair routines:
 *   A  ko_pair_brute  -- the definition (Sec. 1; Sec. 3.1 generalised from
 *                        tau_A to all five counts): every sample pair a<b is
 *                        classified by float comparisons.  O(n^2).
 *   B  ko_pair_gse    -- the paper's sorting-enabled kernel (Sec. 3.2, Steps
 *                        1-5): sort the joint pairs by (u, v), scan for n1
 *                        and n3, count the strictly decreasing pairs of v in
 *                        that order (Step 3, by a top-down merge count written
 *                        from that definition), scan for n2, numerator from
 *                        the tie counts.  O(n log n).
 * Readings of the paper taken here (each also listed in the design notes):
 *   - ties are IEEE float32 equality, so -0.0 ties with +0.0; NaN is refused;
 *   - Step 3 counts a pair only when v strictly decreases (equal v is a tie,
 *     not a discordant pair), whatever merge schedule reaches the count;
 *   - tau_B = (double)(nc-nd) / sqrt((double)(n0-n1) * (double)(n0-n2)),
 *     IEEE round-to-nearest, no fused multiply-add; 0/0 gives NaN;
 *   - the all-pairs output is the strict upper triangle (y < x), numbered
 *     row-major (Sec. 4.1 numbering with the diagonal left out);
 *   - the permutation test (Sec. 1 mentions it for P-values) permutes the
 *     samples of the pair's second row by caller-given permutations and
 *     counts those with |n_c - n_d| at least the observed one; the P-value is
 *     (1 + count) / (B + 1).
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC -ffp-contract=off (no fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define KO_OK 0
#define KO_EINVAL -1
#define KO_ENAN -6
#define KO_ENOMEM -3

typedef struct {
  int64_t nc, nd, n1, n2, n3;
} ko_counts;

/* ---- Routine A: the definition (Sec. 1 and Sec. 3.1) -------------------- */

/* Sign of a comparison, by comparisons only (no subtraction, so no overflow
 * or flush-to-zero can change it). */
static int ko_cmp(float a, float b) { return (a > b) - (a < b); }

void ko_pair_brute(const float* u, const float* v, int64_t n, ko_counts* c) {
  int64_t nc = 0, nd = 0, n1 = 0, n2 = 0, n3 = 0;
  for (int64_t a = 0; a < n; ++a) {
    for (int64_t b = a + 1; b < n; ++b) {
      int su = ko_cmp(u[a], u[b]);
      int sv = ko_cmp(v[a], v[b]);
      if (su == 0) n1++;
      if (sv == 0) n2++;
      if (su == 0 && sv == 0) n3++;
      if (su * sv > 0) nc++;
      if (su * sv < 0) nd++;
    }
  }
  c->nc = nc; c->nd = nd; c->n1 = n1; c->n2 = n2; c->n3 = n3;
}

/* ---- Routine B: the sorting-enabled kernel (Sec. 3.2) ------------------- */

typedef struct {
  float u, v;
} ko_joint;

/* Step 1 order: first by u, then by v (ascending). */
static int ko_joint_cmp(const void* pa, const void* pb) {
  const ko_joint* a = (const ko_joint*)pa;
  const ko_joint* b = (const ko_joint*)pb;
  int c = ko_cmp(a->u, b->u);
  if (c != 0) return c;
  return ko_cmp(a->v, b->v);
}

/* Step 3: n_d is the number of index pairs i < j of the (u, v)-ordered
 * sequence whose v values are strictly decreasing, v_i > v_j (Sec. 3.2; the
 * count does not depend on which merge tree reaches it).  Counted top-down:
 * split the index range into a lower and an upper half, count inside each
 * half (which leaves each half ordered by v), then add the pairs with i in the
 * lower and j in the upper half: for every upper element, in ascending v, the
 * lower elements with a strictly larger v -- all lower elements except those
 * with v at or below it, which a single pointer over the ordered lower half
 * counts.  The two halves are then merged by v (lower first on equal v) so the
 * caller sees its range ordered by v.  tmp holds n entries. */
static int64_t ko_inversions(ko_joint* a, ko_joint* tmp, int64_t n) {
  if (n < 2) return 0;
  const int64_t h = n / 2;
  int64_t count = ko_inversions(a, tmp, h) + ko_inversions(a + h, tmp, n - h);
  int64_t at_or_below = 0;
  for (int64_t j = h; j < n; ++j) {
    while (at_or_below < h && a[at_or_below].v <= a[j].v) ++at_or_below;
    count += h - at_or_below;
  }
  int64_t i = 0, j = h, p = 0;
  while (i < h || j < n) {
    if (j == n || (i < h && a[i].v <= a[j].v)) tmp[p++] = a[i++];
    else tmp[p++] = a[j++];
  }
  memcpy(a, tmp, (size_t)n * sizeof(ko_joint));
  return count;
}

/* Number of tied pairs sum t(t-1)/2 over runs of equal keys in a sorted list;
 * key selects u (0), v (1) or the joint pair (2). */
static int64_t ko_run_pairs(const ko_joint* s, int64_t n, int key) {
  int64_t total = 0, run = 1;
  for (int64_t k = 1; k <= n; ++k) {
    int same = 0;
    if (k < n) {
      if (key == 0) same = s[k].u == s[k - 1].u;
      else if (key == 1) same = s[k].v == s[k - 1].v;
      else same = s[k].u == s[k - 1].u && s[k].v == s[k - 1].v;
    }
    if (same) {
      run++;
    } else {
      total += run * (run - 1) / 2;
      run = 1;
    }
  }
  return total;
}

/* Steps 1-5 for one pair; work must hold 2n joint entries. */
static void ko_pair_gse_work(const float* u, const float* v, int64_t n,
                             ko_counts* c, ko_joint* work) {
  ko_joint* pairs = work;
  ko_joint* buffer = work + n;
  for (int64_t i = 0; i < n; ++i) {
    pairs[i].u = u[i];
    pairs[i].v = v[i];
  }
  qsort(pairs, (size_t)n, sizeof(ko_joint), ko_joint_cmp);   /* Step 1 */
  int64_t n1 = ko_run_pairs(pairs, n, 0);                    /* Step 2 */
  int64_t n3 = ko_run_pairs(pairs, n, 2);
  int64_t nd = ko_inversions(pairs, buffer, n);              /* Step 3 */
  int64_t n2 = ko_run_pairs(pairs, n, 1);                    /* Step 4 */
  int64_t n0 = n * (n - 1) / 2;                              /* Step 5 */
  c->nd = nd;
  c->nc = n0 - n1 - n2 + n3 - nd;
  c->n1 = n1; c->n2 = n2; c->n3 = n3;
}

int ko_pair_gse(const float* u, const float* v, int64_t n, ko_counts* c) {
  ko_joint* work = (ko_joint*)malloc((size_t)(2 * (n > 0 ? n : 1)) * sizeof(ko_joint));
  if (!work) return KO_ENOMEM;
  ko_pair_gse_work(u, v, n, c, work);
  free(work);
  return KO_OK;
}

/* ---- tau from the counts (Eq. 1 and Eq. 3) ------------------------------ */

void ko_tau(const ko_counts* c, int64_t n, double* tau_b, double* tau_a) {
  int64_t n0 = n * (n - 1) / 2;
  double num = (double)(c->nc - c->nd);
  double d1 = (double)(n0 - c->n1);
  double d2 = (double)(n0 - c->n2);
  double prod = d1 * d2;
  double den = sqrt(prod);
  if (tau_b) *tau_b = den == 0.0 ? (double)NAN : num / den;
  if (tau_a) *tau_a = n0 == 0 ? (double)NAN : num / (double)n0;
}

/* ---- validation --------------------------------------------------------- */

static int ko_has_nan(const float* X, int64_t count) {
  for (int64_t i = 0; i < count; ++i)
    if (X[i] != X[i]) return 1;
  return 0;
}

/* ---- strict upper-triangle all-pairs ------------------------------------ */

/* Row-major enumeration of the strict upper triangle: row y owns m-1-y jobs,
 * so its first job id is the running sum of the earlier rows' lengths. */
static int64_t* ko_row_starts(int64_t m) {
  int64_t* start = (int64_t*)malloc((size_t)(m + 1) * sizeof(int64_t));
  if (!start) return NULL;
  int64_t acc = 0;
  for (int64_t y = 0; y < m; ++y) {
    start[y] = acc;
    acc += m - 1 - y;
  }
  start[m] = acc;
  return start;
}

/* Enumerates every strict pair in row-major order; ys/xs receive m(m-1)/2
 * entries each.  Used by the tests to check the library's job mapper. */
int ko_enumerate_pairs(int64_t m, int64_t* ys, int64_t* xs) {
  if (m < 0) return KO_EINVAL;
  int64_t j = 0;
  for (int64_t y = 0; y < m; ++y)
    for (int64_t x = y + 1; x < m; ++x) {
      ys[j] = y;
      xs[j] = x;
      ++j;
    }
  return KO_OK;
}

static void ko_store(int64_t j, const ko_counts* c, int64_t n, int64_t* nc,
                     int64_t* nd, int64_t* n3, double* tau_b, double* tau_a) {
  if (nc) nc[j] = c->nc;
  if (nd) nd[j] = c->nd;
  if (n3) n3[j] = c->n3;
  if (tau_b || tau_a) {
    double tb, ta;
    ko_tau(c, n, &tb, &ta);
    if (tau_b) tau_b[j] = tb;
    if (tau_a) tau_a[j] = ta;
  }
}

/* Tie term of every row on its own: n1 of row r is sum t(t-1)/2 over the
 * groups of equal values in that row (the per-vector half of Steps 2/4). */
static int64_t ko_row_tie_pairs(const float* row, int64_t n, ko_joint* work) {
  for (int64_t i = 0; i < n; ++i) {
    work[i].u = row[i];
    work[i].v = 0.0f;
  }
  qsort(work, (size_t)n, sizeof(ko_joint), ko_joint_cmp);
  return ko_run_pairs(work, n, 0);
}

/* method: 0 = routine A (definition), 1 = routine B (sorting kernel).
 * Outputs (any may be NULL) are indexed by the strict row-major job id.
 * threads <= 0 means the OpenMP default. */
int ko_allpairs(const float* X, int64_t m, int64_t n, int method, int threads,
                int64_t* nc, int64_t* nd, int64_t* n3, double* tau_b,
                double* tau_a, int64_t* n1row) {
  if (m < 2 || n < 2 || !X) return KO_EINVAL;
  if (ko_has_nan(X, m * n)) return KO_ENAN;
  int64_t* start = ko_row_starts(m);
  if (!start) return KO_ENOMEM;
  int fail = 0;
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
#else
  (void)threads;
#endif
#pragma omp parallel
  {
    ko_joint* work = (ko_joint*)malloc((size_t)(2 * n) * sizeof(ko_joint));
    if (!work) {
#pragma omp atomic write
      fail = 1;
    }
    /* every thread reaches the worksharing loop; one without memory idles */
#pragma omp for schedule(dynamic, 1)
    for (int64_t y = 0; y < m; ++y) {
      if (work) {
        const float* u = X + y * n;
        if (n1row) n1row[y] = ko_row_tie_pairs(u, n, work);
        for (int64_t x = y + 1; x < m; ++x) {
          const float* v = X + x * n;
          ko_counts c;
          if (method == 0) ko_pair_brute(u, v, n, &c);
          else ko_pair_gse_work(u, v, n, &c, work);
          ko_store(start[y] + (x - y - 1), &c, n, nc, nd, n3, tau_b, tau_a);
        }
      }
    }
    free(work);
  }
  free(start);
  return fail ? KO_ENOMEM : KO_OK;
}

/* Selected pairs (ys[i], xs[i]) of one matrix, results in slot i.  The pair
 * is evaluated with u = row ys[i] and v = row xs[i] exactly as given. */
int ko_pairs(const float* X, int64_t m, int64_t n, const int64_t* ys,
             const int64_t* xs, int64_t count, int method, int threads,
             int64_t* nc, int64_t* nd, int64_t* n3, int64_t* n1,
             int64_t* n2, double* tau_b, double* tau_a) {
  if (m < 1 || n < 2 || !X || count < 0) return KO_EINVAL;
  for (int64_t i = 0; i < count; ++i)
    if (ys[i] < 0 || ys[i] >= m || xs[i] < 0 || xs[i] >= m) return KO_EINVAL;
  int fail = 0;
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
#else
  (void)threads;
#endif
#pragma omp parallel
  {
    ko_joint* work = (ko_joint*)malloc((size_t)(2 * n) * sizeof(ko_joint));
    if (!work) {
#pragma omp atomic write
      fail = 1;
    }
#pragma omp for schedule(dynamic, 16)
    for (int64_t i = 0; i < count; ++i) {
      if (work) {
        const float* u = X + ys[i] * n;
        const float* v = X + xs[i] * n;
        ko_counts c;
        if (ko_has_nan(u, n) || ko_has_nan(v, n)) {
#pragma omp atomic write
          fail = 2;
          continue;
        }
        if (method == 0) ko_pair_brute(u, v, n, &c);
        else ko_pair_gse_work(u, v, n, &c, work);
        ko_store(i, &c, n, nc, nd, n3, tau_b, tau_a);
        if (n1) n1[i] = c.n1;
        if (n2) n2[i] = c.n2;
      }
    }
    free(work);
  }
  if (fail == 2) return KO_ENAN;
  return fail ? KO_ENOMEM : KO_OK;
}

/* ---- permutation test (Sec. 1: P-values of tau by permutation test) ----- */

/* 1 if row b of perms (n entries) is a permutation of 0..n-1. */
static int ko_is_permutation(const uint16_t* p, int64_t n, unsigned char* seen) {
  memset(seen, 0, (size_t)n);
  for (int64_t t = 0; t < n; ++t) {
    if ((int64_t)p[t] >= n || seen[p[t]]) return 0;
    seen[p[t]] = 1;
  }
  return 1;
}

/* For selected pairs (ys[i], xs[i]): S = n_c - n_d of u = row ys[i] against
 * v = row xs[i], and S_b of u against v with its samples permuted by each of
 * the B permutations (v_b[t] = v[perms[b n + t]]).  count_out[i] = number of
 * b with |S_b| >= |S|; p_out[i] = (1 + count) / (B + 1).  The two tie terms
 * of tau_B do not change when v's samples are permuted, so |tau_B| orders the
 * permutations as |S| does. */
int ko_perm_test(const float* X, int64_t m, int64_t n, const uint16_t* perms, int64_t B,
                 const int64_t* ys, const int64_t* xs, int64_t count, int method,
                 int threads, int64_t* count_out, double* p_out) {
  if (m < 1 || n < 2 || !X || !perms || B < 1 || count < 0) return KO_EINVAL;
  for (int64_t i = 0; i < count; ++i)
    if (ys[i] < 0 || ys[i] >= m || xs[i] < 0 || xs[i] >= m) return KO_EINVAL;
  if (ko_has_nan(X, m * n)) return KO_ENAN;
  unsigned char* seen = (unsigned char*)malloc((size_t)n);
  if (!seen) return KO_ENOMEM;
  for (int64_t b = 0; b < B; ++b)
    if (!ko_is_permutation(perms + b * n, n, seen)) {
      free(seen);
      return KO_EINVAL;
    }
  free(seen);
  int fail = 0;
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
#else
  (void)threads;
#endif
#pragma omp parallel
  {
    ko_joint* work = (ko_joint*)malloc((size_t)(2 * n) * sizeof(ko_joint));
    float* vb = (float*)malloc((size_t)n * sizeof(float));
    if (!work || !vb) {
#pragma omp atomic write
      fail = 1;
    }
#pragma omp for schedule(dynamic, 4)
    for (int64_t i = 0; i < count; ++i) {
      if (!work || !vb) continue;
      const float* u = X + ys[i] * n;
      const float* v = X + xs[i] * n;
      ko_counts c;
      if (method == 0) ko_pair_brute(u, v, n, &c);
      else ko_pair_gse_work(u, v, n, &c, work);
      const int64_t s_obs = llabs(c.nc - c.nd);
      int64_t ge = 0;
      for (int64_t b = 0; b < B; ++b) {
        for (int64_t t = 0; t < n; ++t) vb[t] = v[perms[b * n + t]];
        if (method == 0) ko_pair_brute(u, vb, n, &c);
        else ko_pair_gse_work(u, vb, n, &c, work);
        if (llabs(c.nc - c.nd) >= s_obs) ++ge;
      }
      count_out[i] = ge;
      if (p_out) p_out[i] = (double)(1 + ge) / (double)(B + 1);
    }
    free(work);
    free(vb);
  }
  return fail ? KO_ENOMEM : KO_OK;
}

/* ---- per-row ordering (the rank transform of Sec. 3) -------------------- */

typedef struct {
  float val;
  int64_t idx;
} ko_keyed;

/* Ascending value, equal values by sample index (a stable order). */
static int ko_keyed_cmp(const void* pa, const void* pb) {
  const ko_keyed* a = (const ko_keyed*)pa;
  const ko_keyed* b = (const ko_keyed*)pb;
  int c = ko_cmp(a->val, b->val);
  if (c != 0) return c;
  return (a->idx > b->idx) - (a->idx < b->idx);
}

/* For each row: order[k] = sample at sorted position k (stable ascending),
 * rank[i] = number of distinct values strictly below x[i] (dense rank),
 * n1[r] = sum t(t-1)/2 over tie groups.  Any output may be NULL. */
int ko_rank_rows(const float* X, int64_t m, int64_t n, int32_t* order,
                 int32_t* rank, int64_t* n1) {
  if (m < 1 || n < 1 || !X) return KO_EINVAL;
  if (ko_has_nan(X, m * n)) return KO_ENAN;
  ko_keyed* w = (ko_keyed*)malloc((size_t)n * sizeof(ko_keyed));
  if (!w) return KO_ENOMEM;
  for (int64_t r = 0; r < m; ++r) {
    const float* row = X + r * n;
    for (int64_t i = 0; i < n; ++i) {
      w[i].val = row[i];
      w[i].idx = i;
    }
    qsort(w, (size_t)n, sizeof(ko_keyed), ko_keyed_cmp);
    int64_t dense = 0, run = 1, ties = 0;
    for (int64_t k = 0; k < n; ++k) {
      if (k > 0) {
        if (w[k].val == w[k - 1].val) {
          run++;
        } else {
          dense++;
          ties += run * (run - 1) / 2;
          run = 1;
        }
      }
      if (order) order[r * n + k] = (int32_t)w[k].idx;
      if (rank) rank[r * n + w[k].idx] = (int32_t)dense;
    }
    ties += run * (run - 1) / 2;
    if (n1) n1[r] = ties;
  }
  free(w);
  return KO_OK;
}

/* ---- query search (Sec. 1: rank subject rows by their score) ------------ */

typedef struct {
  double key;
  int64_t idx;
} ko_scored;

/* Larger |tau| first, then smaller database index. */
static int ko_scored_cmp(const void* pa, const void* pb) {
  const ko_scored* a = (const ko_scored*)pa;
  const ko_scored* b = (const ko_scored*)pb;
  if (a->key > b->key) return -1;
  if (a->key < b->key) return 1;
  return (a->idx > b->idx) - (a->idx < b->idx);
}

/* For each of the nq query rows (length n) against all m database rows:
 * tau_B by routine B with u = query, v = database row; the k rows of largest
 * |tau_B| (NaN excluded), ties by smaller index; missing slots are idx -1,
 * tau NaN, nd -1. */
int ko_query_topk(const float* db, int64_t m, int64_t n, const float* q,
                  int64_t nq, int64_t k, int threads, int64_t* idx_out,
                  double* tau_out, int64_t* nd_out) {
  if (m < 1 || n < 2 || nq < 0 || k < 1 || !db || (nq > 0 && !q))
    return KO_EINVAL;
  if (ko_has_nan(db, m * n) || ko_has_nan(q, nq * n)) return KO_ENAN;
  int fail = 0;
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
#else
  (void)threads;
#endif
#pragma omp parallel
  {
    ko_joint* work = (ko_joint*)malloc((size_t)(2 * n) * sizeof(ko_joint));
    ko_scored* sc = (ko_scored*)malloc((size_t)m * sizeof(ko_scored));
    double* taus = (double*)malloc((size_t)m * sizeof(double));
    int64_t* nds = (int64_t*)malloc((size_t)m * sizeof(int64_t));
    int ok = work && sc && taus && nds;
    if (!ok) {
#pragma omp atomic write
      fail = 1;
    }
#pragma omp for schedule(dynamic, 1)
    for (int64_t qi = 0; qi < nq; ++qi) {
      if (ok) {
        const float* u = q + qi * n;
        int64_t valid = 0;
        for (int64_t j = 0; j < m; ++j) {
          ko_counts c;
          ko_pair_gse_work(u, db + j * n, n, &c, work);
          double tb;
          ko_tau(&c, n, &tb, NULL);
          taus[j] = tb;
          nds[j] = c.nd;
          if (tb == tb) {
            sc[valid].key = fabs(tb);
            sc[valid].idx = j;
            valid++;
          }
        }
        qsort(sc, (size_t)valid, sizeof(ko_scored), ko_scored_cmp);
        for (int64_t t = 0; t < k; ++t) {
          int64_t o = qi * k + t;
          if (t < valid) {
            idx_out[o] = sc[t].idx;
            if (tau_out) tau_out[o] = taus[sc[t].idx];
            if (nd_out) nd_out[o] = nds[sc[t].idx];
          } else {
            idx_out[o] = -1;
            if (tau_out) tau_out[o] = (double)NAN;
            if (nd_out) nd_out[o] = -1;
          }
        }
      }
    }
    free(work);
    free(sc);
    free(taus);
    free(nds);
  }
  return fail ? KO_ENOMEM : KO_OK;
}

int ko_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
