// Batched all-pairs over many independent matrices of uneven (m, n), and the
// autotuner that picks the per-pair scheme and tile edge for each sample-count
// class.
//
// A batch plan owns one device arena: a shared status word, one rank
// workspace per matrix (the plain layout), the descriptor table and the unit
// (tile) and row prefixes.  One run is: clear status and tile counters; one
// pre-pass launch over every row of every matrix; for each scheme class
// present, one persistent pair launch whose workgroups take tiles of any
// matrix of the class from atomic counters (Sec. 4.1 notes a shared counter
// balances jobs of varied cost), each kernel with its own register budget;
// the classes run one after another, the most work first (measured: class
// kernels running side by side on parallel streams slow each other down by
// about 10%); then the heavy-row and composite passes.  The sequence is
// captured once in a hipGraph and replayed.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "ktau_internal.h"

namespace ktau {
namespace {

// ------------------------------------------------------------- autotuner

// Sample-count class of n: the smallest scheme capacity that holds it.
int64_t n_class(int64_t n) {
  int64_t c = 128;
  while (c < n) c <<= 1;
  return c;
}

struct Plan {
  int scheme;
  int q;
  double pairs_per_s;
};

// Largest n of a scheme: the numbered ones, and the naive bit-set count.
int64_t plan_capacity(int s) {
  if (s == KTAU_SCHEME_NAIVE) return kBitsMaxN;
  return (s >= 0 && s < kNumSchemes) ? scheme_capacity(s) : -1;
}

std::mutex g_tune_mu;
std::map<int64_t, Plan> g_tuned;   // n class -> best plan (process-wide)

// Cache file: one line per class, "n_class scheme_name q pairs_per_s".
void load_cache(const char* path) {
  if (!path || !*path) return;
  FILE* f = fopen(path, "r");
  if (!f) return;
  char name[64];
  long long cls;
  int q;
  double pps;
  while (fscanf(f, "%lld %63s %d %lf", &cls, name, &q, &pps) == 4) {
    for (int s = 0; s <= kNumSchemes; ++s) {
      const int id = s < kNumSchemes ? s : KTAU_SCHEME_NAIVE;
      if (strcmp(name, scheme_name(id)) == 0 && plan_capacity(id) >= cls && q >= 1 && q <= 64)
        g_tuned[cls] = Plan{id, q, pps};
    }
  }
  fclose(f);
}

void save_cache(const char* path) {
  if (!path || !*path) return;
  std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return;
  for (auto& kv : g_tuned)
    fprintf(f, "%lld %s %d %.6e\n", (long long)kv.first, scheme_name(kv.second.scheme),
            kv.second.q, kv.second.pairs_per_s);
  fclose(f);
  rename(tmp.c_str(), path);
}

// Deterministic timing matrix when no data is at hand (splitmix64 of the
// index): uniform values with about 1.6% exact zeros, a tie run in every row
// as in zero-inflated expression data.
__global__ void synth_kernel(float* X, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  uint64_t z = (uint64_t)i * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  X[i] = (z & 63u) == 0 ? 0.0f : (float)(z >> 40) * (1.0f / 16777216.0f);
}

// Rows of the timing matrix for n samples: about 2^31 merge steps in total,
// so that one candidate's launch takes milliseconds.
int64_t tune_rows(int64_t n) {
  const int64_t m = (int64_t)sqrt(4.0e9 / (double)n);
  return m < 256 ? 256 : m;
}

// Candidate schemes for a class: those that hold the class without more
// than doubling the padding.
std::vector<int> candidates(int64_t cls) {
  std::vector<int> v;
  for (int s = 0; s < kNumNetSchemes; ++s)
    if (scheme_capacity(s) >= cls && scheme_capacity(s) < 2 * cls) v.push_back(s);
  // the merge schemes pad only the last chunk, so every class past one
  // wave's network is theirs too
  if (cls > 4096)
    for (int s : {(int)kMergeK32, (int)kMergeK64})
      if (scheme_capacity(s) >= cls) v.push_back(s);
  // short rows: the naive count of every sample pair from per-row bit sets
  if (cls <= kBitsMaxN) v.push_back(KTAU_SCHEME_NAIVE);
  return v;
}

// Measures every (scheme, q) candidate of class `cls` and records the
// fastest.  The timing matrix is the first rows of `src` (m_src x n_src, a
// matrix of the class from the caller's batch) when given, else a synthetic
// cls-sample matrix.
int tune_class(int64_t cls, const float* src, int64_t m_src, int64_t n_src, hipStream_t s) {
  const int64_t n = src ? n_src : cls;
  int64_t m = tune_rows(n);
  if (src && m > m_src) m = m_src;
  const WsLayout L = ws_layout(m, n);
  float* X = nullptr;
  void* ws = nullptr;
  double* tau = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = KTAU_OK;
  const int64_t P = m * (m - 1) / 2;
  const size_t bits = bits_bytes(m, n);   // 0 past kBitsMaxN
  if ((!src && hipMalloc(&X, (size_t)(m * n) * sizeof(float)) != hipSuccess) ||
      hipMalloc(&ws, L.total + bits) != hipSuccess ||
      hipMalloc(&tau, (size_t)P * sizeof(double)) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    rc = KTAU_ENOMEM;
  }
  Plan best{default_scheme(n), default_q(n), 0.0};
  if (rc == KTAU_OK) {
    if (!src)
      hipLaunchKernelGGL(synth_kernel, dim3((unsigned)((m * n + 255) / 256)), dim3(256), 0, s, X,
                         m * n);
    if (hipGetLastError() != hipSuccess || clear_words((int32_t*)ws, 2, s) != KTAU_OK ||
        prepass_ws(src ? src : X, m, n, ws, nullptr, nullptr, s) != KTAU_OK)
      rc = KTAU_EDEVICE;
    if (rc == KTAU_OK && bits > 0 &&
        launch_bits_prepass(matdesc(ws, m, n, ktau_pair_out{}, 0, 1, 0, 0, nullptr),
                            (uint32_t*)((char*)ws + L.total), s) != hipSuccess)
      rc = KTAU_EDEVICE;
  }
  if (rc == KTAU_OK) {
    ktau_pair_out out{};
    out.tau_b = tau;
    for (int scheme : candidates(cls)) {
      const int q0 = default_q(n);
      for (int q : {q0 / 2, q0, 2 * q0}) {
        if (is_merge(scheme) && q != q0) continue;   // pairs in job order, no tiles
        MatDesc d = matdesc(ws, m, n, out, scheme, q, 0, P, nullptr);
        float best_ms = 1e30f;
        for (int rep = 0; rep < 4; ++rep) {
          auto launch = [&]() {
            return scheme == KTAU_SCHEME_NAIVE
                       ? launch_bits_pairs(d, (const uint32_t*)((char*)ws + L.total), true, s)
                       : launch_pairs_plain(d, true, s);
          };
          if (hipEventRecord(e0, s) != hipSuccess || launch() != hipSuccess ||
              hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
            rc = KTAU_EDEVICE;
            break;
          }
          float ms = 0.f;
          if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) ms = 1e30f;
          if (rep > 0) best_ms = std::min(best_ms, ms);
        }
        if (rc != KTAU_OK) break;
        const double pps = (double)P / (best_ms * 1e-3);
        if (pps > best.pairs_per_s) best = Plan{scheme, q, pps};
      }
      if (rc != KTAU_OK) break;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (X) (void)hipFree(X);
  if (ws) (void)hipFree(ws);
  if (tau) (void)hipFree(tau);
  if (rc == KTAU_OK) g_tuned[cls] = best;
  return rc;
}

// Rows from which a matrix on a network scheme runs as a plain tile launch.
constexpr int64_t kTileLaunchRows = 8192;

// A class is timed on about 2^31 merge steps (a few thousand rows at most);
// tiles of a matrix of kTileLaunchRows rows or more double their edge, up to
// 16, as the plain launches do (the row fetches halve and the tiles still
// fill the chip).
int scale_q(const Plan& p, int64_t m) {
  if (m < kTileLaunchRows || is_merge(p.scheme) || p.scheme == KTAU_SCHEME_NAIVE) return p.q;
  return p.q < 8 ? p.q : 16;
}

// The plan of a matrix with n samples; a class not yet tuned is tuned on
// rep (m_rep x n_rep, may be NULL: synthetic data).
Plan plan_for(int64_t n, bool autotune, const char* cache, hipStream_t s, int* rc,
              const float* rep = nullptr, int64_t m_rep = 0, int64_t n_rep = 0) {
  const int64_t cls = n_class(n);
  if (!autotune) return Plan{default_scheme(n), default_q(n), 0.0};
  std::lock_guard<std::mutex> g(g_tune_mu);
  auto it = g_tuned.find(cls);
  if (it == g_tuned.end()) {
    load_cache(cache);
    it = g_tuned.find(cls);
  }
  if (it == g_tuned.end()) {
    *rc = tune_class(cls, rep, m_rep, n_rep, s);
    if (*rc != KTAU_OK) return Plan{default_scheme(n), default_q(n), 0.0};
    save_cache(cache);
    it = g_tuned.find(cls);
  }
  Plan p = it->second;
  if (plan_capacity(p.scheme) < n) p.scheme = default_scheme(n);
  return p;
}

}  // namespace
}  // namespace ktau

using namespace ktau;

// One scheme class of a batch: a contiguous slice of the descriptor table,
// launched as its own persistent kernel, or (tiles) as one plain tile launch
// per matrix.
struct ClassRun {
  int scheme;
  bool tiles = false;
  int64_t first, count;          // slice of the descriptor table
  int64_t total_units;
  double work = 0.0;             // estimated cost: pairs x network size
  int64_t* prefix = nullptr;     // device [count + 1], unit prefix inside the class
  int64_t* counters = nullptr;   // device: 8 tile counters (one per XCD stretch)
};

struct ktau_batch {
  int64_t count = 0;
  std::vector<MatDesc> host_descs;   // class-sorted
  std::vector<int64_t> slot;         // caller index -> descriptor position
  std::vector<ClassRun> classes;
  char* arena = nullptr;             // device memory owned by the plan
  MatDesc* descs = nullptr;          // device, class-sorted
  int64_t* row_prefix = nullptr;     // device [count + 1]
  int32_t* words = nullptr;          // device: [0] status; int64 counters from byte 64
  int clear_count = 0;               // int32 words cleared before a run
  int64_t total_rows = 0;
  int max_n = 0;
  bool use_graph = true;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap_stream = nullptr;
};

namespace {

// The whole run on stream s.
int enqueue_batch(ktau_batch* b, hipStream_t s) {
  if (clear_words(b->words, b->clear_count, s) != KTAU_OK) return KTAU_EDEVICE;
  int lds_n = 0;   // the longest rows the batched pre-pass sorts in LDS
  for (const MatDesc& d : b->host_descs)
    if (d.n <= kLdsSortMax && d.n > lds_n) lds_n = d.n;
  if (launch_prepass_batch(b->descs, b->count, b->total_rows, b->row_prefix, lds_n, s) !=
      hipSuccess)
    return KTAU_EDEVICE;
  for (const MatDesc& d : b->host_descs)
    if (d.n > kLdsSortMax &&
        launch_prepass(d.X, d.m, d.n, (uint16_t*)d.rv.perm, (uint16_t*)d.rv.rank,
                       (uint16_t*)d.rv.rstart, d.rv.ld, (int64_t*)d.rv.n1, d.n1_out,
                       (int32_t*)d.rv.nruns, (int32_t*)d.rv.nlong, (uint64_t*)d.rv.runs,
                       (int32_t*)d.status,
                       ws_doubled(d.n), d.sort_tmp, s) != hipSuccess)
      return KTAU_EDEVICE;
  for (const ClassRun& c : b->classes) {
    if (is_merge(c.scheme)) {
      // long rows: a workgroup per pair already fills the device, one launch
      // per matrix
      for (int64_t p = c.first; p < c.first + c.count; ++p)
        if (launch_pairs_merge(b->host_descs[p], s) != hipSuccess) return KTAU_EDEVICE;
      continue;
    }
    if (c.scheme == KTAU_SCHEME_NAIVE) {
      // short rows: each matrix's bit sets from its ranks, then its pairs
      for (int64_t p = c.first; p < c.first + c.count; ++p) {
        const MatDesc& d = b->host_descs[p];
        if (launch_bits_prepass(d, d.bits, s) != hipSuccess ||
            launch_bits_pairs(d, d.bits, true, s) != hipSuccess)
          return KTAU_EDEVICE;
      }
      continue;
    }
    if (c.tiles) {
      for (int64_t p = c.first; p < c.first + c.count; ++p)
        if (launch_pair_tiles(b->host_descs[p], s) != hipSuccess) return KTAU_EDEVICE;
      continue;
    }
    if (launch_pairs_persistent(c.scheme, b->descs + c.first, c.count, c.total_units, c.prefix,
                                c.counters, b->words, s) != hipSuccess)
      return KTAU_EDEVICE;
  }
  if (launch_tie_passes_batch(b->descs, b->count, b->max_n, s) != hipSuccess) return KTAU_EDEVICE;
  return KTAU_OK;
}

void free_batch(ktau_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  if (b->arena) (void)hipFree(b->arena);
  delete b;
}

}  // namespace

extern "C" {

void ktau_batch_default_opts(ktau_batch_opts* o) {
  if (!o) return;
  o->use_graph = 1;
  o->autotune = 1;
  o->force_scheme = -1;
  o->force_q = 0;
  o->tune_cache = nullptr;
}

int ktau_batch_create(const ktau_matrix* mats, int64_t count, const ktau_batch_opts* opts,
                      void* stream, ktau_batch** out) {
  if (!mats || count < 1 || !out) return KTAU_EINVAL;
  *out = nullptr;
  ktau_batch_opts o;
  ktau_batch_default_opts(&o);
  if (opts) o = *opts;
  for (int64_t i = 0; i < count; ++i) {
    const int rc = check_shape(mats[i].m, mats[i].n);
    if (rc != KTAU_OK) return rc;
    if (!mats[i].X_dev) return KTAU_EINVAL;
  }
  if ((o.force_scheme >= kNumSchemes && o.force_scheme != KTAU_SCHEME_NAIVE) || o.force_q < 0 ||
      o.force_q > 64)
    return KTAU_EINVAL;
  if (o.force_scheme >= 0)
    for (int64_t i = 0; i < count; ++i)
      if (plan_capacity(o.force_scheme) < mats[i].n) return KTAU_EINVAL;
  const hipStream_t s = (hipStream_t)stream;
  const char* cache = o.tune_cache ? o.tune_cache : getenv("KTAU_TUNE_CACHE");

  // plans (a class still to be tuned is timed on its matrix with the most
  // pairs), then the class-sorted order
  std::map<int64_t, int64_t> rep;   // n class -> matrix index
  for (int64_t i = 0; i < count; ++i) {
    auto it = rep.find(n_class(mats[i].n));
    if (it == rep.end() || mats[i].m > mats[it->second].m) rep[n_class(mats[i].n)] = i;
  }
  std::vector<Plan> plans(count);
  for (int64_t i = 0; i < count; ++i) {
    int rc = KTAU_OK;
    const ktau_matrix& r = mats[rep[n_class(mats[i].n)]];
    plans[i] = plan_for(mats[i].n, o.autotune != 0 && o.force_scheme < 0, cache, s, &rc, r.X_dev,
                        r.m, r.n);
    if (rc != KTAU_OK) return rc;
    if (o.force_scheme >= 0) plans[i].scheme = o.force_scheme;
    if (o.force_q > 0) plans[i].q = o.force_q;
    else plans[i].q = scale_q(plans[i], mats[i].m);
  }
  // Matrices of kTileLaunchRows rows or more on a network scheme run the
  // plain tile launch (a workgroup per tile, its waves sharing the tile's
  // rows; measured 8% faster than the persistent kernel's per-wave tiles at
  // 16384 x 1024, which keep four times as many rows in flight per CU); the
  // others share their scheme's persistent kernel.
  auto tiled = [&](int64_t i) {
    return mats[i].m >= kTileLaunchRows && !is_merge(plans[i].scheme) &&
           plans[i].scheme != KTAU_SCHEME_NAIVE;
  };
  std::vector<int64_t> order(count);
  for (int64_t i = 0; i < count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t c) {
    return plans[a].scheme != plans[c].scheme ? plans[a].scheme < plans[c].scheme
                                              : tiled(a) < tiled(c);
  });

  ktau_batch* b = new ktau_batch();
  b->count = count;
  b->use_graph = o.use_graph != 0;
  b->slot.resize(count);
  for (int64_t p = 0; p < count; ++p) b->slot[order[p]] = p;
  for (int64_t p = 0; p < count; ++p) {
    const int sc = plans[order[p]].scheme;
    const bool tl = tiled(order[p]);
    if (b->classes.empty() || b->classes.back().scheme != sc || b->classes.back().tiles != tl) {
      ClassRun c;
      c.scheme = sc;
      c.tiles = tl;
      c.first = p;
      c.count = 0;
      c.total_units = 0;
      b->classes.push_back(c);
    }
    b->classes.back().count++;
  }
  const int64_t ncls = (int64_t)b->classes.size();
  // arena: words (status, then 8 tile counters per class) | descs | row
  // prefix | class unit prefixes | workspaces
  const size_t words_bytes = 64 + (size_t)ncls * 8 * sizeof(int64_t);
  size_t off = (size_t)round_up((int64_t)words_bytes, (int64_t)kAlign);
  const size_t desc_off = off;
  off = (size_t)round_up((int64_t)(off + (size_t)count * sizeof(MatDesc)), (int64_t)kAlign);
  const size_t rp_off = off;
  off = (size_t)round_up((int64_t)(off + (size_t)(count + 1) * 8), (int64_t)kAlign);
  const size_t up_off = off;
  off = (size_t)round_up((int64_t)(off + (size_t)(count + ncls) * 8), (int64_t)kAlign);
  std::vector<size_t> ws_off(count);
  for (int64_t p = 0; p < count; ++p) {
    const ktau_matrix& mt = mats[order[p]];
    ws_off[p] = off;
    off += ws_layout(mt.m, mt.n).total;
    if (plans[order[p]].scheme == KTAU_SCHEME_NAIVE)
      off = (size_t)round_up((int64_t)(off + bits_bytes(mt.m, mt.n)), (int64_t)kAlign);
  }
  if (hipMalloc((void**)&b->arena, off) != hipSuccess) {
    delete b;
    return KTAU_ENOMEM;
  }
  b->words = (int32_t*)b->arena;
  b->clear_count = (int)(words_bytes / sizeof(int32_t));
  b->descs = (MatDesc*)(b->arena + desc_off);
  b->row_prefix = (int64_t*)(b->arena + rp_off);
  int64_t* up_dev = (int64_t*)(b->arena + up_off);

  std::vector<int64_t> rprefix(count + 1, 0), uprefix;
  b->host_descs.resize(count);
  for (int64_t c = 0; c < ncls; ++c) {
    ClassRun& cr = b->classes[c];
    cr.prefix = up_dev + cr.first + c;
    cr.counters = (int64_t*)(b->arena + 64) + 8 * c;
    int64_t acc = 0;
    uprefix.push_back(0);
    for (int64_t p = cr.first; p < cr.first + cr.count; ++p) {
      const ktau_matrix& mt = mats[order[p]];
      const Plan& pl = plans[order[p]];
      MatDesc d = matdesc(b->arena + ws_off[p], mt.m, mt.n, mt.out, pl.scheme, pl.q, 0,
                          mt.m * (mt.m - 1) / 2, b->words);
      d.X = mt.X_dev;
      d.n1_out = mt.out.n1;
      if (pl.scheme == KTAU_SCHEME_NAIVE)
        d.bits = (uint32_t*)(b->arena + ws_off[p] + ws_layout(mt.m, mt.n).total);
      d.unit_begin = acc;
      acc += d.n_units;
      uprefix.push_back(acc);
      cr.work += (double)(mt.m * (mt.m - 1) / 2) *
                 (double)(is_merge(pl.scheme) || pl.scheme == KTAU_SCHEME_NAIVE
                              ? mt.n
                              : scheme_capacity(pl.scheme));
      rprefix[p + 1] = rprefix[p] + mt.m;
      b->host_descs[p] = d;
      b->max_n = std::max(b->max_n, (int)mt.n);
    }
    cr.total_units = acc;
  }
  b->total_rows = rprefix[count];
  int rc = KTAU_OK;
  if (hipMemcpy(b->descs, b->host_descs.data(), (size_t)count * sizeof(MatDesc),
                hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->row_prefix, rprefix.data(), (size_t)(count + 1) * 8,
                hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(up_dev, uprefix.data(), uprefix.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
    rc = KTAU_EDEVICE;
  // the most work first
  std::stable_sort(b->classes.begin(), b->classes.end(),
                   [](const ClassRun& a, const ClassRun& c) { return a.work > c.work; });
  // query each class kernel's occupancy now, outside any capture
  for (ClassRun& c : b->classes) {
    if (rc != KTAU_OK) break;
    const hipError_t e =
        c.scheme == KTAU_SCHEME_NAIVE || c.tiles
            ? hipSuccess
            : is_merge(c.scheme)
                  ? prepare_pairs_merge(c.scheme)
                  : launch_pairs_persistent(c.scheme, b->descs, 0, 0, nullptr, nullptr, b->words, s);
    if (e != hipSuccess) rc = KTAU_EDEVICE;
  }
  if (rc != KTAU_OK) {
    free_batch(b);
    return rc;
  }
  *out = b;
  return KTAU_OK;
}

int ktau_batch_run(ktau_batch* b, void* stream) {
  if (!b) return KTAU_EINVAL;
  const hipStream_t s = (hipStream_t)stream;
  if (!b->use_graph) return enqueue_batch(b, s);
  // first run: capture the whole sequence once
  if (!b->exec) {
    if (hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess)
      return KTAU_EDEVICE;
    if (hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return KTAU_EDEVICE;
    const int rc = enqueue_batch(b, b->cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
    if (rc != KTAU_OK || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return rc != KTAU_OK ? rc : KTAU_EDEVICE;
    }
    b->graph = g;
    if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
      b->exec = nullptr;
      return KTAU_EDEVICE;
    }
  }
  return hipGraphLaunch(b->exec, s) == hipSuccess ? KTAU_OK : KTAU_EDEVICE;
}

int ktau_batch_status(ktau_batch* b, void* stream) {
  if (!b) return KTAU_EINVAL;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return KTAU_EDEVICE;
  int32_t st = 0;
  if (hipMemcpy(&st, b->words, sizeof(st), hipMemcpyDeviceToHost) != hipSuccess)
    return KTAU_EDEVICE;
  return st;
}

int ktau_batch_plan(const ktau_batch* b, int64_t i, int32_t* scheme, int32_t* q) {
  if (!b || i < 0 || i >= b->count) return KTAU_EINVAL;
  const MatDesc& d = b->host_descs[b->slot[i]];
  if (scheme) *scheme = d.scheme;
  if (q) *q = d.q;
  return KTAU_OK;
}

void ktau_batch_destroy(ktau_batch* b) {
  if (b) free_batch(b);
}

int ktau_autotune(const int64_t* ns, int64_t count, const char* cache_path, void* stream,
                  int32_t* schemes_out, int32_t* q_out) {
  if (!ns || count < 0) return KTAU_EINVAL;
  for (int64_t i = 0; i < count; ++i) {
    if (ns[i] < 2) return KTAU_EINVAL;
    if (ns[i] > KTAU_MAX_N) return KTAU_ERANGE;
  }
  for (int64_t i = 0; i < count; ++i) {
    int rc = KTAU_OK;
    const Plan p = plan_for(ns[i], true, cache_path, (hipStream_t)stream, &rc);
    if (rc != KTAU_OK) return rc;
    if (schemes_out) schemes_out[i] = p.scheme;
    if (q_out) q_out[i] = p.q;
  }
  if (cache_path && *cache_path) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    save_cache(cache_path);
  }
  return KTAU_OK;
}

}  // extern "C"
