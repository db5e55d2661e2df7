// Query-vs-database search (Sec. 1: rank the subject rows of a database by
// their score against a query row): tau_B of every query row against every
// resident, pre-ranked database row, then the k database rows of largest
// |tau_B| per query.
//
// The database is ranked once (ktau_db_create) and stays in HBM.  A query
// call ranks its nq rows, runs one wave per (query, database row) pair with
// the same per-pair routine as all-pairs, a composite pass for pairs whose two
// rows are both heavily tied, and an exact top-k: chunks of 4096 candidates
// are bitonic-sorted in LDS by (|tau| descending, row ascending) and cut to k,
// repeatedly, until k remain.
#include <stdlib.h>
#include <string.h>

#include "ktau_pairdev.h"
#include "ktau_query.h"

namespace ktau {
namespace {

// ------------------------------------------------------------ pair kernels

template <int K, int G>
__global__ void __launch_bounds__(kBlock, (fast_waves<K, G>())) query_pairs_kernel(QueryDesc qd) {
  using FL = FastLds<K, G>;
  constexpr int kGroups = FL::kGroups;
  __shared__ uint32_t lds[FL::kBlockWords];
  uint32_t* red = FL::red(lds);
  if (*qd.status != 0) return;
  const int group = threadIdx.x / G;
  const int lane = threadIdx.x % G;
  uint32_t* buf = lds + group * FastLds<K, G>::kWords;
  const int64_t jobs = qd.nq * qd.m;
  const int64_t budget = direct_budget(qd.n);
  Deferred<G> done;
  auto store = [&](int64_t slot, int64_t a, int64_t b, uint32_t d, uint32_t t) {
    store_cross(qd, slot, a, b, d, t);
  };
  for (int64_t i = (int64_t)blockIdx.x * kGroups + group; i < jobs;
       i += (int64_t)gridDim.x * kGroups) {
    const int64_t qi = i / qd.m, j = i - qi * qd.m;
    uint32_t nd, n3;
    if (!pair_fast<K, G>(qd.rq, qi, qd.rdb, j, qd.n, budget, buf, red, lane, nd, n3)) continue;
    done.add(lane, i, qd.rq.n1[qi], qd.rdb.n1[j], nd, n3);
    if (done.full()) done.flush_with(lane, store);
  }
  done.flush_with(lane, store);
}

// Pairs of a heavy query row and a heavy database row.
template <int K, int G>
__global__ void __launch_bounds__(kBlock) query_composite_kernel(QueryDesc qd) {
  constexpr int kGroups = kBlock / G;
  __shared__ uint32_t lds[kGroups * CompLds<K, G>::kWords];
  __shared__ uint32_t red[kWavesPerBlock];
  if (*qd.status != 0) return;
  const int64_t hq = *qd.q_heavy_count, hd = *qd.db_heavy_count;
  const int group = threadIdx.x / G;
  const int lane = threadIdx.x % G;
  uint32_t* buf = lds + group * CompLds<K, G>::kWords;
  for (int64_t i = (int64_t)blockIdx.x * kGroups + group; i < hq * hd;
       i += (int64_t)gridDim.x * kGroups) {
    const int64_t qi = qd.q_heavy[i / hd], j = qd.db_heavy[i % hd];
    uint32_t nd, n3;
    pair_composite<K, G>(qd.rq, qi, qd.rdb, j, qd.n, buf, red, lane, nd, n3);
    if (lane == 0) store_cross(qd, qi * qd.m + j, qd.rq.n1[qi], qd.rdb.n1[j], nd, n3);
  }
}

// ------------------------------------------------------------------ top-k

constexpr int kChunk = 4096;   // candidates sorted per workgroup

struct TopItem {
  uint64_t key;   // bits(|tau|) + 1, or 0 for NaN / padding
  int32_t idx;    // database row
  int32_t pad;
};

__device__ __forceinline__ bool before(const TopItem& a, const TopItem& b) {
  return a.key > b.key || (a.key == b.key && a.idx < b.idx);
}

__device__ __forceinline__ uint64_t tau_key(double t) {
  if (t != t) return 0;
  return (uint64_t)__double_as_longlong(fabs(t)) + 1;
}

// Compare-exchange stages of width `stride` down to 1 over the first `cnt`
// items: the pair (i, i ^ stride) is put in `before` order, reversed where
// bit `dir` of i is set (dir = 0: never).
__device__ void bitonic_stages(TopItem* s, int cnt, int stride, int dir) {
  for (; stride > 0; stride >>= 1) {
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
      const int j = i ^ stride;
      if (j > i) {
        const bool up = dir == 0 || (i & dir) == 0;
        const TopItem a = s[i], b = s[j];
        if (up ? before(b, a) : before(a, b)) {
          s[i] = b;
          s[j] = a;
        }
      }
    }
    __syncthreads();
  }
}

// The k2 best of `cnt` items of LDS (both powers of two, k2 <= cnt), in
// `before` order, in s[0 .. k2): every block of k2 items is sorted, then
// blocks are merged pairwise keeping the better half -- the better of A[i]
// and B[k2 - 1 - i] over i is the k2 best of A and B, as a bitonic sequence
// that log2(k2) more stages sort -- until one block is left.
__device__ void topk_items(TopItem* s, int cnt, int k2) {
  for (int size = 2; size <= k2; size <<= 1) bitonic_stages(s, cnt, size >> 1, size < k2 ? size : 0);
  for (int step = k2; step < cnt; step <<= 1) {
    // blocks at multiples of step: block b keeps the best of b and b + step
    for (int i = threadIdx.x; i < cnt / 2; i += blockDim.x) {
      const int b = (i / k2) * 2 * step, t = i % k2;
      if (b + step < cnt) {
        const TopItem a = s[b + t], c = s[b + step + k2 - 1 - t];
        if (before(c, a)) s[b + t] = c;
      }
    }
    __syncthreads();
    for (int stride = k2 >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < cnt / 2; i += blockDim.x) {
        const int b = (i / k2) * 2 * step, t = i % k2;
        const int j = t ^ stride;
        if (b < cnt && j > t) {
          const TopItem a = s[b + t], c = s[b + j];
          if (before(c, a)) {
            s[b + t] = c;
            s[b + j] = a;
          }
        }
      }
      __syncthreads();
    }
  }
}

// One round: every query's list of `len` items (or of tau values when
// `from_tau`) is cut, chunk by chunk, to its k best; output lists have
// ceil(len / kChunk) * k items.
__global__ void __launch_bounds__(256)
topk_round_kernel(const double* __restrict__ tau, const TopItem* __restrict__ in,
                  int64_t len, int k, TopItem* __restrict__ out, int64_t out_len) {
  extern __shared__ TopItem s_items[];
  const int64_t qi = blockIdx.y;
  const int64_t c0 = (int64_t)blockIdx.x * kChunk;
  const int64_t cnt_real = len - c0 < kChunk ? len - c0 : kChunk;
  int cnt = 1;
  while (cnt < cnt_real) cnt <<= 1;
  if (cnt < k) {
    int c = cnt;
    while (c < k) c <<= 1;
    cnt = c;
  }
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
    TopItem t;
    t.key = 0;
    t.idx = 0x7FFFFFFF;
    t.pad = 0;
    if (i < cnt_real) {
      const int64_t g = c0 + i;
      if (tau) {
        t.key = tau_key(tau[qi * len + g]);
        t.idx = (int32_t)g;
      } else {
        t = in[qi * len + g];
      }
    }
    s_items[i] = t;
  }
  __syncthreads();
  int k2 = 1;
  while (k2 < k) k2 <<= 1;
  topk_items(s_items, cnt, k2);
  for (int i = threadIdx.x; i < k; i += blockDim.x)
    out[qi * out_len + (int64_t)blockIdx.x * k + i] = s_items[i];
}

// Final k items of each query -> caller arrays (idx -1, tau NaN, nd -1 for
// missing results).
__global__ void topk_write_kernel(const TopItem* __restrict__ items, int64_t nq, int k,
                                  const double* __restrict__ tau, const int64_t* __restrict__ nd,
                                  int64_t m, int64_t* __restrict__ idx_out,
                                  double* __restrict__ tau_out, int64_t* __restrict__ nd_out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nq * k) return;
  const int64_t qi = i / k;
  const TopItem t = items[i];
  const bool ok = t.key != 0;
  const int64_t j = t.idx;
  if (idx_out) idx_out[i] = ok ? j : -1;
  if (tau_out) tau_out[i] = ok ? tau[qi * m + j] : __builtin_nan("");
  if (nd_out) nd_out[i] = ok ? nd[qi * m + j] : -1;
}

template <int K, int G>
hipError_t query_pairs_t(const QueryDesc& qd, hipStream_t s) {
  constexpr int kGroups = kBlock / G;
  const int64_t jobs = qd.nq * qd.m;
  // enough workgroups to fill the device several times over, each group
  // then finishing many pairs (their tau stores go out together)
  int64_t grid = (jobs + kGroups - 1) / kGroups;
  if (grid > kMaxPairGrid) grid = kMaxPairGrid;
  if (grid < 1) return hipSuccess;
  hipLaunchKernelGGL((query_pairs_kernel<K, G>), dim3((unsigned)grid), dim3(kBlock), 0, s, qd);
  return hipGetLastError();
}

// Heavy x heavy pairs, on whole waves or 256-lane blocks chosen by n.
hipError_t query_composite(const QueryDesc& qd, hipStream_t s) {
  if (qd.n > kCompositeMaxN) return hipSuccess;   // no heavy rows there
#define KTAU_COMP(K, G) \
  hipLaunchKernelGGL((query_composite_kernel<K, G>), dim3(256), dim3(kBlock), 0, s, qd)
  if (qd.n <= 128) KTAU_COMP(2, 64);
  else if (qd.n <= 256) KTAU_COMP(4, 64);
  else if (qd.n <= 512) KTAU_COMP(8, 64);
  else if (qd.n <= 1024) KTAU_COMP(16, 64);
  else if (qd.n <= 2048) KTAU_COMP(8, 256);
  else if (qd.n <= 4096) KTAU_COMP(16, 256);
  else if (qd.n <= 8192) KTAU_COMP(32, 256);
  else KTAU_COMP(64, 256);
#undef KTAU_COMP
  return hipGetLastError();
}

}  // namespace

// The pair scheme of queries against a database of n samples: the naive
// bit-set count up to 128 samples (measured faster there, as on the plain
// path), else the fastest network scheme.
int query_default_scheme(int64_t n) { return n <= 128 ? KTAU_SCHEME_NAIVE : network_scheme(n); }

int64_t topk_rounds_len(int64_t len, int k, int64_t* out_len) {
  // returns the number of rounds; out_len receives the longest list written
  int64_t rounds = 0, cur = len, longest = 0;
  do {
    const int64_t chunks = (cur + kChunk - 1) / kChunk;
    cur = chunks * k;
    longest = cur > longest ? cur : longest;
    ++rounds;
  } while (cur > k);
  if (out_len) *out_len = longest;
  return rounds;
}

size_t query_scratch_bytes(int64_t nq, int64_t m, int64_t n, int k, bool naive) {
  int64_t longest = 0;
  topk_rounds_len(m, k, &longest);
  size_t b = ws_layout(nq, n).total;
  if (naive) b = (size_t)round_up((int64_t)(b + bits_bytes(nq, n)), (int64_t)kAlign);
  b += (size_t)round_up(nq * m * 8, (int64_t)kAlign);            // tau
  b += (size_t)round_up(nq * m * 8, (int64_t)kAlign);            // nd
  b += 2 * (size_t)round_up(nq * longest * (int64_t)sizeof(TopItem), (int64_t)kAlign);
  return b;
}

int launch_query(const DbView& db, const float* Q, int64_t nq, int k, void* scratch,
                 int64_t* idx_out, double* tau_out, int64_t* nd_out, int32_t* status,
                 hipStream_t s) {
  if (nq == 0) return KTAU_OK;
  const int64_t m = db.m, n = db.n;
  int64_t longest = 0;
  topk_rounds_len(m, k, &longest);
  char* base = (char*)scratch;
  const bool naive = db.scheme == KTAU_SCHEME_NAIVE;
  size_t off = ws_layout(nq, n).total;
  uint32_t* qbits = (uint32_t*)(base + off);
  if (naive) off = (size_t)round_up((int64_t)(off + bits_bytes(nq, n)), (int64_t)kAlign);
  double* tau = (double*)(base + off);
  off += (size_t)round_up(nq * m * 8, (int64_t)kAlign);
  int64_t* nd = (int64_t*)(base + off);
  off += (size_t)round_up(nq * m * 8, (int64_t)kAlign);
  TopItem* ia = (TopItem*)(base + off);
  off += (size_t)round_up(nq * longest * (int64_t)sizeof(TopItem), (int64_t)kAlign);
  TopItem* ib = (TopItem*)(base + off);

  // rank the query rows into the scratch head (its status word is unused:
  // the caller's status word collects NaN reports)
  ktau_pair_out none{};
  MatDesc qdesc = matdesc(scratch, nq, n, none, db.scheme, 8, 0, 0, status);
  if (clear_words((int32_t*)scratch, 2, s) != KTAU_OK) return KTAU_EDEVICE;
  if (prepass_ws(Q, nq, n, scratch, nullptr, status, s) != KTAU_OK) return KTAU_EDEVICE;
  // (the bit sets count tied pairs exactly: no composite pass)
  const bool composite = !naive && db.heavy_rows != 0 && n <= kCompositeMaxN;
  if (naive && launch_bits_prepass(qdesc, qbits, s) != hipSuccess) return KTAU_EDEVICE;
  if (composite && launch_heavy(qdesc, s) != hipSuccess) return KTAU_EDEVICE;

  QueryDesc qd;
  memset(&qd, 0, sizeof(qd));
  qd.rq = qdesc.rv;
  qd.rdb = db.rv;
  qd.nq = nq;
  qd.m = m;
  qd.n = (int32_t)n;
  qd.tau = tau;
  qd.nd = nd;
  qd.status = status;
  qd.q_heavy = qdesc.heavy;
  qd.q_heavy_count = qdesc.heavy_count;
  qd.db_heavy = db.heavy;
  qd.db_heavy_count = db.heavy_count;
  hipError_t e;
  switch (db.scheme) {
#define KTAU_CASE(S, K, G) \
  case S: e = query_pairs_t<K, G>(qd, s); break;
    KTAU_FOR_EACH_SCHEME(KTAU_CASE)
#undef KTAU_CASE
    case KTAU_SCHEME_NAIVE: e = launch_bits_query(qd, qbits, db.bits, s); break;
    default: e = hipErrorInvalidValue; break;
  }
  if (e == hipSuccess && composite) e = query_composite(qd, s);
  if (e != hipSuccess) return KTAU_EDEVICE;

  // top-k rounds: tau -> ia -> ib -> ia ...
  int64_t len = m;
  const TopItem* src = nullptr;
  TopItem* dst = ia;
  bool first = true;
  for (;;) {
    const int64_t chunks = (len + kChunk - 1) / kChunk;
    const int64_t out_len = chunks * k;
    int cnt = 1;
    while (cnt < (len < kChunk ? len : kChunk)) cnt <<= 1;
    while (cnt < k) cnt <<= 1;
    hipLaunchKernelGGL(topk_round_kernel, dim3((unsigned)chunks, (unsigned)nq), dim3(256),
                       (size_t)cnt * sizeof(TopItem), s, first ? tau : nullptr, src, len, k, dst,
                       out_len);
    if (hipGetLastError() != hipSuccess) return KTAU_EDEVICE;
    first = false;
    len = out_len;
    if (len <= k) break;
    src = dst;
    dst = dst == ia ? ib : ia;
  }
  const int64_t total = nq * k;
  hipLaunchKernelGGL(topk_write_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                     dst, nq, k, tau, nd, m, idx_out, tau_out, nd_out);
  return hipGetLastError() == hipSuccess ? KTAU_OK : KTAU_EDEVICE;
}

}  // namespace ktau

using namespace ktau;

extern "C" {

int ktau_db_create_ex(const float* X, int64_t m, int64_t n, int scheme, void* stream,
                      ktau_db** out) {
  if (!out || !X) return KTAU_EINVAL;
  *out = nullptr;
  if (m < 1 || n < 2 || m > (int64_t)0x7fffffff) return KTAU_EINVAL;
  if (n > KTAU_MAX_N_NETWORK) return KTAU_ERANGE;
  if (scheme == KTAU_SCHEME_NAIVE) {
    if (n > kBitsMaxN) return KTAU_EINVAL;
  } else if (scheme >= 0 && (scheme >= kNumNetSchemes || scheme_capacity(scheme) < n)) {
    return KTAU_EINVAL;
  }
  const hipStream_t s = (hipStream_t)stream;
  ktau_db* db = new ktau_db();
  db->v.m = m;
  db->v.n = n;
  db->v.scheme = scheme >= 0 ? scheme : query_default_scheme(n);
  const bool naive = db->v.scheme == KTAU_SCHEME_NAIVE;
  const WsLayout L = ws_layout(m, n);
  if (hipMalloc(&db->ws, L.total + (naive ? bits_bytes(m, n) : 0)) != hipSuccess) {
    delete db;
    return KTAU_ENOMEM;
  }
  ktau_pair_out none{};
  MatDesc d = matdesc(db->ws, m, n, none, db->v.scheme, 8, 0, 0, nullptr);
  db->v.rv = d.rv;
  db->v.heavy = d.heavy;
  db->v.heavy_count = d.heavy_count;
  if (naive) db->v.bits = (uint32_t*)((char*)db->ws + L.total);
  int rc = KTAU_OK;
  if (clear_words((int32_t*)db->ws, 2, s) != KTAU_OK ||
      prepass_ws(X, m, n, db->ws, nullptr, nullptr, s) != KTAU_OK ||
      launch_heavy(d, s) != hipSuccess ||
      (naive && launch_bits_prepass(d, db->v.bits, s) != hipSuccess))
    rc = KTAU_EDEVICE;
  if (rc == KTAU_OK) {
    rc = ktau_status(db->ws, stream);
  }
  // the number of heavy database rows: without any, no query pair can need
  // the composite pass and queries skip it
  if (rc == KTAU_OK &&
      hipMemcpy(&db->v.heavy_rows, db->v.heavy_count, sizeof(int32_t), hipMemcpyDeviceToHost) !=
          hipSuccess)
    rc = KTAU_EDEVICE;
  if (rc != KTAU_OK) {
    (void)hipFree(db->ws);
    delete db;
    return rc;
  }
  *out = db;
  return KTAU_OK;
}

int ktau_db_create(const float* X, int64_t m, int64_t n, void* stream, ktau_db** out) {
  return ktau_db_create_ex(X, m, n, -1, stream, out);
}

void ktau_db_destroy(ktau_db* db) {
  if (!db) return;
  if (db->ws) (void)hipFree(db->ws);
  delete db;
}

int64_t ktau_db_rows(const ktau_db* db) { return db ? db->v.m : -1; }
int64_t ktau_db_samples(const ktau_db* db) { return db ? db->v.n : -1; }

size_t ktau_query_workspace_size(const ktau_db* db, int64_t nq, int64_t k) {
  if (!db || nq < 0 || k < 1 || k > KTAU_MAX_K) return 0;
  return kWsHeader + query_scratch_bytes(nq > 0 ? nq : 1, db->v.m, db->v.n, (int)k,
                                        db->v.scheme == KTAU_SCHEME_NAIVE);
}

int ktau_query(const ktau_db* db, const float* Q, int64_t nq, int64_t k, int64_t* idx_out,
               double* tau_out, int64_t* nd_out, void* ws, size_t ws_bytes, void* stream) {
  if (!db || (!Q && nq > 0) || nq < 0 || !idx_out || !ws) return KTAU_EINVAL;
  if (k < 1 || k > KTAU_MAX_K) return KTAU_ERANGE;
  if (((uintptr_t)ws) % kAlign != 0) return KTAU_EINVAL;
  if (ws_bytes < ktau_query_workspace_size(db, nq, k)) return KTAU_ENOMEM;
  const hipStream_t s = (hipStream_t)stream;
  int32_t* status = (int32_t*)ws;
  if (clear_words(status, 2, s) != KTAU_OK) return KTAU_EDEVICE;
  return launch_query(db->v, Q, nq, (int)k, (char*)ws + kWsHeader, idx_out, tau_out, nd_out,
                      status, s);
}

}  // extern "C"
