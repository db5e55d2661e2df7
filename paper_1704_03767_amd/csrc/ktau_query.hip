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

struct TopItem {
  uint64_t key;   // bits(|tau|) + 1, or 0 for NaN / padding
  int32_t idx;    // database row
  int32_t pad;
};

__device__ __forceinline__ bool before(const TopItem& a, const TopItem& b) {
  return a.key > b.key || (a.key == b.key && a.idx < b.idx);
}

// Order key of tau_B: |tau| descending is key descending (the bits of a
// non-negative double order as integers); NaN gets 0, below every number.
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

constexpr int kSelThreads = 1024;
constexpr int kSelWaves = kSelThreads / 64;

// The exact top k of one query row per workgroup (R15: |tau_B| descending,
// then database row ascending; NaN never returned; missing results idx -1,
// tau NaN, nd -1).  A radix select finds the k-th largest key K*, 8 bits a
// pass from the top (a histogram of the keys under the bits decided so far,
// then the digit where the count from the top reaches what is still needed);
// the keys above K* all belong to the top k, and of those equal to K* the
// first in row order fill it up (a scan in row order).  The k chosen items
// are then sorted in LDS and written out.
__global__ void __launch_bounds__(kSelThreads)
topk_select_kernel(const double* __restrict__ tau, const int64_t* __restrict__ nd, int64_t m,
                   int k, int64_t* __restrict__ idx_out, double* __restrict__ tau_out,
                   int64_t* __restrict__ nd_out) {
  __shared__ uint32_t hist[256];
  __shared__ uint32_t wtot[kSelWaves];
  __shared__ TopItem cand[KTAU_MAX_K];
  __shared__ uint64_t s_prefix;
  __shared__ uint32_t s_need, s_gt, s_count;
  const int64_t qi = blockIdx.x;
  const double* t = tau + qi * m;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  uint64_t prefix = 0;          // the bits of K* decided so far
  uint32_t need = (uint32_t)k;  // keys under that prefix still to take
  uint32_t gt = 0;              // keys above the prefix's range (all taken)
  for (int shift = 56; shift >= 0; shift -= 8) {
    for (int i = tid; i < 256; i += kSelThreads) hist[i] = 0;
    __syncthreads();
    for (int64_t j = tid; j < m; j += kSelThreads) {
      const uint64_t key = tau_key(t[j]);
      if (shift == 56 || (key >> (shift + 8)) == (prefix >> (shift + 8)))
        atomicAdd(&hist[(uint32_t)(key >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (wave == 0) {
      // lane l holds bins 255 - 4l .. 252 - 4l; counts from the top down
      const int d0 = 255 - 4 * lane;
      uint32_t h[4], sum = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        h[q] = hist[d0 - q];
        sum += h[q];
      }
      uint32_t incl = sum;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = __shfl_up(incl, d, 64);
        if (lane >= d) incl += o;
      }
      const uint32_t excl = incl - sum;
      const uint64_t hit = __ballot(excl < need && incl >= need);
      // the lane holding the digit; if all the keys under the prefix are
      // fewer than needed, all of them are taken (digit 0, lowest bins)
      const int src = hit ? __ffsll((unsigned long long)hit) - 1 : 63;
      if (lane == src) {
        uint32_t cum = excl;
        int digit = 0;
        if (hit) {
          digit = d0 - 3;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            if (cum + h[q] >= need) {
              digit = d0 - q;
              break;
            }
            cum += h[q];
          }
        } else {
          cum = incl - h[3];
        }
        s_prefix = prefix | ((uint64_t)digit << shift);
        s_need = need - cum;
        s_gt = gt + cum;
      }
    }
    __syncthreads();
    prefix = s_prefix;
    need = s_need;
    gt = s_gt;
  }
  const uint64_t kstar = prefix;
  // keys above K*, in any order
  if (tid == 0) s_count = 0;
  __syncthreads();
  for (int64_t j = tid; j < m; j += kSelThreads) {
    const uint64_t key = tau_key(t[j]);
    if (key > kstar) {
      const uint32_t at = atomicAdd(&s_count, 1u);
      cand[at] = TopItem{key, (int32_t)j, 0};
    }
  }
  // keys equal to K* (never NaN), the first `take` in row order
  const uint32_t take = kstar == 0 ? 0u : need;
  uint32_t run = 0;
  for (int64_t j0 = 0; j0 < m && run < take; j0 += kSelThreads) {
    const int64_t j = j0 + tid;
    const bool eq = j < m && tau_key(t[j]) == kstar;
    const uint64_t mask = __ballot(eq);
    const uint32_t below = (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
    if (lane == 0) wtot[wave] = (uint32_t)__popcll(mask);
    __syncthreads();
    uint32_t ahead = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kSelWaves; ++w) {
      const uint32_t c = wtot[w];
      ahead += w < wave ? c : 0u;
      all += c;
    }
    const uint32_t at = run + ahead + below;
    if (eq && at < take) cand[gt + at] = TopItem{kstar, (int32_t)j, 0};
    run += all;
    __syncthreads();
  }
  const uint32_t filled = gt + (run < take ? run : take);
  int k2 = 1;
  while (k2 < k) k2 <<= 1;
  for (int i = tid; i < k2; i += kSelThreads)
    if ((uint32_t)i >= filled) cand[i] = TopItem{0, 0x7FFFFFFF, 0};
  __syncthreads();
  for (int size = 2; size <= k2; size <<= 1)
    bitonic_stages(cand, k2, size >> 1, size < k2 ? size : 0);
  for (int i = tid; i < k; i += kSelThreads) {
    const TopItem c = cand[i];
    const bool ok = c.key != 0;
    const int64_t o = qi * k + i;
    if (idx_out) idx_out[o] = ok ? (int64_t)c.idx : -1;
    if (tau_out) tau_out[o] = ok ? t[c.idx] : __builtin_nan("");
    if (nd_out) nd_out[o] = ok ? nd[qi * m + c.idx] : -1;
  }
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

size_t query_scratch_bytes(int64_t nq, int64_t m, int64_t n, int k, bool naive) {
  (void)k;
  size_t b = ws_layout(nq, n).total;
  if (naive) b = (size_t)round_up((int64_t)(b + bits_bytes(nq, n)), (int64_t)kAlign);
  b += (size_t)round_up(nq * m * 8, (int64_t)kAlign);            // tau
  b += (size_t)round_up(nq * m * 8, (int64_t)kAlign);            // nd
  return b;
}

int launch_query(const DbView& db, const float* Q, int64_t nq, int k, void* scratch,
                 int64_t* idx_out, double* tau_out, int64_t* nd_out, int32_t* status,
                 hipStream_t s) {
  if (nq == 0) return KTAU_OK;
  const int64_t m = db.m, n = db.n;
  char* base = (char*)scratch;
  const bool naive = db.scheme == KTAU_SCHEME_NAIVE;
  size_t off = ws_layout(nq, n).total;
  uint32_t* qbits = (uint32_t*)(base + off);
  if (naive) off = (size_t)round_up((int64_t)(off + bits_bytes(nq, n)), (int64_t)kAlign);
  double* tau = (double*)(base + off);
  off += (size_t)round_up(nq * m * 8, (int64_t)kAlign);
  int64_t* nd = (int64_t*)(base + off);

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

  // exact top-k, one workgroup per query row
  hipLaunchKernelGGL(topk_select_kernel, dim3((unsigned)nq), dim3(kSelThreads), 0, s, tau, nd, m,
                     k, idx_out, tau_out, nd_out);
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
