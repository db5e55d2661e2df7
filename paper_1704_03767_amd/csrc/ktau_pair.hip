// Pair kernels: exact n_d and n3 for every strict pair of rows (Sec. 3.2
// Steps 1-5, with the per-row halves already done by the rank pre-pass).
//
// For a pair (u, v) the samples are taken in u's sorted order (perm_u) and v
// is replaced by its dense ranks, v'[k] = rank_v[perm_u[k]].  Discordant pairs
// are then the strict inversions of v' (Algorithm 2), except that pairs inside
// one tie run of u must not count.  Three exact ways to meet that:
//   * u has no ties (n1_u == 0): nothing to remove.  Of the two rows the one
//     with the smaller n1 is taken as u (tau is symmetric, Sec. 1);
//   * few u ties: the inversions X and the joint ties n3 inside each u run are
//     counted directly and X is subtracted;
//   * many u ties: Step 1 is done literally -- a merge sort on the composite
//     key (u run, v') orders the samples by (u, v) (its own count is X), the
//     equal composite keys give n3, and a second merge sort on v' alone
//     counts n_d (Step 3).
// The merge sort with counting is the hot loop: a group of G lanes (one wave
// or a 256-lane workgroup) holds the pair's keys, K per lane, in registers.
// Lanes first sort their own K keys (counting inversions among them), then
// log2(G) merge levels run through LDS: each lane finds its output window by
// a merge-path search and merges K outputs serially; every right-run element
// taken adds the number of left-run elements still waiting (Algorithm 2).
#include "ktau_internal.h"

namespace ktau {
namespace {

constexpr int kBlock = 256;      // threads per workgroup for every pair kernel
constexpr int kWavesPerBlock = kBlock / 64;

// ---------------------------------------------------------------- utilities

template <int G>
__device__ inline void group_sync() {
  if constexpr (G == 64) {
    // one wave: LDS operations of a wave complete in order; this only stops
    // the compiler from moving LDS accesses across the point
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

__device__ inline uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// Sum over the group; every lane gets the total.
template <int G>
__device__ inline uint32_t group_sum(uint32_t v, uint32_t* red) {
  v = wave_sum(v);
  if constexpr (G == 64) {
    return v;
  } else {
    const int wave = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[wave] = v;
    __syncthreads();
    uint32_t t = 0;
#pragma unroll
    for (int w = 0; w < G / 64; ++w) t += red[w];
    return t;
  }
}

// ---------------------------------------------------- in-lane sort and count

// Strict inversions among the lane's K keys, then a bitonic sorting network
// leaves them ascending.  All indices are compile-time after unrolling, so
// the keys stay in registers.
template <int K>
__device__ inline uint32_t lane_sort_count(uint32_t (&key)[K]) {
  uint32_t c = 0;
#pragma unroll
  for (int i = 0; i < K; ++i)
#pragma unroll
    for (int j = i + 1; j < K; ++j) c += key[i] > key[j] ? 1u : 0u;
#pragma unroll
  for (int size = 2; size <= K; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
#pragma unroll
      for (int i = 0; i < K; ++i) {
        const int j = i ^ stride;
        if (j > i) {
          const bool up = (i & size) == 0;
          uint32_t a = key[i], b = key[j];
          uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
          key[i] = up ? lo : hi;
          key[j] = up ? hi : lo;
        }
      }
    }
  }
  return c;
}

// ------------------------------------------------------- merge levels (LDS)

// buf holds 2*G*K + 8 keys for this group.  On entry every lane's K keys are
// sorted; on exit the group's G*K keys are sorted (lane-blocked) and the
// return value is this lane's share of the cross-lane inversions.
template <int K, int G>
__device__ inline uint32_t merge_levels(uint32_t (&key)[K], uint32_t* buf, int lane) {
  constexpr int N = G * K;
  uint32_t cnt = 0;
  int cur = 0;
#pragma unroll 1
  for (int s = K; s < N; s <<= 1) {
    uint32_t* b = buf + cur * N;
#pragma unroll
    for (int r = 0; r < K; ++r) b[lane * K + r] = key[r];
    group_sync<G>();
    const int p = lane * K;
    const int l0 = p & ~(2 * s - 1);
    const int diag = p - l0;
    const uint32_t* A = b + l0;
    const uint32_t* B = A + s;
    // merge path: number of A elements among the first `diag` outputs, with
    // A first on equal keys
    int lo = diag > s ? diag - s : 0;
    int hi = diag < s ? diag : s;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (A[mid] <= B[diag - 1 - mid]) lo = mid + 1;
      else hi = mid;
    }
    int ia = lo, ib = diag - lo;
    uint32_t a = ia < s ? A[ia] : kSentinel;
    uint32_t bb = ib < s ? B[ib] : kSentinel;
#pragma unroll
    for (int t = 0; t < K; ++t) {
      const bool takeB = bb < a;   // strict: equal keys are not discordant
      key[t] = takeB ? bb : a;
      if (takeB) {
        cnt += (uint32_t)(s - ia);
        ++ib;
        bb = ib < s ? B[ib] : kSentinel;
      } else {
        ++ia;
        a = ia < s ? A[ia] : kSentinel;
      }
    }
    cur ^= 1;
  }
  return cnt;
}

template <int K, int G>
__device__ inline uint32_t sort_count(uint32_t (&key)[K], uint32_t* buf, int lane, uint32_t* red) {
  uint32_t c = lane_sort_count<K>(key);
  c += merge_levels<K, G>(key, buf, lane);
  return group_sum<G>(c, red);
}

// --------------------------------------------------------------- one pair

struct PairCounts {
  uint32_t nd;
  uint32_t n3;
};

// Exact n_d and n3 of rows (y, x).  Every lane of the group calls this with
// the same arguments; all lanes receive the result.
template <int K, int G>
__device__ inline PairCounts pair_counts(const RankView& rv, int64_t y, int64_t x, int n,
                                         uint32_t* buf, uint32_t* red, int lane) {
  const int64_t n1y = rv.n1[y], n1x = rv.n1[x];
  int64_t u = y, v = x, n1u = n1y;
  if (n1x < n1y) {
    u = x;
    v = y;
    n1u = n1x;
  }
  const uint16_t* pu = rv.perm + u * rv.ld;
  const uint16_t* rk = rv.rank + v * rv.ld;
  const uint16_t* ru = rv.rstart + u * rv.ld;
  const int k0 = lane * K;
  uint32_t key[K];
#pragma unroll
  for (int r = 0; r < K; ++r) {
    const int k = k0 + r;
    key[r] = k < n ? (uint32_t)rk[pu[k]] : kPadKey;
  }
  PairCounts out;
  if (n1u == 0) {
    out.nd = sort_count<K, G>(key, buf, lane, red);
    out.n3 = 0;
    return out;
  }
  // Direct count inside u's tie runs costs sum_k (k - run start) = n1_u
  // comparisons; use it while that is below the cost of a second sort.
  const int64_t direct_budget = (int64_t)4 * n * (32 - __clz(n));
  if (n1u <= direct_budget) {
    // v' in u order goes to merge region 1; the first merge level writes only
    // region 0 and its group sync orders every lane's reads before region 1
    // is written again
    uint32_t* vb = buf + G * K;
#pragma unroll
    for (int r = 0; r < K; ++r) vb[k0 + r] = key[r];
    group_sync<G>();
    uint32_t xin = 0, tie = 0;
#pragma unroll
    for (int r = 0; r < K; ++r) {
      const int k = k0 + r;
      if (k < n) {
        const uint32_t me = key[r];
        for (int j = ru[k]; j < k; ++j) {
          const uint32_t o = vb[j];
          xin += o > me ? 1u : 0u;
          tie += o == me ? 1u : 0u;
        }
      }
    }
    const uint32_t inv = sort_count<K, G>(key, buf, lane, red);
    out.nd = inv - group_sum<G>(xin, red);
    out.n3 = group_sum<G>(tie, red);
    return out;
  }
  // Literal Step 1: sort by (u run, v'), count joint ties, then Step 3.
#pragma unroll
  for (int r = 0; r < K; ++r) {
    const int k = k0 + r;
    if (k < n) key[r] |= (uint32_t)ru[k] << 16;
  }
  (void)sort_count<K, G>(key, buf, lane, red);
  // joint ties: in the (u, v)-sorted sequence, sum over positions of the
  // number of earlier positions holding an equal composite key.  The last
  // merge level (log2 G of them, an even number) read region 1, so region 0
  // is free.
  uint32_t* sb = buf;
#pragma unroll
  for (int r = 0; r < K; ++r) sb[k0 + r] = key[r];
  group_sync<G>();
  uint32_t tie = 0;
#pragma unroll
  for (int r = 0; r < K; ++r) {
    const int k = k0 + r;
    if (k < n) {
      int lo = 0, hi = k;   // first position with a key equal to key[r]
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (sb[mid] < key[r]) lo = mid + 1;
        else hi = mid;
      }
      tie += (uint32_t)(k - lo);
    }
  }
  out.n3 = group_sum<G>(tie, red);
#pragma unroll
  for (int r = 0; r < K; ++r)
    if (key[r] != kPadKey) key[r] &= 0xFFFFu;
  group_sync<G>();
  out.nd = sort_count<K, G>(key, buf, lane, red);
  return out;
}

// Step 5 and Eq. 1/3: store the counts and tau of job slot `slot`.
__device__ inline void store_pair(const PairOut& o, int64_t slot, int64_t n, int64_t n1y,
                                  int64_t n1x, uint32_t nd32, uint32_t n332) {
  const int64_t n0 = n * (n - 1) / 2;
  const int64_t nd = nd32, n3 = n332;
  const int64_t nc = n0 - n1y - n1x + n3 - nd;
  if (o.nc) o.nc[slot] = nc;
  if (o.nd) o.nd[slot] = nd;
  if (o.n3) o.n3[slot] = n3;
  const double num = (double)(nc - nd);
  if (o.tau_b) {
    const double d1 = (double)(n0 - n1y);
    const double d2 = (double)(n0 - n1x);
    const double prod = d1 * d2;
    const double den = sqrt(prod);
    o.tau_b[slot] = den == 0.0 ? __builtin_nan("") : num / den;
  }
  if (o.tau_a) o.tau_a[slot] = num / (double)n0;
}

// LDS per group: two merge regions of G*K keys (plus slack for the
// speculative read one past a run end).
template <int K, int G>
struct GroupLds {
  static constexpr int kWords = 2 * G * K + 16;
};

template <int K, int G>
__device__ inline void do_pair(const RankView& rv, const PairOut& out, int64_t m, int n,
                               int64_t y, int64_t x, int64_t slot, uint32_t* buf,
                               uint32_t* red, int lane) {
  PairCounts c = pair_counts<K, G>(rv, y, x, n, buf, red, lane);
  if (lane == 0) store_pair(out, slot, n, rv.n1[y], rv.n1[x], c.nd, c.n3);
}

// ------------------------------------------------------------------ kernels

// Plain launch, tile order: one q x q tile (Eq. 11-14) per workgroup
// iteration; its pairs go to the waves round-robin (G = 64) or one after
// another to the whole workgroup (G = 256).
template <int K, int G>
__global__ void __launch_bounds__(kBlock)
pairs_tiles_kernel(RankView rv, int64_t m, int n, int q, int64_t w, int64_t tile_begin,
                   int64_t tile_count, PairOut out, const int32_t* __restrict__ status) {
  constexpr int kGroups = kBlock / G;
  constexpr int kWords = GroupLds<K, G>::kWords;
  __shared__ uint32_t lds[kGroups * kWords];
  __shared__ uint32_t red[kWavesPerBlock];
  if (*status != 0) return;
  const int group = threadIdx.x / G;
  const int lane = threadIdx.x % G;
  uint32_t* buf = lds + group * kWords;
  for (int64_t t = blockIdx.x; t < tile_count; t += gridDim.x) {
    int64_t yq, xq;
    tile_coord(w, tile_begin + t, yq, xq);
    for (int p = group; p < q * q; p += kGroups) {
      const int64_t y = yq * q + p / q, x = xq * q + p % q;
      if (y >= x || x >= m) continue;
      do_pair<K, G>(rv, out, m, n, y, x, strict_job(m, y, x), buf, red, lane);
    }
  }
}

// Plain launch, job order: strict job ids [J_begin, J_end), one per group.
template <int K, int G>
__global__ void __launch_bounds__(kBlock)
pairs_jobs_kernel(RankView rv, int64_t m, int n, int64_t J_begin, int64_t J_end, PairOut out,
                  const int32_t* __restrict__ status) {
  constexpr int kGroups = kBlock / G;
  constexpr int kWords = GroupLds<K, G>::kWords;
  __shared__ uint32_t lds[kGroups * kWords];
  __shared__ uint32_t red[kWavesPerBlock];
  if (*status != 0) return;
  const int group = threadIdx.x / G;
  const int lane = threadIdx.x % G;
  uint32_t* buf = lds + group * kWords;
  const int64_t count = J_end - J_begin;
  for (int64_t i = (int64_t)blockIdx.x * kGroups + group; i < count;
       i += (int64_t)gridDim.x * kGroups) {
    int64_t y, x;
    strict_pair(m, J_begin + i, y, x);
    do_pair<K, G>(rv, out, m, n, y, x, i, buf, red, lane);
  }
}

// Persistent launch over the concatenated tile spaces of many matrices.
// Units (tiles) are taken from an atomic counter; a unit is located by binary
// search on the per-matrix unit prefix, then Eq. 13-14 inside its matrix.
template <int K, int G>
__device__ inline void batch_unit(const BatchDesc& d, int64_t t, uint32_t* lds_all,
                                  uint32_t* red) {
  constexpr int kGroups = kBlock / G;
  constexpr int kWords = GroupLds<K, G>::kWords;
  const int group = threadIdx.x / G;
  const int lane = threadIdx.x % G;
  uint32_t* buf = lds_all + group * kWords;
  int64_t yq, xq;
  tile_coord(d.w, t, yq, xq);
  const int q = d.q;
  for (int p = group; p < q * q; p += kGroups) {
    const int64_t y = yq * q + p / q, x = xq * q + p % q;
    if (y >= x || x >= d.m) continue;
    do_pair<K, G>(d.rv, d.out, d.m, d.n, y, x, strict_job(d.m, y, x), buf, red, lane);
  }
}

constexpr int kBatchLdsWords = 2 * 256 * 16 + 16;   // the largest group footprint

__global__ void __launch_bounds__(kBlock)
pairs_batch_kernel(const BatchDesc* __restrict__ descs, int64_t count, int64_t total_units,
                   const int64_t* __restrict__ unit_prefix, int64_t* __restrict__ counter,
                   const int32_t* __restrict__ status) {
  __shared__ uint32_t lds[kBatchLdsWords];
  __shared__ uint32_t red[kWavesPerBlock];
  __shared__ int64_t s_unit;
  if (*status != 0) return;
  for (;;) {
    if (threadIdx.x == 0) s_unit = (int64_t)atomicAdd((unsigned long long*)counter, 1ull);
    __syncthreads();
    const int64_t unit = s_unit;
    __syncthreads();
    if (unit >= total_units) break;
    // matrix b with unit_prefix[b] <= unit < unit_prefix[b + 1]
    int64_t lo = 0, hi = count - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (unit_prefix[mid] <= unit) lo = mid;
      else hi = mid - 1;
    }
    const BatchDesc& d = descs[lo];
    const int64_t t = unit - d.unit_begin;
    switch (d.scheme) {
      case kWaveK2: batch_unit<2, 64>(d, t, lds, red); break;
      case kWaveK4: batch_unit<4, 64>(d, t, lds, red); break;
      case kWaveK8: batch_unit<8, 64>(d, t, lds, red); break;
      case kWaveK16: batch_unit<16, 64>(d, t, lds, red); break;
      case kBlockK4: batch_unit<4, 256>(d, t, lds, red); break;
      case kBlockK8: batch_unit<8, 256>(d, t, lds, red); break;
      default: batch_unit<16, 256>(d, t, lds, red); break;
    }
  }
}

template <int K, int G>
hipError_t launch_tiles_t(const RankView& rv, int64_t m, int n, int q, int64_t w,
                          int64_t tile_begin, int64_t tile_count, const PairOut& out,
                          const int32_t* status, hipStream_t s) {
  int64_t grid = tile_count < (1ll << 30) ? tile_count : (1ll << 30);
  if (grid < 1) return hipSuccess;
  hipLaunchKernelGGL((pairs_tiles_kernel<K, G>), dim3((unsigned)grid), dim3(kBlock), 0, s, rv, m,
                     n, q, w, tile_begin, tile_count, out, status);
  return hipGetLastError();
}

template <int K, int G>
hipError_t launch_jobs_t(const RankView& rv, int64_t m, int n, int64_t J_begin, int64_t J_end,
                         const PairOut& out, const int32_t* status, hipStream_t s) {
  constexpr int kGroups = kBlock / G;
  int64_t count = J_end - J_begin;
  int64_t grid = (count + kGroups - 1) / kGroups;
  if (grid > (1ll << 30)) grid = 1ll << 30;
  if (grid < 1) return hipSuccess;
  hipLaunchKernelGGL((pairs_jobs_kernel<K, G>), dim3((unsigned)grid), dim3(kBlock), 0, s, rv, m, n,
                     J_begin, J_end, out, status);
  return hipGetLastError();
}

}  // namespace

const char* scheme_name(int s) {
  static const char* names[] = {"wave_k2", "wave_k4", "wave_k8", "wave_k16",
                                "block_k4", "block_k8", "block_k16"};
  return (s >= 0 && s < kNumSchemes) ? names[s] : "invalid";
}

int default_scheme(int64_t n) {
  if (n <= 128) return kWaveK2;
  if (n <= 256) return kWaveK4;
  if (n <= 512) return kWaveK8;
  if (n <= 1024) return kWaveK16;
  if (n <= 2048) return kBlockK8;
  return kBlockK16;
}

hipError_t launch_pairs_tiles(int scheme, const RankView& rv, int64_t m, int n, int q, int64_t w,
                              int64_t tile_begin, int64_t tile_count, const PairOut& out,
                              const int32_t* status, hipStream_t s) {
  switch (scheme) {
    case kWaveK2: return launch_tiles_t<2, 64>(rv, m, n, q, w, tile_begin, tile_count, out, status, s);
    case kWaveK4: return launch_tiles_t<4, 64>(rv, m, n, q, w, tile_begin, tile_count, out, status, s);
    case kWaveK8: return launch_tiles_t<8, 64>(rv, m, n, q, w, tile_begin, tile_count, out, status, s);
    case kWaveK16: return launch_tiles_t<16, 64>(rv, m, n, q, w, tile_begin, tile_count, out, status, s);
    case kBlockK4: return launch_tiles_t<4, 256>(rv, m, n, q, w, tile_begin, tile_count, out, status, s);
    case kBlockK8: return launch_tiles_t<8, 256>(rv, m, n, q, w, tile_begin, tile_count, out, status, s);
    case kBlockK16: return launch_tiles_t<16, 256>(rv, m, n, q, w, tile_begin, tile_count, out, status, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_pairs_jobs(int scheme, const RankView& rv, int64_t m, int n, int64_t J_begin,
                             int64_t J_end, const PairOut& out, const int32_t* status,
                             hipStream_t s) {
  switch (scheme) {
    case kWaveK2: return launch_jobs_t<2, 64>(rv, m, n, J_begin, J_end, out, status, s);
    case kWaveK4: return launch_jobs_t<4, 64>(rv, m, n, J_begin, J_end, out, status, s);
    case kWaveK8: return launch_jobs_t<8, 64>(rv, m, n, J_begin, J_end, out, status, s);
    case kWaveK16: return launch_jobs_t<16, 64>(rv, m, n, J_begin, J_end, out, status, s);
    case kBlockK4: return launch_jobs_t<4, 256>(rv, m, n, J_begin, J_end, out, status, s);
    case kBlockK8: return launch_jobs_t<8, 256>(rv, m, n, J_begin, J_end, out, status, s);
    case kBlockK16: return launch_jobs_t<16, 256>(rv, m, n, J_begin, J_end, out, status, s);
    default: return hipErrorInvalidValue;
  }
}

int persistent_grid(int /*max_lanes*/) {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) == hipSuccess) cus = p.multiProcessorCount;
  }
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, pairs_batch_kernel, kBlock, 0) !=
          hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  return cus * per_cu;
}

hipError_t launch_pairs_batch(const BatchDesc* descs_dev, int64_t count, int64_t total_units,
                              const int64_t* unit_prefix_dev, int64_t* counter_dev, int grid,
                              int /*max_lanes*/, const int32_t* status, hipStream_t s) {
  if (total_units < 1) return hipSuccess;
  hipLaunchKernelGGL(pairs_batch_kernel, dim3((unsigned)grid), dim3(kBlock), 0, s, descs_dev,
                     count, total_units, unit_prefix_dev, counter_dev, status);
  return hipGetLastError();
}

}  // namespace ktau
