// Pair kernels: exact n_d and n3 for every strict pair of rows (Sec. 3.2
// Steps 1-5, with the per-row halves already done by the rank pre-pass).
//
// For a pair (u, v) the samples are taken in u's sorted order (perm_u) and v
// is replaced by its dense ranks, v'[k] = rank_v[perm_u[k]].  Discordant pairs
// are then the strict inversions of v' (Algorithm 2), except that pairs inside
// one tie run of u must not count.  Of the two rows the one with the smaller
// tie term n1 is taken as u (tau is symmetric, Sec. 1).  Then:
//   * u has no ties: n_d is the inversion count of v';
//   * u has ties, n1_u within a budget of about 4 n log2 n comparisons: the
//     inversions X and the joint ties n3 inside each u run are counted
//     directly (each position against the earlier positions of its run) and
//     n_d = inversions(v') - X;
//   * both rows have more ties than that: the pair is left to a second pass
//     (composite kernel) that does Step 1 literally -- a merge sort on the
//     composite key (u run, v') orders the samples by (u, v), equal composite
//     keys give n3, and a second merge sort on v' alone counts n_d (Step 3).
// The inversion count of the first two cases is the register-resident tagged
// bitonic network of ktau_bitonic.h.  The composite pass uses an LDS merge
// path with 32-bit keys.  Keeping it in its own kernel keeps the register
// budget of the main kernels small.
#include "ktau_order.h"
#include "ktau_pairdev.h"

namespace ktau {
namespace {

// One q x q tile (Eq. 11-14) of a matrix, tile coordinates (yq, xq); its
// pairs go round-robin to the `workers` groups that run it, this thread's
// group being number `worker` among them.
template <int K, int G>
__device__ __forceinline__ void tile_pairs(const MatDesc& d, int64_t yq, int64_t xq,
                                           uint32_t* lds_all, uint32_t* red, int worker,
                                           int workers) {
  const int group = threadIdx.x / G;
  const int lane = threadIdx.x % G;
  uint32_t* lds = lds_all + group * FastLds<K, G>::kWords;
  const int q = d.q;
  const int64_t budget = direct_budget(d.n);
  Deferred<G> done;
  // pair p of the tile is (row p / q, column p % q); (py, px) follow p
  int py = worker / q, px = worker % q;
  const int step_y = workers / q, step_x = workers % q;
  auto next = [&]() {
    py += step_y;
    px += step_x;
    if (px >= q) {
      px -= q;
      ++py;
    }
  };
  for (int p = worker; p < q * q; p += workers, next()) {
    const int64_t y = yq * q + py, x = xq * q + px;
    if (y >= x || x >= d.m) continue;
    uint32_t nd, n3;
    if (!pair_fast<K, G>(d.rv, y, d.rv, x, d.n, budget, lds, red, lane, nd, n3)) continue;
    done.add(lane, strict_job(d.m, y, x), d.rv.n1[y], d.rv.n1[x], nd, n3);
    if (done.full()) done.flush(lane, d.out, d.n);
  }
  done.flush(lane, d.out, d.n);
}

// Plain launch over the tiles.  With one workgroup per tile the tiles follow
// the XCD-aware band schedule (input rows reused from L2); otherwise a grid
// stride over the tile ids.  (A single call site of the pair routine halves
// the code but measured about 1% slower.)
template <int K, int G>
__global__ void __launch_bounds__(kBlock, (fast_waves<K, G>())) pairs_tiles_kernel(MatDesc d) {
  using FL = FastLds<K, G>;
  __shared__ uint32_t lds[FL::kBlockWords];
  uint32_t* red = FL::red(lds);
  if (*d.status != 0) return;
  const int group = threadIdx.x / G;
  int64_t yq, xq;
  if ((int64_t)gridDim.x == d.n_units) {
    scheduled_tile(d.w, d.n_units, blockIdx.x, yq, xq);
    tile_pairs<K, G>(d, yq, xq, lds, red, group, FL::kGroups);
    return;
  }
  for (int64_t t = blockIdx.x; t < d.n_units; t += gridDim.x) {
    tile_coord(d.w, t, yq, xq);
    tile_pairs<K, G>(d, yq, xq, lds, red, group, FL::kGroups);
  }
}

// Plain launch, job order: strict job ids [J_begin, J_end), one per group.
template <int K, int G>
__global__ void __launch_bounds__(kBlock, (fast_waves<K, G>())) pairs_jobs_kernel(MatDesc d) {
  using FL = FastLds<K, G>;
  constexpr int kGroups = FL::kGroups;
  __shared__ uint32_t lds[FL::kBlockWords];
  uint32_t* red = FL::red(lds);
  if (*d.status != 0) return;
  const int group = threadIdx.x / G;
  const int lane = threadIdx.x % G;
  uint32_t* buf = lds + group * FastLds<K, G>::kWords;
  const int64_t count = d.J_end - d.J_begin;
  const int64_t budget = direct_budget(d.n);
  Deferred<G> done;
  for (int64_t i = (int64_t)blockIdx.x * kGroups + group; i < count;
       i += (int64_t)gridDim.x * kGroups) {
    int64_t y, x;
    strict_pair(d.m, d.J_begin + i, y, x);
    uint32_t nd, n3;
    if (!pair_fast<K, G>(d.rv, y, d.rv, x, d.n, budget, buf, red, lane, nd, n3)) continue;
    done.add(lane, i, d.rv.n1[y], d.rv.n1[x], nd, n3);
    if (done.full()) done.flush(lane, d.out, d.n);
  }
  done.flush(lane, d.out, d.n);
}

// Persistent launch over the concatenated tile spaces of the matrices of one
// scheme class.  The unit (tile) space is cut into kXcds contiguous
// stretches; workgroup b starts on stretch b mod kXcds (the XCD it runs on),
// taking units from that stretch's atomic counter, so each XCD works
// through consecutive units; a worker whose stretch is used up moves on to
// the following stretches, which keeps the load balanced when workgroups
// start late (other kernels of the batch hold the CUs).  With groups of up to
// 64 lanes every wave is a
// worker of its own (no workgroup-wide hand-off of units); 256-lane groups
// take units per workgroup.  A unit is located by binary search on the
// per-matrix unit prefix, and inside its matrix the units follow the band
// order (input rows reused from the XCD's L2).
template <int K, int G>
__global__ void __launch_bounds__(kBlock, (fast_waves<K, G>()))
pairs_persistent_kernel(const MatDesc* __restrict__ descs, int64_t count, int64_t total_units,
                        const int64_t* __restrict__ unit_prefix, int64_t* __restrict__ counters,
                        const int32_t* __restrict__ status) {
  using FL = FastLds<K, G>;
  __shared__ uint32_t lds[FL::kBlockWords];
  uint32_t* red = FL::red(lds);
  if (*status != 0) return;
  const int64_t per = total_units / kXcds, rem = total_units % kXcds;
  constexpr bool kWaveWorkers = G <= 64;
  const int worker = kWaveWorkers ? (int)(threadIdx.x & 63) / G : 0;
  const int workers = kWaveWorkers ? 64 / G : 1;
  int64_t x = blockIdx.x % kXcds;
  int64_t first = x * per + (x < rem ? x : rem);
  int64_t len = per + (x < rem ? 1 : 0);
  for (int visited = 0;;) {
    int64_t k;
    if constexpr (kWaveWorkers) {
      // lane 0 of the wave takes the unit; every lane reads it from lane 0
      uint64_t got = 0;
      if ((threadIdx.x & 63) == 0) got = atomicAdd((unsigned long long*)(counters + x), 1ull);
      const uint32_t lo32 = __builtin_amdgcn_readfirstlane((uint32_t)got);
      const uint32_t hi32 = __builtin_amdgcn_readfirstlane((uint32_t)(got >> 32));
      k = (int64_t)(((uint64_t)hi32 << 32) | lo32);
    } else {
      int64_t* slot = FL::unit(lds);
      if (threadIdx.x == 0) *slot = (int64_t)atomicAdd((unsigned long long*)(counters + x), 1ull);
      __syncthreads();
      k = *slot;
      __syncthreads();
    }
    if (k >= len) {
      if (++visited == kXcds) break;
      x = (x + 1) % kXcds;
      first = x * per + (x < rem ? x : rem);
      len = per + (x < rem ? 1 : 0);
      continue;
    }
    const int64_t unit = first + k;
    // matrix b with unit_prefix[b] <= unit < unit_prefix[b + 1]
    int64_t lo = 0, hi = count - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (unit_prefix[mid] <= unit) lo = mid;
      else hi = mid - 1;
    }
    int64_t yq, xq;
    band_tile(descs[lo].w, unit - unit_prefix[lo], yq, xq);
    tile_pairs<K, G>(descs[lo], yq, xq, lds, red, worker, workers);
  }
}

// ================================================== heavy-tie row lists

// One workgroup per matrix: the ascending list of rows whose tie term exceeds
// the direct budget, and its length.
__device__ void heavy_rows(const MatDesc& d) {
  __shared__ int s_base;
  __shared__ int s_wave[kWavesPerBlock];
  const int64_t budget = direct_budget(d.n);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x == 0) s_base = 0;
  __syncthreads();
  for (int64_t r0 = 0; r0 < d.m; r0 += kBlock) {
    const int64_t r = r0 + threadIdx.x;
    const bool h = r < d.m && d.rv.n1[r] > budget;
    const uint64_t mask = __ballot(h);
    const int before = __popcll(mask & ((1ull << lane) - 1ull));
    if (lane == 0) s_wave[wave] = __popcll(mask);
    __syncthreads();
    int off = s_base;
    for (int w = 0; w < wave; ++w) off += s_wave[w];
    if (h) d.heavy[off + before] = (int32_t)r;
    __syncthreads();
    if (threadIdx.x == 0)
      for (int w = 0; w < kWavesPerBlock; ++w) s_base += s_wave[w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *d.heavy_count = s_base;
}

__global__ void __launch_bounds__(kBlock) heavy_plain_kernel(MatDesc d) {
  if (*d.status != 0) return;
  heavy_rows(d);
}

__global__ void __launch_bounds__(kBlock) heavy_batch_kernel(const MatDesc* descs) {
  const MatDesc d = descs[blockIdx.x];
  if (*d.status != 0) return;
  if (d.scheme == KTAU_SCHEME_NAIVE) {
    // the bit-set count is exact for tied pairs too: no composite pass
    if (threadIdx.x == 0) *d.heavy_count = 0;
    return;
  }
  heavy_rows(d);
}

// Every pair of heavy rows of one matrix, grid-strided over its heavy
// sub-triangle; results land at the pair's job slot if it is in range.
template <int K, int G>
__device__ void composite_matrix(const MatDesc& d, uint32_t* lds_all, uint32_t* red) {
  constexpr int kGroups = kBlock / G;
  const int group = threadIdx.x / G;
  const int lane = threadIdx.x % G;
  uint32_t* buf = lds_all + group * CompLds<K, G>::kWords;
  const int64_t hc = *d.heavy_count;
  const int64_t jobs = hc * (hc - 1) / 2;
  for (int64_t i = (int64_t)blockIdx.x * kGroups + group; i < jobs;
       i += (int64_t)gridDim.x * kGroups) {
    int64_t a, b;
    strict_pair(hc, i, a, b);
    const int64_t y = d.heavy[a], x = d.heavy[b];
    const int64_t J = strict_job(d.m, y, x);
    if (J < d.J_begin || J >= d.J_end) continue;
    uint32_t nd, n3;
    pair_composite<K, G>(d.rv, y, d.rv, x, d.n, buf, red, lane, nd, n3);
    if (lane == 0) store_pair(d.out, J - d.J_begin, d.n, d.rv.n1[y], d.rv.n1[x], nd, n3);
  }
}

// The composite pass runs on whole waves or 256-lane blocks, chosen on the
// host by n (the largest n of a batch): (K, G) = (2, 64) for n <= 128 up to
// (64, 256) for n <= 16384.  It is rare; the fast path's scheme does not
// matter to it.
#define KTAU_FOR_EACH_COMPOSITE(X) \
  X(128, 2, 64) X(256, 4, 64) X(512, 8, 64) X(1024, 16, 64) X(2048, 8, 256) X(4096, 16, 256) \
  X(8192, 32, 256) X(16384, 64, 256)

template <int K, int G>
__global__ void __launch_bounds__(kBlock) composite_plain_kernel(MatDesc d) {
  constexpr int kGroups = kBlock / G;
  __shared__ uint32_t lds[kGroups * CompLds<K, G>::kWords];
  __shared__ uint32_t red[kWavesPerBlock];
  if (*d.status != 0) return;
  if (*d.heavy_count < 2) return;
  composite_matrix<K, G>(d, lds, red);
}

template <int K, int G>
__global__ void __launch_bounds__(kBlock) composite_batch_kernel(const MatDesc* descs,
                                                                 int64_t count) {
  constexpr int kGroups = kBlock / G;
  __shared__ uint32_t lds[kGroups * CompLds<K, G>::kWords];
  __shared__ uint32_t red[kWavesPerBlock];
  for (int64_t b = 0; b < count; ++b) {
    const MatDesc d = descs[b];
    if (*d.status != 0) continue;
    if (*d.heavy_count < 2) continue;
    composite_matrix<K, G>(d, lds, red);
  }
}

int device_cus() {
  static const int cus = [] {
    int dev = 0, v = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
      hipDeviceProp_t p;
      if (hipGetDeviceProperties(&p, dev) == hipSuccess) v = p.multiProcessorCount;
    }
    return v;
  }();
  return cus;
}

template <int K, int G>
hipError_t launch_tiles_t(const MatDesc& d, hipStream_t s) {
  int64_t grid = d.n_units < (1ll << 30) ? d.n_units : (1ll << 30);
  if (grid < 1) return hipSuccess;
  hipLaunchKernelGGL((pairs_tiles_kernel<K, G>), dim3((unsigned)grid), dim3(kBlock), 0, s, d);
  return hipGetLastError();
}

template <int K, int G>
hipError_t launch_jobs_t(const MatDesc& d, hipStream_t s) {
  constexpr int kGroups = FastLds<K, G>::kGroups;
  int64_t count = d.J_end - d.J_begin;
  int64_t grid = (count + kGroups - 1) / kGroups;
  if (grid > kMaxPairGrid) grid = kMaxPairGrid;
  if (grid < 1) return hipSuccess;
  hipLaunchKernelGGL((pairs_jobs_kernel<K, G>), dim3((unsigned)grid), dim3(kBlock), 0, s, d);
  return hipGetLastError();
}

}  // namespace

const char* scheme_name(int s) {
  static const char* names[] = {"wave_k2",   "wave_k4",   "wave_k8",   "wave_k16",  "block_k4",
                                "block_k8",  "block_k16", "sub8_k16",  "sub16_k16", "sub16_k32",
                                "sub16_k64", "sub32_k32", "sub32_k64", "wave_k32",  "wave_k64",
                                "sub8_k32",  "sub8_k64",  "block_k32", "block_k64",
                                "block_k128", "merge_k32", "merge_k64"};
  static_assert(sizeof(names) / sizeof(names[0]) == kNumSchemes, "one name per scheme");
  if (s == KTAU_SCHEME_NAIVE) return "naive_bits";
  return (s >= 0 && s < kNumSchemes) ? names[s] : "invalid";
}

// Network scheme per capacity class on MI355X: the fastest measured on
// log-normal rows with a run of zeros, over every scheme whose network fits,
// except up to 512 samples, where 8-lane groups (3% faster there) split the
// in-run tie walk of heavily tied rows over too few lanes.
int network_scheme(int64_t n) {
  if (n <= 128) return kSub8K16;
  if (n <= 256) return kSub8K32;
  if (n <= 512) return kSub16K32;
  if (n <= 1024) return kSub16K64;
  if (n <= 2048) return kSub32K64;
  if (n <= 4096) return kWaveK64;
  if (n <= 8192) return kBlockK32;
  if (n <= 16384) return kBlockK64;
  return kBlockK128;
}

// Up to 4096 samples a whole pair fits one wave's network; longer rows take
// the merge scheme (chunks of 4096 on a network, merge path above them).
int default_scheme(int64_t n) { return n <= 4096 ? network_scheme(n) : kMergeK64; }

int default_q(int64_t n) { return n <= 4096 ? 8 : n <= 16384 ? 4 : 2; }

// Plain launches know m: from 8192 rows on, 16 x 16 tiles (half the row
// fetches of 8 x 8, and still ample tiles to fill the chip).
int plain_q(int64_t m, int64_t n) { return n <= 4096 && m >= 8192 ? 16 : default_q(n); }

hipError_t launch_pair_tiles(const MatDesc& d, hipStream_t s) {
  switch (d.scheme) {
#define KTAU_CASE(S, K, G) \
  case S: return launch_tiles_t<K, G>(d, s);
    KTAU_FOR_EACH_SCHEME(KTAU_CASE)
#undef KTAU_CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_pairs_plain(const MatDesc& d, bool tiles, hipStream_t s) {
  hipError_t e;
#define KTAU_CASE(S, K, G) \
  case S: e = tiles ? launch_tiles_t<K, G>(d, s) : launch_jobs_t<K, G>(d, s); break;
  switch (d.scheme) {
    KTAU_FOR_EACH_SCHEME(KTAU_CASE)
    case kMergeK32:
    case kMergeK64: e = launch_pairs_merge(d, s); break;
    default: return hipErrorInvalidValue;
  }
#undef KTAU_CASE
  if (e != hipSuccess) return e;
  // heavy rows, then the composite pass over their pairs (none beyond
  // kCompositeMaxN: there every pair counts its ties directly)
  if (d.n > kCompositeMaxN) return hipSuccess;
  hipLaunchKernelGGL(heavy_plain_kernel, dim3(1), dim3(kBlock), 0, s, d);
  if ((e = hipGetLastError()) != hipSuccess) return e;
#define KTAU_COMP(N, K, G)                                                                    \
  if (d.n <= N) {                                                                             \
    hipLaunchKernelGGL((composite_plain_kernel<K, G>), dim3((unsigned)device_cus()),           \
                       dim3(kBlock), 0, s, d);                                                 \
    return hipGetLastError();                                                                 \
  }
  KTAU_FOR_EACH_COMPOSITE(KTAU_COMP)
#undef KTAU_COMP
  return hipErrorInvalidValue;
}

template <int K, int G>
hipError_t persistent_t(const MatDesc* descs, int64_t count, int64_t total_units,
                        const int64_t* prefix, int64_t* counters, const int32_t* status,
                        hipStream_t s) {
  // occupancy is queried once per scheme (first call, outside any capture)
  static const int per_cu = [] {
    int v = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, pairs_persistent_kernel<K, G>, kBlock,
                                                     0) != hipSuccess ||
        v < 1)
      v = 1;
    return v;
  }();
  int64_t grid = (int64_t)device_cus() * per_cu;
  if (grid > total_units) grid = total_units;
  if (grid < 1) return hipSuccess;
  hipLaunchKernelGGL((pairs_persistent_kernel<K, G>), dim3((unsigned)grid), dim3(kBlock), 0, s,
                     descs, count, total_units, prefix, counters, status);
  return hipGetLastError();
}

hipError_t launch_pairs_persistent(int scheme, const MatDesc* d, int64_t count, int64_t total,
                                   const int64_t* prefix, int64_t* counters,
                                   const int32_t* status, hipStream_t s) {
  switch (scheme) {
#define KTAU_CASE(S, K, G) \
  case S: return persistent_t<K, G>(d, count, total, prefix, counters, status, s);
    KTAU_FOR_EACH_SCHEME(KTAU_CASE)
#undef KTAU_CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_heavy(const MatDesc& d, hipStream_t s) {
  hipLaunchKernelGGL(heavy_plain_kernel, dim3(1), dim3(kBlock), 0, s, d);
  return hipGetLastError();
}

hipError_t launch_tie_passes_batch(const MatDesc* descs_dev, int64_t count, int max_n,
                                   hipStream_t s) {
  // matrices longer than kCompositeMaxN have no heavy rows (their budget is
  // unbounded); the composite kernel for the others holds kCompositeMaxN
  if (max_n > kCompositeMaxN) max_n = (int)kCompositeMaxN;
  hipLaunchKernelGGL(heavy_batch_kernel, dim3((unsigned)count), dim3(kBlock), 0, s, descs_dev);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
#define KTAU_COMP(N, K, G)                                                                    \
  if (max_n <= N) {                                                                           \
    hipLaunchKernelGGL((composite_batch_kernel<K, G>), dim3((unsigned)device_cus()),           \
                       dim3(kBlock), 0, s, descs_dev, count);                                  \
    return hipGetLastError();                                                                 \
  }
  KTAU_FOR_EACH_COMPOSITE(KTAU_COMP)
#undef KTAU_COMP
  return hipErrorInvalidValue;
}

}  // namespace ktau
