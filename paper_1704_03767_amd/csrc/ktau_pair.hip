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
#include "ktau_bitonic.h"
#include "ktau_internal.h"

namespace ktau {
namespace {

constexpr int kBlock = 256;      // threads per workgroup for every pair kernel
constexpr int kWavesPerBlock = kBlock / 64;

// ---------------------------------------------------------------- utilities

template <int G>
__device__ __forceinline__ void group_sync() {
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

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// Sum over the group; every lane gets the total.
template <int G>
__device__ __forceinline__ uint32_t group_sum(uint32_t v, uint32_t* red) {
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

// K consecutive uint16 from a 2K-byte aligned address, by vector loads.
template <int K>
__device__ __forceinline__ void load_u16(const uint16_t* p, uint16_t (&out)[K]) {
  if constexpr (K == 2) {
    const uint32_t w = *(const uint32_t*)p;
    out[0] = (uint16_t)w;
    out[1] = (uint16_t)(w >> 16);
  } else if constexpr (K == 4) {
    const uint2 w = *(const uint2*)p;
    out[0] = (uint16_t)w.x;
    out[1] = (uint16_t)(w.x >> 16);
    out[2] = (uint16_t)w.y;
    out[3] = (uint16_t)(w.y >> 16);
  } else {
#pragma unroll
    for (int i = 0; i < K / 8; ++i) {
      const uint4 w = ((const uint4*)p)[i];
      const uint32_t a[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        out[8 * i + 2 * c] = (uint16_t)a[c];
        out[8 * i + 2 * c + 1] = (uint16_t)(a[c] >> 16);
      }
    }
  }
}

template <int K>
__device__ __forceinline__ void store_u16(uint16_t* p, const uint16_t (&in)[K]) {
#pragma unroll
  for (int i = 0; i < K / 2; ++i)
    ((uint32_t*)p)[i] = (uint32_t)in[2 * i] | ((uint32_t)in[2 * i + 1] << 16);
}

// Step 5 and Eq. 1/3: store the counts and tau of job slot `slot`.
__device__ __forceinline__ void store_pair(const PairOut& o, int64_t slot, int64_t n, int64_t n1y,
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

// ======================================================= main (fast) path

// LDS words per group: the v rank row (uint16), reused for v' on the tie
// path, plus the network's exchange buffer for 256-lane groups.
template <int K, int G>
struct FastLds {
  static constexpr int kRowWords = K * G / 2;
  static constexpr int kXWords = G == 256 ? (K / 2) * 256 : 0;
  static constexpr int kWords = kRowWords + kXWords + 16;
};

// n_d and n3 of rows (y, x) unless both rows exceed the tie budget (then
// returns false and the composite pass handles the pair).  Called by every
// lane of the group with the same arguments.
template <int K, int G>
__device__ __forceinline__ bool pair_fast(const RankView& rv, int64_t y, int64_t x, int n,
                                          int64_t budget, uint32_t* lds, uint32_t* red, int lane,
                                          uint32_t& nd, uint32_t& n3) {
  using FL = FastLds<K, G>;
  using Net = bitonic::Net<K, G>;
  const int64_t n1y = rv.n1[y], n1x = rv.n1[x];
  if (n1y > budget && n1x > budget) return false;
  int64_t u = y, v = x, n1u = n1y;
  if (n1x < n1y) {
    u = x;
    v = y;
    n1u = n1x;
  }
  const int k0 = lane * K;
  const bool in_row = k0 + K <= rv.ld;           // vector loads stay inside the row
  uint16_t* row = (uint16_t*)lds;
  uint32_t* xbuf = lds + FL::kRowWords;
  // stage v's rank row in LDS
  {
    uint16_t r[K];
    if (in_row) {
      load_u16<K>(rv.rank + v * rv.ld + k0, r);
      store_u16<K>(row + k0, r);
    }
  }
  uint16_t p[K];
  if (in_row) load_u16<K>(rv.perm + u * rv.ld + k0, p);
  group_sync<G>();
  uint32_t key[K];
#pragma unroll
  for (int r = 0; r < K; ++r) key[r] = (k0 + r < n) ? (uint32_t)row[p[r]] : 0x7FFFu;
  uint32_t xin = 0, tie = 0;
  if (n1u != 0) {
    // v' in u order replaces the rank row once every lane has gathered
    group_sync<G>();
    {
      uint16_t kv[K];
#pragma unroll
      for (int r = 0; r < K; ++r) kv[r] = (uint16_t)key[r];
      if (in_row) store_u16<K>(row + k0, kv);
    }
    group_sync<G>();
    // positions up to the end of u's last tie run, spread over lanes with
    // stride G so that one run is shared by many lanes; each is compared
    // with the earlier positions of its run
    const uint16_t* ru = rv.rstart + u * rv.ld;
    const int end = rv.tie_end[u];
    for (int k = lane; k < end; k += G) {
      const int s = ru[k];
      const uint32_t me = row[k];
      for (int j = s; j < k; ++j) {
        const uint32_t o = row[j];
        xin += o > me ? 1u : 0u;
        tie += o == me ? 1u : 0u;
      }
    }
  }
  const uint32_t inv = group_sum<G>(Net::count(key, lane, xbuf), red);
  if (n1u != 0) {
    nd = inv - group_sum<G>(xin, red);
    n3 = group_sum<G>(tie, red);
  } else {
    nd = inv;
    n3 = 0;
  }
  return true;
}

// One q x q tile (Eq. 11-14) of a matrix; its pairs go to the waves
// round-robin (G = 64) or one after another to the whole workgroup (G = 256).
template <int K, int G>
__device__ __forceinline__ void tile_pairs(const MatDesc& d, int64_t t, uint32_t* lds_all,
                                           uint32_t* red) {
  constexpr int kGroups = kBlock / G;
  const int group = threadIdx.x / G;
  const int lane = threadIdx.x % G;
  uint32_t* lds = lds_all + group * FastLds<K, G>::kWords;
  int64_t yq, xq;
  tile_coord(d.w, t, yq, xq);
  const int q = d.q;
  const int64_t budget = direct_budget(d.n);
  for (int p = group; p < q * q; p += kGroups) {
    const int64_t y = yq * q + p / q, x = xq * q + p % q;
    if (y >= x || x >= d.m) continue;
    uint32_t nd, n3;
    if (pair_fast<K, G>(d.rv, y, x, d.n, budget, lds, red, lane, nd, n3) && lane == 0)
      store_pair(d.out, strict_job(d.m, y, x), d.n, d.rv.n1[y], d.rv.n1[x], nd, n3);
  }
}

// Plain launch, tile order.
template <int K, int G>
__global__ void __launch_bounds__(kBlock) pairs_tiles_kernel(MatDesc d) {
  __shared__ uint32_t lds[(kBlock / G) * FastLds<K, G>::kWords];
  __shared__ uint32_t red[kWavesPerBlock];
  if (*d.status != 0) return;
  for (int64_t t = blockIdx.x; t < d.n_units; t += gridDim.x) tile_pairs<K, G>(d, t, lds, red);
}

// Plain launch, job order: strict job ids [J_begin, J_end), one per group.
template <int K, int G>
__global__ void __launch_bounds__(kBlock) pairs_jobs_kernel(MatDesc d) {
  constexpr int kGroups = kBlock / G;
  __shared__ uint32_t lds[kGroups * FastLds<K, G>::kWords];
  __shared__ uint32_t red[kWavesPerBlock];
  if (*d.status != 0) return;
  const int group = threadIdx.x / G;
  const int lane = threadIdx.x % G;
  uint32_t* buf = lds + group * FastLds<K, G>::kWords;
  const int64_t count = d.J_end - d.J_begin;
  const int64_t budget = direct_budget(d.n);
  for (int64_t i = (int64_t)blockIdx.x * kGroups + group; i < count;
       i += (int64_t)gridDim.x * kGroups) {
    int64_t y, x;
    strict_pair(d.m, d.J_begin + i, y, x);
    uint32_t nd, n3;
    if (pair_fast<K, G>(d.rv, y, x, d.n, budget, buf, red, lane, nd, n3) && lane == 0)
      store_pair(d.out, i, d.n, d.rv.n1[y], d.rv.n1[x], nd, n3);
  }
}

// Persistent launch over the concatenated tile spaces of the matrices of one
// scheme class.  Units (tiles) are taken from an atomic counter; a unit is
// located by binary search on the per-matrix unit prefix, then Eq. 13-14
// inside its matrix.
template <int K, int G>
__global__ void __launch_bounds__(kBlock)
pairs_persistent_kernel(const MatDesc* __restrict__ descs, int64_t count, int64_t total_units,
                        const int64_t* __restrict__ unit_prefix, int64_t* __restrict__ counter,
                        const int32_t* __restrict__ status) {
  __shared__ uint32_t lds[(kBlock / G) * FastLds<K, G>::kWords];
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
    tile_pairs<K, G>(descs[lo], unit - unit_prefix[lo], lds, red);
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
  heavy_rows(d);
}

// ============================================ composite pass (LDS merge)

// In-lane: strict inversions among the lane's K keys, then a bitonic sorting
// network leaves them ascending (indices are compile-time, keys stay in
// registers).
template <int K>
__device__ __forceinline__ uint32_t lane_sort_count(uint32_t (&key)[K]) {
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

// buf holds 2*G*K + 16 keys.  On entry every lane's K keys are sorted; on exit
// the group's keys are sorted (lane-blocked) and the return value is this
// lane's share of the cross-lane inversions (Algorithm 2: a right-run key
// taken before left-run keys adds the number of left keys still waiting).
template <int K, int G>
__device__ __forceinline__ uint32_t merge_levels(uint32_t (&key)[K], uint32_t* buf, int lane) {
  constexpr int N = G * K;
  uint32_t cnt = 0;
  int cur = 0;
#pragma unroll 1
  for (int s = K; s < N; s <<= 1) {
    uint32_t* b = buf + cur * N;
#pragma unroll
    for (int r = 0; r < K; ++r) b[lane * K + r] = key[r];
    group_sync<G>();
    const int pos = lane * K;
    const int l0 = pos & ~(2 * s - 1);
    const int diag = pos - l0;
    const uint32_t* A = b + l0;
    // merge path: number of A keys among the first `diag` outputs, A first
    // on equal keys
    int lo = diag > s ? diag - s : 0;
    int hi = diag < s ? diag : s;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (A[mid] <= A[s + diag - 1 - mid]) lo = mid + 1;
      else hi = mid;
    }
    int ia = lo, ib = diag - lo;
    uint32_t a = ia < s ? A[ia] : kSentinel;
    uint32_t bb = ib < s ? A[s + ib] : kSentinel;
#pragma unroll
    for (int t = 0; t < K; ++t) {
      const bool takeB = bb < a;   // strict: equal keys are not discordant
      key[t] = takeB ? bb : a;
      cnt += takeB ? (uint32_t)(s - ia) : 0u;
      ia += takeB ? 0 : 1;
      ib += takeB ? 1 : 0;
      const int idx = takeB ? ib : ia;
      const uint32_t raw = A[takeB ? s + ib : ia];
      const uint32_t nv = idx < s ? raw : kSentinel;
      a = takeB ? a : nv;
      bb = takeB ? nv : bb;
    }
    cur ^= 1;
  }
  return cnt;
}

template <int K, int G>
__device__ __forceinline__ uint32_t sort_count(uint32_t (&key)[K], uint32_t* buf, int lane,
                                               uint32_t* red) {
  uint32_t c = lane_sort_count<K>(key);
  c += merge_levels<K, G>(key, buf, lane);
  return group_sum<G>(c, red);
}

template <int K, int G>
struct CompLds {
  static constexpr int kWords = 2 * G * K + 16;
};

// Both rows heavy: Step 1 literally (sort by (u run, v')), joint ties from
// equal composite keys, then Step 3 on v' alone.
template <int K, int G>
__device__ void pair_composite(const RankView& rv, int64_t y, int64_t x, int n, uint32_t* buf,
                               uint32_t* red, int lane, uint32_t& nd, uint32_t& n3) {
  const int64_t n1y = rv.n1[y], n1x = rv.n1[x];
  int64_t u = y, v = x;
  if (n1x < n1y) {
    u = x;
    v = y;
  }
  const uint16_t* pu = rv.perm + u * rv.ld;
  const uint16_t* rk = rv.rank + v * rv.ld;
  const uint16_t* ru = rv.rstart + u * rv.ld;
  const int k0 = lane * K;
  uint32_t key[K];
#pragma unroll
  for (int r = 0; r < K; ++r) {
    const int k = k0 + r;
    key[r] = k < n ? ((uint32_t)ru[k] << 16) | (uint32_t)rk[pu[k]] : kPadKey;
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
      int lo = 0, hi = k;   // first position holding a key equal to key[r]
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (sb[mid] < key[r]) lo = mid + 1;
        else hi = mid;
      }
      tie += (uint32_t)(k - lo);
    }
  }
  n3 = group_sum<G>(tie, red);
#pragma unroll
  for (int r = 0; r < K; ++r)
    if (key[r] != kPadKey) key[r] &= 0xFFFFu;
  group_sync<G>();
  nd = sort_count<K, G>(key, buf, lane, red);
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
    pair_composite<K, G>(d.rv, y, x, d.n, buf, red, lane, nd, n3);
    if (lane == 0) store_pair(d.out, J - d.J_begin, d.n, d.rv.n1[y], d.rv.n1[x], nd, n3);
  }
}

constexpr int kCompLdsWords = CompLds<16, 256>::kWords > 4 * CompLds<16, 64>::kWords
                                  ? CompLds<16, 256>::kWords
                                  : 4 * CompLds<16, 64>::kWords;

__device__ void composite_dispatch(const MatDesc& d, uint32_t* lds, uint32_t* red) {
  switch (d.scheme) {
    case kWaveK2: composite_matrix<2, 64>(d, lds, red); break;
    case kWaveK4: composite_matrix<4, 64>(d, lds, red); break;
    case kWaveK8: composite_matrix<8, 64>(d, lds, red); break;
    case kWaveK16: composite_matrix<16, 64>(d, lds, red); break;
    case kBlockK4: composite_matrix<4, 256>(d, lds, red); break;
    case kBlockK8: composite_matrix<8, 256>(d, lds, red); break;
    default: composite_matrix<16, 256>(d, lds, red); break;
  }
}

__global__ void __launch_bounds__(kBlock) composite_plain_kernel(MatDesc d) {
  __shared__ uint32_t lds[kCompLdsWords];
  __shared__ uint32_t red[kWavesPerBlock];
  if (*d.status != 0) return;
  if (*d.heavy_count < 2) return;
  composite_dispatch(d, lds, red);
}

__global__ void __launch_bounds__(kBlock) composite_batch_kernel(const MatDesc* descs,
                                                                 int64_t count) {
  __shared__ uint32_t lds[kCompLdsWords];
  __shared__ uint32_t red[kWavesPerBlock];
  for (int64_t b = 0; b < count; ++b) {
    const MatDesc d = descs[b];
    if (*d.status != 0) continue;
    if (*d.heavy_count < 2) continue;
    composite_dispatch(d, lds, red);
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
  constexpr int kGroups = kBlock / G;
  int64_t count = d.J_end - d.J_begin;
  int64_t grid = (count + kGroups - 1) / kGroups;
  if (grid > (1ll << 30)) grid = 1ll << 30;
  if (grid < 1) return hipSuccess;
  hipLaunchKernelGGL((pairs_jobs_kernel<K, G>), dim3((unsigned)grid), dim3(kBlock), 0, s, d);
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

hipError_t launch_pairs_plain(const MatDesc& d, bool tiles, hipStream_t s) {
  hipError_t e;
#define KTAU_CASE(S, K, G) \
  case S: e = tiles ? launch_tiles_t<K, G>(d, s) : launch_jobs_t<K, G>(d, s); break;
  switch (d.scheme) {
    KTAU_CASE(kWaveK2, 2, 64)
    KTAU_CASE(kWaveK4, 4, 64)
    KTAU_CASE(kWaveK8, 8, 64)
    KTAU_CASE(kWaveK16, 16, 64)
    KTAU_CASE(kBlockK4, 4, 256)
    KTAU_CASE(kBlockK8, 8, 256)
    KTAU_CASE(kBlockK16, 16, 256)
    default: return hipErrorInvalidValue;
  }
#undef KTAU_CASE
  if (e != hipSuccess) return e;
  // heavy rows, then the composite pass over their pairs
  hipLaunchKernelGGL(heavy_plain_kernel, dim3(1), dim3(kBlock), 0, s, d);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(composite_plain_kernel, dim3((unsigned)device_cus()), dim3(kBlock), 0, s, d);
  return hipGetLastError();
}

template <int K, int G>
hipError_t persistent_t(const MatDesc* descs, int64_t count, int64_t total_units,
                        const int64_t* prefix, int64_t* counter, const int32_t* status,
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
                     descs, count, total_units, prefix, counter, status);
  return hipGetLastError();
}

hipError_t launch_pairs_persistent(int scheme, const MatDesc* d, int64_t count, int64_t total,
                                   const int64_t* prefix, int64_t* counter, const int32_t* status,
                                   hipStream_t s) {
  switch (scheme) {
    case kWaveK2: return persistent_t<2, 64>(d, count, total, prefix, counter, status, s);
    case kWaveK4: return persistent_t<4, 64>(d, count, total, prefix, counter, status, s);
    case kWaveK8: return persistent_t<8, 64>(d, count, total, prefix, counter, status, s);
    case kWaveK16: return persistent_t<16, 64>(d, count, total, prefix, counter, status, s);
    case kBlockK4: return persistent_t<4, 256>(d, count, total, prefix, counter, status, s);
    case kBlockK8: return persistent_t<8, 256>(d, count, total, prefix, counter, status, s);
    case kBlockK16: return persistent_t<16, 256>(d, count, total, prefix, counter, status, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_tie_passes_batch(const MatDesc* descs_dev, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(heavy_batch_kernel, dim3((unsigned)count), dim3(kBlock), 0, s, descs_dev);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(composite_batch_kernel, dim3((unsigned)device_cus()), dim3(kBlock), 0, s,
                     descs_dev, count);
  return hipGetLastError();
}

}  // namespace ktau
