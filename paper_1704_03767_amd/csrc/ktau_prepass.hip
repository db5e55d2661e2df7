// Rank pre-pass: every variable is ranked once (Sec. 3), and the per-vector
// half of the sorting kernel's Steps 1, 2 and 4 (Sec. 3.2) is done here once
// per row instead of once per pair: the ascending order of the row (ties by
// sample index), its dense ranks, the start of every tie run, and the tie term
// n1 = sum t(t-1)/2; and the list of its tie runs with the number of
// within-run pairs before each, so that the pair kernels can share a pair's
// in-run comparisons evenly among lanes.
//
// One 256-thread workgroup per row.  The row's (value key, sample) pairs are
// bitonic-sorted in LDS as 64-bit words (order-preserving 32-bit key << 16 |
// sample), then block scans produce dense ranks and run starts.  Rows longer
// than 16384 samples sort blocks of 16384 in LDS and run the stages that span
// blocks in a global scratch slot.  Into a pair workspace of rows up to 32768
// samples the sample indices and ranks are written doubled (byte offsets into
// a rank row, and ranks with a free low bit for the pair network's tag);
// longer rows, and the rank entry point, get them plain.
#include <limits.h>

#include "ktau_internal.h"

namespace ktau {
namespace {

constexpr int kThreads = 256;       // rows up to 4096 samples, and batches
constexpr int kLongThreads = 1024;  // rows of 8192 samples and more

// Order-preserving map float32 -> uint32 with -0.0 folded onto +0.0 (IEEE
// equality decides ties).  NaN never reaches a comparison: it is flagged.
__device__ inline uint32_t float_key(float f, bool& nan) {
  uint32_t b = __float_as_uint(f);
  nan = (b & 0x7fffffffu) > 0x7f800000u;
  if (b == 0x80000000u) b = 0u;
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// Block-wide exclusive scan (sum) of one int per thread; also returns the total.
template <int T>
__device__ inline int block_excl_sum(int v, int* sh, int& total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int incl = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int t = __shfl_up(incl, d, 64);
    if (lane >= d) incl += t;
  }
  if (lane == 63) sh[wave] = incl;
  __syncthreads();
  int base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < T / 64; ++w) {
    int s = sh[w];
    if (w < wave) base += s;
    tot += s;
  }
  __syncthreads();
  total = tot;
  return base + incl - v;
}

// Block-wide exclusive scan (max) of one non-negative int per thread.
template <int T>
__device__ inline int block_excl_max(int v, int* sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int incl = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int t = __shfl_up(incl, d, 64);
    if (lane >= d) incl = max(incl, t);
  }
  int excl_in_wave = __shfl_up(incl, 1, 64);
  if (lane == 0) excl_in_wave = 0;
  if (lane == 63) sh[wave] = incl;
  __syncthreads();
  int base = 0;
#pragma unroll
  for (int w = 0; w < T / 64; ++w)
    if (w < wave) base = max(base, sh[w]);
  __syncthreads();
  return max(base, excl_in_wave);
}

// Block-wide exclusive suffix scan (min): the minimum of v over the threads
// after this one (INT_MAX for the last).
template <int T>
__device__ inline int block_excl_suffix_min(int v, int* sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int incl = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int t = __shfl_down(incl, d, 64);
    if (lane + d < 64) incl = min(incl, t);
  }
  int excl_in_wave = __shfl_down(incl, 1, 64);
  if (lane == 63) excl_in_wave = INT_MAX;
  if (lane == 0) sh[wave] = incl;
  __syncthreads();
  int after = INT_MAX;
#pragma unroll
  for (int w = 0; w < T / 64; ++w)
    if (w > wave) after = min(after, sh[w]);
  __syncthreads();
  return min(after, excl_in_wave);
}

// Loads row x as 64-bit sort words (order-preserving key << 16 | sample; all
// ones past n) for positions base .. base+cnt-1 into s; tells every thread of
// the block whether a NaN was seen.
template <int T>
__device__ inline bool load_keys(const float* __restrict__ x, int n, int base, int cnt,
                                 uint64_t* s) {
  bool any_nan = false;
  for (int i = threadIdx.x; i < cnt; i += T) {
    const int g = base + i;
    uint64_t w = ~0ull;
    if (g < n) {
      bool nan;
      const uint32_t k = float_key(x[g], nan);
      any_nan |= nan;
      w = ((uint64_t)k << 16) | (uint64_t)g;
    }
    s[i] = w;
  }
  return __syncthreads_or(any_nan);
}

// Compare-exchange stages of an ascending bitonic sort, applied to the cnt
// words at s that sit at positions base.. of the whole sort: levels (block
// sizes) k_first .. k_last, the first of them from stage distance j_first
// down, every later one complete.  A block of size k holding position g runs
// ascending iff (g & k) == 0.  Every stage distance used must be below cnt.
template <int T>
__device__ inline void bitonic_stages(uint64_t* s, int cnt, int base, int k_first, int k_last,
                                      int j_first) {
  for (int k = k_first; k <= k_last; k <<= 1) {
    for (int j = (k == k_first ? j_first : k >> 1); j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < cnt; i += T) {
        const int p = i ^ j;
        if (p > i) {
          const uint64_t a = s[i], b = s[p];
          const bool up = ((base + i) & k) == 0;
          if ((a > b) == up) {
            s[i] = b;
            s[p] = a;
          }
        }
      }
      __syncthreads();
    }
  }
}

// Passes over the row's npow2 ascending sort words `keys` (LDS, or global
// scratch for long rows): perm, dense ranks, run starts and n1, then the
// list of tie runs.
template <int T>
__device__ __forceinline__ void rank_outputs(const uint64_t* keys, int64_t row, int n, int npow2,
                             uint16_t* __restrict__ perm, uint16_t* __restrict__ rank,
                             uint16_t* __restrict__ rstart, int64_t ld,
                             int64_t* __restrict__ n1_ws, int64_t* __restrict__ n1_out,
                             int32_t* __restrict__ nruns, int32_t* __restrict__ nlong,
                             uint64_t* __restrict__ runs, int dbl) {
  __shared__ int s_scan[T / 64];
  __shared__ unsigned long long s_n1;
  const int tid = threadIdx.x;
  if (tid == 0) s_n1 = 0;
  auto key_at = [&](int k) { return keys[k] >> 16; };
  // Each thread owns `chunk` consecutive sorted positions.
  const int chunk = npow2 / T > 0 ? npow2 / T : 1;
  const int k0 = tid * chunk;
  // Pass 1: count value changes (for dense ranks); the last and the first
  // run start after position 0 in the chunk.
  int changes = 0, last_start = 0, first_change = INT_MAX;
  for (int c = 0; c < chunk; ++c) {
    const int k = k0 + c;
    if (k < n && k > 0 && key_at(k) != key_at(k - 1)) {
      ++changes;
      last_start = k;
      first_change = min(first_change, k);
    }
  }
  int total_changes;
  const int rank_base = block_excl_sum<T>(changes, s_scan, total_changes);
  const int start_base = block_excl_max<T>(last_start, s_scan);
  // the first run start after this chunk (n if none): where a run still open
  // at the chunk's end stops
  const int next_start = min(block_excl_suffix_min<T>(first_change, s_scan), n);
  // Pass 2: write perm, rank and rstart; accumulate n1.
  uint16_t* prow = perm ? perm + row * ld : nullptr;
  uint16_t* rrow = rank ? rank + row * ld : nullptr;
  uint16_t* srow = rstart ? rstart + row * ld : nullptr;
  int r = rank_base, st = start_base;
  unsigned long long ties = 0;
  for (int c = 0; c < chunk; ++c) {
    const int k = k0 + c;
    if (k < n) {
      const uint64_t w = keys[k];
      const int sample = (int)(w & 0xFFFFu);
      if (k > 0 && (w >> 16) != key_at(k - 1)) {
        ++r;
        st = k;
      }
      if (prow) prow[k] = (uint16_t)(sample << dbl);
      if (rrow) rrow[sample] = (uint16_t)(r << dbl);
      if (srow) srow[k] = (uint16_t)st;
      ties += (unsigned long long)(k - st);
    } else if (k < ld) {
      if (prow) prow[k] = (uint16_t)(k << dbl);
      if (srow) srow[k] = (uint16_t)k;
    }
  }
  // Padding of rows longer than the sort width (a workspace row of fewer
  // than 64 samples is padded to 128).
  for (int k = npow2 + tid; k < ld; k += T) {
    if (prow) prow[k] = (uint16_t)(k << dbl);
    if (srow) srow[k] = (uint16_t)k;
  }
  // Tail positions n..ld-1 map to themselves and a padding rank at or above
  // every real rank (0xFFFE doubled, 0xFFFF plain), so the pair kernels
  // gather padding keys without a bounds test.
  if (rrow)
    for (int i = n + tid; i < ld; i += T) rrow[i] = (uint16_t)(dbl ? 0xFFFEu : 0xFFFFu);
  atomicAdd(&s_n1, ties);
  __syncthreads();
  if (tid == 0) {
    if (n1_ws) n1_ws[row] = (int64_t)s_n1;
    if (n1_out) n1_out[row] = (int64_t)s_n1;
  }
  if (!runs) return;
  // Pass 3: tie runs of length >= 2, in sorted order, the long ones
  // (kLongRunMin < length <= kLongRunMax) listed after all the others.  A
  // thread owns the runs that start in its chunk (a run still open at the
  // chunk's end stops at next_start); block scans give each run its index and
  // the number of within-run pairs of all runs listed before it.
  auto run_end = [&](int k) {
    int e = k + 1;
    while (e < k0 + chunk && e < n && key_at(e) == key_at(k)) ++e;
    return e == k0 + chunk && e < n ? next_start : e;
  };
  auto starts_run = [&](int k) {
    return k + 1 < n && (k == 0 || key_at(k) != key_at(k - 1)) && key_at(k + 1) == key_at(k);
  };
  auto is_long = [](int len) { return len > kLongRunMin && len <= kLongRunMax; };
  // (pair counts below n(n-1)/2 < 2^31 for n <= 65536; products in 64 bits)
  auto run_pairs = [](int len) { return (int)((int64_t)len * (len - 1) / 2); };
  int my_s = 0, my_l = 0, my_sp = 0, my_lp = 0;
  for (int c = 0; c < chunk; ++c) {
    const int k = k0 + c;
    if (starts_run(k)) {
      const int len = run_end(k) - k;
      if (is_long(len)) {
        ++my_l;
        my_lp += run_pairs(len);
      } else {
        ++my_s;
        my_sp += run_pairs(len);
      }
    }
  }
  int tot_s, tot_l, tot_sp, tot_lp;
  int idx_s = block_excl_sum<T>(my_s, s_scan, tot_s);
  int idx_l = tot_s + block_excl_sum<T>(my_l, s_scan, tot_l);
  int pr_s = block_excl_sum<T>(my_sp, s_scan, tot_sp);
  int pr_l = tot_sp + block_excl_sum<T>(my_lp, s_scan, tot_lp);
  uint64_t* rrow_runs = runs + row * (ld / 2);
  for (int c = 0; c < chunk && my_s + my_l > 0; ++c) {
    const int k = k0 + c;
    if (starts_run(k)) {
      const int len = run_end(k) - k;
      const bool lg = is_long(len);
      int& idx = lg ? idx_l : idx_s;
      int& pr = lg ? pr_l : pr_s;
      // entry: start (bits 0-15), length - 1 (16-31), earlier pairs (32-63)
      rrow_runs[idx++] =
          ((uint64_t)(uint32_t)pr << 32) | ((uint64_t)(len - 1) << 16) | (uint64_t)k;
      pr += run_pairs(len);
    }
  }
  if (tid == 0 && nruns) nruns[row] = tot_s + tot_l;
  if (tid == 0 && nlong) nlong[row] = tot_l;
}

// Ranks row `row` of one matrix; s_keys holds npow2 <= kLdsSortMax words.
template <int T>
__device__ __forceinline__ void prepass_row(const float* __restrict__ X, int64_t row, int n, int npow2,
                            uint16_t* __restrict__ perm, uint16_t* __restrict__ rank,
                            uint16_t* __restrict__ rstart, int64_t ld,
                            int64_t* __restrict__ n1_ws, int64_t* __restrict__ n1_out,
                            int32_t* __restrict__ nruns, int32_t* __restrict__ nlong,
                            uint64_t* __restrict__ runs,
                            int32_t* __restrict__ status, uint64_t* s_keys, int dbl) {
  if (load_keys<T>(X + row * (int64_t)n, n, 0, npow2, s_keys)) {
    if (threadIdx.x == 0) atomicExch(status, KTAU_ENAN);
    return;
  }
  bitonic_stages<T>(s_keys, npow2, 0, 2, npow2, 1);
  rank_outputs<T>(s_keys, row, n, npow2, perm, rank, rstart, ld, n1_ws, n1_out, nruns, nlong, runs,
               dbl);
}

// A row longer than kLdsSortMax (H), sorted as npow2 = 2H or 4H words in this
// workgroup's global slot g.  Blocks of H are sorted in LDS (block b
// ascending iff b is even, as the next level wants them) and stored in the
// slot; every later level runs its stages of distance H and more over the
// whole slot, and its stages below H per block in LDS again.  The passes then
// read the sorted words from the slot.
template <int T>
__device__ __forceinline__ void prepass_row_long(const float* __restrict__ X, int64_t row, int n,
                                 uint16_t* __restrict__ perm, uint16_t* __restrict__ rank,
                                 uint16_t* __restrict__ rstart, int64_t ld,
                                 int64_t* __restrict__ n1_ws, int64_t* __restrict__ n1_out,
                                 int32_t* __restrict__ nruns, int32_t* __restrict__ nlong,
                            uint64_t* __restrict__ runs,
                                 int32_t* __restrict__ status, uint64_t* s_keys, uint64_t* g,
                                 int dbl) {
  constexpr int H = kLdsSortMax;
  const float* x = X + row * (int64_t)n;
  int npow2 = 2 * H;
  while (npow2 < n) npow2 <<= 1;
  for (int b = 0; b < npow2 / H; ++b) {
    // A block with r < H samples (the last one, or none at all) sorts only
    // the smallest power of two P >= r of its words, in the block's
    // direction, and the rest of the block is padding: above every sample, it
    // follows an ascending block's sorted words and precedes a descending
    // one's.
    const int r = n - b * H;
    int P = H;
    if (r < H) {
      P = 1;
      while (P < r) P <<= 1;
    }
    if (load_keys<T>(x, n, b * H, P, s_keys)) {
      if (threadIdx.x == 0) atomicExch(status, KTAU_ENAN);
      return;
    }
    const bool desc = (b & 1) != 0;
    // a base with bit P set turns the last level descending and leaves the
    // lower levels as at base 0 (b H has no bits below H)
    bitonic_stages<T>(s_keys, P, desc ? P : 0, 2, P, 1);
    const int off = desc ? H - P : 0;
    for (int i = threadIdx.x; i < H; i += T) {
      const int q = i - off;
      g[b * H + i] = (q >= 0 && q < P) ? s_keys[q] : ~0ull;
    }
    __syncthreads();
  }
  for (int k = 2 * H; k <= npow2; k <<= 1) {
    for (int j = k >> 1; j >= H; j >>= 1) {
      for (int i = threadIdx.x; i < npow2; i += T) {
        const int p = i ^ j;
        if (p > i) {
          const uint64_t a = g[i], c = g[p];
          const bool up = (i & k) == 0;
          if ((a > c) == up) {
            g[i] = c;
            g[p] = a;
          }
        }
      }
      __syncthreads();
    }
    for (int b = 0; b < npow2 / H; ++b) {
      for (int i = threadIdx.x; i < H; i += T) s_keys[i] = g[b * H + i];
      __syncthreads();
      bitonic_stages<T>(s_keys, H, b * H, k, k, H >> 1);
      for (int i = threadIdx.x; i < H; i += T) g[b * H + i] = s_keys[i];
      __syncthreads();
    }
  }
  rank_outputs<T>(g, row, n, npow2, perm, rank, rstart, ld, n1_ws, n1_out, nruns, nlong, runs, dbl);
}

template <int T>
__global__ void __launch_bounds__(T)
prepass_kernel(const float* __restrict__ X, int64_t m, int n, int npow2,
               uint16_t* __restrict__ perm, uint16_t* __restrict__ rank,
               uint16_t* __restrict__ rstart, int64_t ld, int64_t* __restrict__ n1_ws,
               int64_t* __restrict__ n1_out, int32_t* __restrict__ nruns,
               int32_t* __restrict__ nlong, uint64_t* __restrict__ runs,
               int32_t* __restrict__ status, int dbl) {
  extern __shared__ uint64_t s_keys[];
  const int64_t row = blockIdx.x;
  if (row >= m) return;
  prepass_row<T>(X, row, n, npow2, perm, rank, rstart, ld, n1_ws, n1_out, nruns, nlong, runs,
                 status, s_keys, dbl);
}

// Long rows: a grid of at most kSortSlots workgroups, each with its own
// scratch slot of sort_slot_words(n) words, strides over the rows.
__global__ void __launch_bounds__(kLongThreads)
prepass_long_kernel(const float* __restrict__ X, int64_t m, int n, uint16_t* __restrict__ perm,
                    uint16_t* __restrict__ rank, uint16_t* __restrict__ rstart, int64_t ld,
                    int64_t* __restrict__ n1_ws, int64_t* __restrict__ n1_out,
                    int32_t* __restrict__ nruns, int32_t* __restrict__ nlong,
                    uint64_t* __restrict__ runs, int32_t* __restrict__ status,
                    uint64_t* __restrict__ scratch, int dbl) {
  extern __shared__ uint64_t s_keys[];
  uint64_t* g = scratch + (int64_t)blockIdx.x * sort_slot_words(n);
  for (int64_t row = blockIdx.x; row < m; row += gridDim.x) {
    prepass_row_long<kLongThreads>(X, row, n, perm, rank, rstart, ld, n1_ws, n1_out, nruns, nlong,
                                   runs, status, s_keys, g, dbl);
    __syncthreads();
  }
}

// Every row of every matrix of a batch: block b ranks global row b, found by
// binary search on the per-matrix row prefix.  Rows longer than kLdsSortMax
// are left to prepass_long_kernel.
__global__ void __launch_bounds__(kThreads)
prepass_batch_kernel(const MatDesc* __restrict__ descs, int64_t count,
                     const int64_t* __restrict__ row_prefix) {
  extern __shared__ uint64_t s_keys[];
  const int64_t g = blockIdx.x;
  int64_t lo = 0, hi = count - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (row_prefix[mid] <= g) lo = mid;
    else hi = mid - 1;
  }
  const MatDesc& d = descs[lo];
  if (d.n > kLdsSortMax) return;
  const int64_t row = g - row_prefix[lo];
  int npow2 = 64;
  while (npow2 < d.n) npow2 <<= 1;
  prepass_row<kThreads>(d.X, row, d.n, npow2, (uint16_t*)d.rv.perm, (uint16_t*)d.rv.rank,
              (uint16_t*)d.rv.rstart, d.rv.ld, (int64_t*)d.rv.n1, d.n1_out,
              (int32_t*)d.rv.nruns, (int32_t*)d.rv.nlong, (uint64_t*)d.rv.runs, (int32_t*)d.status,
              s_keys, 1);
}

// Rows longer than 8192 samples sort 128 KB of keys in LDS, above the 64 KB
// of dynamic LDS a launch gets by default; raise the kernel's limit.
template <typename F>
hipError_t allow_lds(F kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace

hipError_t launch_prepass_batch(const MatDesc* descs_dev, int64_t count, int64_t total_rows,
                                const int64_t* row_prefix_dev, int max_n, hipStream_t s) {
  if (max_n < 1) return hipSuccess;
  int npow2 = 64;
  while (npow2 < max_n) npow2 <<= 1;
  const size_t lds = (size_t)npow2 * sizeof(uint64_t);
  hipError_t e = allow_lds(prepass_batch_kernel, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(prepass_batch_kernel, dim3((unsigned)total_rows), dim3(kThreads), lds, s,
                     descs_dev, count, row_prefix_dev);
  return hipGetLastError();
}

hipError_t launch_prepass(const float* X, int64_t m, int64_t n, uint16_t* perm, uint16_t* rank,
                          uint16_t* rstart, int64_t ld, int64_t* n1_ws, int64_t* n1_out,
                          int32_t* nruns, int32_t* nlong, uint64_t* runs, int32_t* status,
                          bool doubled,
                          uint64_t* sort_tmp, hipStream_t s) {
  if (n > kLdsSortMax) {
    const size_t lds = (size_t)kLdsSortMax * sizeof(uint64_t);
    hipError_t e = allow_lds(prepass_long_kernel, lds);
    if (e != hipSuccess) return e;
    const int64_t grid = m < kSortSlots ? m : kSortSlots;
    hipLaunchKernelGGL(prepass_long_kernel, dim3((unsigned)grid), dim3(kLongThreads), lds, s, X, m,
                       (int)n, perm, rank, rstart, ld, n1_ws, n1_out, nruns, nlong, runs, status,
                       sort_tmp, doubled ? 1 : 0);
    return hipGetLastError();
  }
  int npow2 = 64;
  while (npow2 < n) npow2 <<= 1;
  const size_t lds = (size_t)npow2 * sizeof(uint64_t);
  // a row of 8192 or more keys holds 64 KB of LDS or more, so few of its
  // workgroups share a CU: give each the full 1024 threads
  if (npow2 >= 8192) {
    hipError_t e = allow_lds(prepass_kernel<kLongThreads>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(prepass_kernel<kLongThreads>, dim3((unsigned)m), dim3(kLongThreads), lds,
                       s, X, m, (int)n, npow2, perm, rank, rstart, ld, n1_ws, n1_out, nruns,
                       nlong, runs, status, doubled ? 1 : 0);
    return hipGetLastError();
  }
  hipError_t e = allow_lds(prepass_kernel<kThreads>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(prepass_kernel<kThreads>, dim3((unsigned)m), dim3(kThreads), lds, s, X, m,
                     (int)n, npow2, perm, rank, rstart, ld, n1_ws, n1_out, nruns, nlong, runs,
                     status, doubled ? 1 : 0);
  return hipGetLastError();
}

}  // namespace ktau
