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
// sample), then block scans produce dense ranks and run starts.  Into a pair
// workspace the sample indices and ranks are written doubled (byte offsets
// into a rank row, and ranks with a free low bit for the pair network's
// tag); the rank entry point writes them plain.
#include "ktau_internal.h"

namespace ktau {
namespace {

constexpr int kThreads = 256;

// Order-preserving map float32 -> uint32 with -0.0 folded onto +0.0 (IEEE
// equality decides ties).  NaN never reaches a comparison: it is flagged.
__device__ inline uint32_t float_key(float f, bool& nan) {
  uint32_t b = __float_as_uint(f);
  nan = (b & 0x7fffffffu) > 0x7f800000u;
  if (b == 0x80000000u) b = 0u;
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// Block-wide exclusive scan (sum) of one int per thread; also returns the total.
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
  for (int w = 0; w < kThreads / 64; ++w) {
    int s = sh[w];
    if (w < wave) base += s;
    tot += s;
  }
  __syncthreads();
  total = tot;
  return base + incl - v;
}

// Block-wide exclusive scan (max) of one non-negative int per thread.
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
  for (int w = 0; w < kThreads / 64; ++w)
    if (w < wave) base = max(base, sh[w]);
  __syncthreads();
  return max(base, excl_in_wave);
}

// Ranks row `row` of one matrix; s_keys holds npow2 64-bit words.
__device__ void prepass_row(const float* __restrict__ X, int64_t row, int n, int npow2,
                            uint16_t* __restrict__ perm, uint16_t* __restrict__ rank,
                            uint16_t* __restrict__ rstart, int64_t ld,
                            int64_t* __restrict__ n1_ws, int64_t* __restrict__ n1_out,
                            int32_t* __restrict__ nruns, uint64_t* __restrict__ runs,
                            int32_t* __restrict__ status, uint64_t* s_keys, int dbl) {
  __shared__ int s_scan[kThreads / 64];
  __shared__ unsigned long long s_n1;
  const float* x = X + row * (int64_t)n;
  const int tid = threadIdx.x;

  bool any_nan = false;
  for (int i = tid; i < npow2; i += kThreads) {
    uint64_t w = ~0ull;
    if (i < n) {
      bool nan;
      uint32_t k = float_key(x[i], nan);
      any_nan |= nan;
      w = ((uint64_t)k << 16) | (uint64_t)i;
    }
    s_keys[i] = w;
  }
  if (tid == 0) s_n1 = 0;
  if (__syncthreads_or(any_nan)) {
    if (tid == 0) atomicExch(status, KTAU_ENAN);
    return;
  }

  // Bitonic sort of npow2 64-bit words, ascending.
  for (int k = 2; k <= npow2; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = tid; i < npow2; i += kThreads) {
        int p = i ^ j;
        if (p > i) {
          uint64_t a = s_keys[i], b = s_keys[p];
          bool up = (i & k) == 0;
          if ((a > b) == up) {
            s_keys[i] = b;
            s_keys[p] = a;
          }
        }
      }
      __syncthreads();
    }
  }

  // Each thread owns `chunk` consecutive sorted positions.
  const int chunk = npow2 / kThreads > 0 ? npow2 / kThreads : 1;
  const int k0 = tid * chunk;
  // Pass 1: count value changes (for dense ranks) and the last run start.
  int changes = 0, last_start = 0;
  for (int c = 0; c < chunk; ++c) {
    int k = k0 + c;
    if (k < n && k > 0 && (s_keys[k] >> 16) != (s_keys[k - 1] >> 16)) {
      ++changes;
      last_start = k;
    }
  }
  int total_changes;
  int rank_base = block_excl_sum(changes, s_scan, total_changes);
  int start_base = block_excl_max(last_start, s_scan);
  // Pass 2: write perm, rank and rstart; accumulate n1.
  uint16_t* prow = perm ? perm + row * ld : nullptr;
  uint16_t* rrow = rank ? rank + row * ld : nullptr;
  uint16_t* srow = rstart ? rstart + row * ld : nullptr;
  int r = rank_base, st = start_base;
  unsigned long long ties = 0;
  for (int c = 0; c < chunk; ++c) {
    int k = k0 + c;
    if (k < n) {
      uint64_t w = s_keys[k];
      int sample = (int)(w & 0xFFFFu);
      if (k > 0 && (w >> 16) != (s_keys[k - 1] >> 16)) {
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
  // Padding of rows longer than the sort width (ld > npow2 never happens for
  // the workspace layout, but callers may pass a wider ld).
  for (int k = npow2 + tid; k < ld; k += kThreads) {
    if (prow) prow[k] = (uint16_t)(k << dbl);
    if (srow) srow[k] = (uint16_t)k;
  }
  // Tail positions n..ld-1 map to themselves and rank 0x7FFF (doubled in a
  // workspace), above every real rank, so the pair kernels gather padding
  // keys without a bounds test.
  if (rrow)
    for (int i = n + tid; i < ld; i += kThreads) rrow[i] = (uint16_t)(0x7FFF << dbl);
  atomicAdd(&s_n1, ties);
  __syncthreads();
  if (tid == 0) {
    if (n1_ws) n1_ws[row] = (int64_t)s_n1;
    if (n1_out) n1_out[row] = (int64_t)s_n1;
  }
  if (!runs) return;
  // Pass 3: tie runs of length >= 2, in sorted order.  A thread owns the runs
  // that start in its chunk; block scans give their index and the number of
  // within-run pairs of all earlier runs.
  auto key_at = [&](int k) { return s_keys[k] >> 16; };
  int my_runs = 0, my_pairs = 0;
  for (int c = 0; c < chunk; ++c) {
    const int k = k0 + c;
    if (k + 1 < n && (k == 0 || key_at(k) != key_at(k - 1)) && key_at(k + 1) == key_at(k)) {
      int e = k + 2;
      while (e < n && key_at(e) == key_at(k)) ++e;
      ++my_runs;
      my_pairs += (e - k) * (e - k - 1) / 2;
    }
  }
  int total_runs, total_pairs;
  int run_idx = block_excl_sum(my_runs, s_scan, total_runs);
  int pairs = block_excl_sum(my_pairs, s_scan, total_pairs);
  uint64_t* rrow_runs = runs + row * (ld / 2);
  for (int c = 0; c < chunk && my_runs > 0; ++c) {
    const int k = k0 + c;
    if (k + 1 < n && (k == 0 || key_at(k) != key_at(k - 1)) && key_at(k + 1) == key_at(k)) {
      int e = k + 2;
      while (e < n && key_at(e) == key_at(k)) ++e;
      const int len = e - k;
      rrow_runs[run_idx++] =
          ((uint64_t)(uint32_t)pairs << 32) | ((uint64_t)len << 16) | (uint64_t)k;
      pairs += len * (len - 1) / 2;
    }
  }
  if (tid == 0 && nruns) nruns[row] = total_runs;
}

__global__ void __launch_bounds__(kThreads)
prepass_kernel(const float* __restrict__ X, int64_t m, int n, int npow2,
               uint16_t* __restrict__ perm, uint16_t* __restrict__ rank,
               uint16_t* __restrict__ rstart, int64_t ld, int64_t* __restrict__ n1_ws,
               int64_t* __restrict__ n1_out, int32_t* __restrict__ nruns,
               uint64_t* __restrict__ runs, int32_t* __restrict__ status, int dbl) {
  extern __shared__ uint64_t s_keys[];
  const int64_t row = blockIdx.x;
  if (row >= m) return;
  prepass_row(X, row, n, npow2, perm, rank, rstart, ld, n1_ws, n1_out, nruns, runs, status,
              s_keys, dbl);
}

// Every row of every matrix of a batch: block b ranks global row b, found by
// binary search on the per-matrix row prefix.
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
  const int64_t row = g - row_prefix[lo];
  int npow2 = 64;
  while (npow2 < d.n) npow2 <<= 1;
  prepass_row(d.X, row, d.n, npow2, (uint16_t*)d.rv.perm, (uint16_t*)d.rv.rank,
              (uint16_t*)d.rv.rstart, d.rv.ld, (int64_t*)d.rv.n1, d.n1_out,
              (int32_t*)d.rv.nruns, (uint64_t*)d.rv.runs, (int32_t*)d.status, s_keys, 1);
}

// Rows longer than 8192 samples sort 128 KB of keys, above the 64 KB of
// dynamic LDS a launch gets by default; raise the kernel's limit once.
template <typename F>
hipError_t allow_lds(F kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace

hipError_t launch_prepass_batch(const MatDesc* descs_dev, int64_t count, int64_t total_rows,
                                const int64_t* row_prefix_dev, int max_n, hipStream_t s) {
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
                          int32_t* nruns, uint64_t* runs, int32_t* status, bool doubled,
                          hipStream_t s) {
  int npow2 = 64;
  while (npow2 < n) npow2 <<= 1;
  const size_t lds = (size_t)npow2 * sizeof(uint64_t);
  hipError_t e = allow_lds(prepass_kernel, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(prepass_kernel, dim3((unsigned)m), dim3(kThreads), lds, s, X, m, (int)n,
                     npow2, perm, rank, rstart, ld, n1_ws, n1_out, nruns, runs, status,
                     doubled ? 1 : 0);
  return hipGetLastError();
}

}  // namespace ktau
