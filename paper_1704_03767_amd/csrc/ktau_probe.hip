// Measured denominators for the rooflines: two small kernels whose work per
// launch is known exactly, timed by the caller.
//
// VALU: every lane keeps 16 independent 32-bit sums and adds its neighbour
// to each, 16 v_add_u32 per iteration, with the loop counter in scalar
// registers; the result is stored so that nothing is removed.
// LDS: every lane reads 16 x 16 bytes per iteration (ds_read_b128) from
// consecutive 16-byte slots of a 64 KB buffer, so a wave's 1024 bytes per
// read fall on all banks without conflicts; the reads are xor-folded and
// stored, and an empty compiler barrier per iteration keeps them in the loop.
#include "ktau_internal.h"

namespace ktau {
namespace {

constexpr int kProbeThreads = 256;
constexpr int kProbeChains = 16;
constexpr int kLdsProbeWords = 16384;   // 64 KB
constexpr int kLdsProbeReads = 16;      // 16-byte reads per lane per iteration

__global__ void __launch_bounds__(kProbeThreads) probe_valu_kernel(uint32_t* out, int iters,
                                                                   uint32_t seed) {
  uint32_t a[kProbeChains];
#pragma unroll
  for (int k = 0; k < kProbeChains; ++k) a[k] = seed + threadIdx.x * 31u + (uint32_t)k;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < kProbeChains; ++k) a[k] += a[(k + 1) % kProbeChains];
  }
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kProbeChains; ++k) s ^= a[k];
  out[(int64_t)blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

__global__ void __launch_bounds__(kProbeThreads) probe_lds_kernel(uint32_t* out, int iters,
                                                                  uint32_t seed) {
  __shared__ uint4 buf[kLdsProbeWords / 4];
  for (int i = threadIdx.x; i < kLdsProbeWords / 4; i += kProbeThreads)
    buf[i] = make_uint4(seed + i, seed ^ i, seed + 3 * i, i);
  __syncthreads();
  // wave w reads the 1 KB windows w*64 + 256 j (j = 0..15) of 64 slots
  const uint4* p = buf + (threadIdx.x >> 6) * 64 + (threadIdx.x & 63);
  uint32_t acc0 = 0, acc1 = 0;
  for (int i = 0; i < iters; ++i) {
    __asm__ volatile("" ::: "memory");
#pragma unroll
    for (int j = 0; j < kLdsProbeReads; ++j) {
      const uint4 v = p[j * 256];
      acc0 ^= v.x ^ v.y ^ v.z;
      acc1 ^= v.w;
    }
  }
  out[(int64_t)blockIdx.x * kProbeThreads + threadIdx.x] = acc0 ^ acc1;
}

}  // namespace
}  // namespace ktau

using namespace ktau;

extern "C" {

int ktau_probe_threads(void) { return kProbeThreads; }
int ktau_probe_valu_ops_per_iter(void) { return kProbeChains; }
int ktau_probe_lds_bytes_per_iter(void) { return kLdsProbeReads * 16; }

int ktau_probe_valu(uint32_t* out, int64_t blocks, int iters, void* stream) {
  if (!out || blocks < 1 || blocks > 0x7fffffff || iters < 1) return KTAU_EINVAL;
  hipLaunchKernelGGL(probe_valu_kernel, dim3((unsigned)blocks), dim3(kProbeThreads), 0,
                     (hipStream_t)stream, out, iters, 0x9E3779B9u);
  return hipGetLastError() == hipSuccess ? KTAU_OK : KTAU_EDEVICE;
}

int ktau_probe_lds(uint32_t* out, int64_t blocks, int iters, void* stream) {
  if (!out || blocks < 1 || blocks > 0x7fffffff || iters < 1) return KTAU_EINVAL;
  hipLaunchKernelGGL(probe_lds_kernel, dim3((unsigned)blocks), dim3(kProbeThreads), 0,
                     (hipStream_t)stream, out, iters, 0x85EBCA6Bu);
  return hipGetLastError() == hipSuccess ? KTAU_OK : KTAU_EDEVICE;
}

}  // extern "C"
