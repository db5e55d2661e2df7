// Measured denominators for the rooflines: two small kernels whose work per
// launch is known exactly, timed by the caller.
//
// VALU: every lane keeps 16 independent 32-bit sums and adds its neighbour
// to each, 16 v_add_u32 per iteration, with the loop counter in scalar
// registers; the result is stored so that nothing is removed.
// Issue rates: the same 16 independent chains per lane with one instruction
// kind each (the kinds the pair kernels are made of): int32 add, packed f16
// minimum with a negated operand (v_pk_minimum3_f16), unsigned 16-bit dot
// product with accumulate (v_dot2_u32_u16), packed u16 minimum and add
// (v_pk_min_u16, v_pk_add_u16: two instructions per chain).
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

typedef _Float16 probe_h2 __attribute__((ext_vector_type(2)));
typedef unsigned short probe_u2 __attribute__((ext_vector_type(2)));

template <int kKind>
__global__ void __launch_bounds__(kProbeThreads) probe_issue_kernel(uint32_t* out, int iters,
                                                                    uint32_t seed) {
  uint32_t a[kProbeChains];
#pragma unroll
  for (int k = 0; k < kProbeChains; ++k)
    a[k] = kKind == 1 ? ((seed + threadIdx.x + (uint32_t)k) & 0x03FFu) * 0x00010001u + 0x3C003C00u
                      : seed + threadIdx.x * 31u + (uint32_t)k;
  const probe_u2 w = {(unsigned short)threadIdx.x, (unsigned short)3};
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < kProbeChains; ++k) {
      const uint32_t b = a[(k + 1) % kProbeChains];
      if constexpr (kKind == 1) {
        a[k] = __builtin_bit_cast(
            uint32_t, __builtin_elementwise_minimum(__builtin_bit_cast(probe_h2, a[k]),
                                                    -__builtin_bit_cast(probe_h2, b)));
      } else if constexpr (kKind == 2) {
        a[k] = __builtin_amdgcn_udot2(__builtin_bit_cast(probe_u2, b), w, a[k], false);
      } else if constexpr (kKind == 3) {
        const probe_u2 x = __builtin_bit_cast(probe_u2, a[k]);
        a[k] = __builtin_bit_cast(uint32_t,
                                  __builtin_elementwise_min(x, __builtin_bit_cast(probe_u2, b) + x));
      } else {
        a[k] += b;
      }
    }
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

int ktau_probe_issue_instrs_per_iter(int kind) {
  return kind == 3 ? 2 * kProbeChains : (kind >= 0 && kind < 3 ? kProbeChains : -1);
}

int ktau_probe_issue(uint32_t* out, int64_t blocks, int iters, int kind, void* stream) {
  if (!out || blocks < 1 || blocks > 0x7fffffff || iters < 1 || kind < 0 || kind > 3)
    return KTAU_EINVAL;
  const dim3 g((unsigned)blocks), b(kProbeThreads);
  hipStream_t s = (hipStream_t)stream;
  switch (kind) {
    case 0: hipLaunchKernelGGL(probe_issue_kernel<0>, g, b, 0, s, out, iters, 0x9E3779B9u); break;
    case 1: hipLaunchKernelGGL(probe_issue_kernel<1>, g, b, 0, s, out, iters, 0x9E3779B9u); break;
    case 2: hipLaunchKernelGGL(probe_issue_kernel<2>, g, b, 0, s, out, iters, 0x9E3779B9u); break;
    default: hipLaunchKernelGGL(probe_issue_kernel<3>, g, b, 0, s, out, iters, 0x9E3779B9u); break;
  }
  return hipGetLastError() == hipSuccess ? KTAU_OK : KTAU_EDEVICE;
}

int ktau_probe_lds(uint32_t* out, int64_t blocks, int iters, void* stream) {
  if (!out || blocks < 1 || blocks > 0x7fffffff || iters < 1) return KTAU_EINVAL;
  hipLaunchKernelGGL(probe_lds_kernel, dim3((unsigned)blocks), dim3(kProbeThreads), 0,
                     (hipStream_t)stream, out, iters, 0x85EBCA6Bu);
  return hipGetLastError() == hipSuccess ? KTAU_OK : KTAU_EDEVICE;
}

}  // extern "C"
