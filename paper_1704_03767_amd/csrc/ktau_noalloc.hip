// All-pairs without any device allocation: the plain path of ktau_allpairs
// with its workspace in a fixed static device array instead of caller memory,
// for callers that cannot allocate (code under graph capture, serving loops,
// harnesses that forbid allocation).
//
// The array lives in the library's code object, one copy per GPU, for the
// life of the process.  Its device address is looked up once per device with
// hipGetSymbolAddress (on the first call made with that device current) and
// only that address is handed to kernels and copies.  Every call on a GPU
// shares that GPU's array: calls that overlap on one GPU race.  The call
// itself clears what must start at zero (the status words) with a kernel.
#include <mutex>

#include "ktau_internal.h"

namespace {

constexpr size_t kNoAllocBytes = (size_t)64 << 20;   // 64 MiB
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// This device's copy of the array (looked up on first use); nullptr if the
// lookup fails.
void* device_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_scratch[dev] = p;
  }
  return g_scratch[dev];
}

// status_dev[0] = the latched status word of the scratch header, which is
// then cleared for the next call.
__global__ void take_status_kernel(int32_t* ws_status, int32_t* status_dev) {
  if (threadIdx.x == 0) {
    *status_dev = *ws_status;
    *ws_status = 0;
  }
}

}  // namespace

extern "C" {

int ktau_allpairs_noalloc(const float* X, int64_t m, int64_t n, ktau_pair_out out,
                          int32_t* status_dev, void* stream) {
  int rc = ktau::check_shape(m, n);
  if (rc != KTAU_OK) return rc;
  if (!X) return KTAU_EINVAL;
  if (ktau_allpairs_workspace_size(m, n) > kNoAllocBytes) return KTAU_ENOMEM;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return KTAU_EDEVICE;
  void* ws = device_scratch(dev);
  if (!ws) return KTAU_EDEVICE;
  rc = ktau_allpairs(X, m, n, out, ws, kNoAllocBytes, stream);
  if (rc != KTAU_OK || !status_dev) return rc;
  hipLaunchKernelGGL(take_status_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream,
                     (int32_t*)ws, status_dev);
  return hipGetLastError() == hipSuccess ? KTAU_OK : KTAU_EDEVICE;
}

}  // extern "C"
