// C ABI of libktau: argument checks, workspace layout and launches for the
// job mapper, the rank pre-pass and the plain all-pairs calls.
#include <stdlib.h>
#include <string.h>

#include "ktau_internal.h"

namespace ktau {
namespace {

__global__ void clear_status_kernel(int32_t* status) { *status = 0; }

struct WsLayout {
  size_t perm, rank, rstart, n1, total;
  int64_t ld;
};

WsLayout ws_layout(int64_t m, int64_t n) {
  WsLayout L;
  L.ld = round_up(n, kRowAlign);
  size_t rowbytes = (size_t)m * (size_t)L.ld * sizeof(uint16_t);
  size_t off = kWsHeader;
  L.perm = off;
  off = (size_t)round_up((int64_t)(off + rowbytes), (int64_t)kAlign);
  L.rank = off;
  off = (size_t)round_up((int64_t)(off + rowbytes), (int64_t)kAlign);
  L.rstart = off;
  off = (size_t)round_up((int64_t)(off + rowbytes), (int64_t)kAlign);
  L.n1 = off;
  off = (size_t)round_up((int64_t)(off + (size_t)m * sizeof(int64_t)), (int64_t)kAlign);
  L.total = off;
  return L;
}

int check_shape(int64_t m, int64_t n) {
  if (m < 2 || n < 2 || m > (int64_t)0x7fffffff) return KTAU_EINVAL;
  if (n > KTAU_MAX_N) return KTAU_ERANGE;
  return KTAU_OK;
}

int env_int(const char* name, int dflt) {
  const char* s = getenv(name);
  if (!s || !*s) return dflt;
  return atoi(s);
}

}  // namespace

// Shared by the batch and server units.
int run_prepass_into(const float* X, int64_t m, int64_t n, void* ws, RankView& rv,
                     int64_t* n1_out, int32_t*& status, hipStream_t s) {
  WsLayout L = ws_layout(m, n);
  char* base = (char*)ws;
  status = (int32_t*)base;
  uint16_t* perm = (uint16_t*)(base + L.perm);
  uint16_t* rank = (uint16_t*)(base + L.rank);
  uint16_t* rstart = (uint16_t*)(base + L.rstart);
  int64_t* n1 = (int64_t*)(base + L.n1);
  if (launch_prepass(X, m, n, perm, rank, rstart, L.ld, n1, n1_out, status, s) != hipSuccess)
    return KTAU_EDEVICE;
  rv.perm = perm;
  rv.rank = rank;
  rv.rstart = rstart;
  rv.n1 = n1;
  rv.ld = L.ld;
  return KTAU_OK;
}

size_t workspace_bytes(int64_t m, int64_t n) { return ws_layout(m, n).total; }

int clear_status(int32_t* status, hipStream_t s) {
  hipLaunchKernelGGL(clear_status_kernel, dim3(1), dim3(1), 0, s, status);
  return hipGetLastError() == hipSuccess ? KTAU_OK : KTAU_EDEVICE;
}

}  // namespace ktau

using namespace ktau;

extern "C" {

const char* ktau_status_string(int status) {
  switch (status) {
    case KTAU_OK: return "ok";
    case KTAU_EINVAL: return "invalid argument";
    case KTAU_ERANGE: return "out of range";
    case KTAU_ENOMEM: return "out of memory or workspace too small";
    case KTAU_EDEVICE: return "HIP runtime error";
    case KTAU_EBUSY: return "admission refused";
    case KTAU_ENAN: return "NaN in input";
    case KTAU_ECANCELED: return "request cancelled";
    case KTAU_ETIMEDOUT: return "timed out";
    default: return "unknown status";
  }
}

int64_t ktau_pair_to_job(int64_t m, int64_t y, int64_t x) {
  if (m < 2 || y < 0 || x <= y || x >= m) return -1;
  return strict_job(m, y, x);
}

int ktau_job_to_pair(int64_t m, int64_t J, int64_t* y, int64_t* x) {
  if (m < 2 || !y || !x) return KTAU_EINVAL;
  if (J < 0 || J >= m * (m - 1) / 2) return KTAU_ERANGE;
  strict_pair(m, J, *y, *x);
  return KTAU_OK;
}

int ktau_tile_to_coord(int64_t w, int64_t t, int64_t* yq, int64_t* xq) {
  if (w < 1 || !yq || !xq) return KTAU_EINVAL;
  if (t < 0 || t >= w * (w + 1) / 2) return KTAU_ERANGE;
  tile_coord(w, t, *yq, *xq);
  return KTAU_OK;
}

int ktau_rank(const float* X, int64_t m, int64_t n, uint16_t* perm, uint16_t* rank,
              uint16_t* rstart, int64_t* n1, int32_t* status, void* stream) {
  if (!X || !status || m < 1 || n < 1 || m > (int64_t)0x7fffffff) return KTAU_EINVAL;
  if (n > KTAU_MAX_N) return KTAU_ERANGE;
  hipError_t e = launch_prepass(X, m, n, perm, rank, rstart, n, nullptr, n1, status,
                                (hipStream_t)stream);
  return e == hipSuccess ? KTAU_OK : KTAU_EDEVICE;
}

size_t ktau_allpairs_workspace_size(int64_t m, int64_t n) {
  if (check_shape(m, n) != KTAU_OK) return 0;
  return workspace_bytes(m, n);
}

int ktau_scheme_count(void) { return kNumSchemes; }
const char* ktau_scheme_name(int scheme) { return scheme_name(scheme); }
int64_t ktau_scheme_capacity(int scheme) {
  return (scheme >= 0 && scheme < kNumSchemes) ? scheme_capacity(scheme) : -1;
}
int ktau_default_scheme(int64_t n) { return default_scheme(n); }

int ktau_allpairs_ex(const float* X, int64_t m, int64_t n, int64_t J_begin, int64_t J_end,
                     ktau_pair_out out, void* ws, size_t ws_bytes, int scheme, int q,
                     void* stream) {
  int rc = check_shape(m, n);
  if (rc != KTAU_OK) return rc;
  if (!X || !ws) return KTAU_EINVAL;
  if (((uintptr_t)ws) % kAlign != 0) return KTAU_EINVAL;
  const int64_t P = m * (m - 1) / 2;
  const bool full = J_begin < 0;
  if (full) {
    J_begin = 0;
    J_end = P;
  }
  if (J_begin > J_end || J_end > P) return KTAU_ERANGE;
  if (ws_bytes < workspace_bytes(m, n)) return KTAU_ENOMEM;
  if (scheme < 0) scheme = env_int("KTAU_FORCE_SCHEME", default_scheme(n));
  if (scheme < 0 || scheme >= kNumSchemes || scheme_capacity(scheme) < n) return KTAU_EINVAL;
  if (q <= 0) q = env_int("KTAU_TILE_Q", 8);
  if (q < 1 || q > 64) return KTAU_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  RankView rv;
  int32_t* status = nullptr;
  if (clear_status((int32_t*)ws, s) != KTAU_OK) return KTAU_EDEVICE;
  rc = run_prepass_into(X, m, n, ws, rv, out.n1, status, s);
  if (rc != KTAU_OK) return rc;
  PairOut po{out.nc, out.nd, out.n3, out.tau_b, out.tau_a};
  hipError_t e;
  if (full) {
    const int64_t w = (m + q - 1) / q;
    e = launch_pairs_tiles(scheme, rv, m, (int)n, q, w, 0, w * (w + 1) / 2, po, status, s);
  } else {
    e = launch_pairs_jobs(scheme, rv, m, (int)n, J_begin, J_end, po, status, s);
  }
  return e == hipSuccess ? KTAU_OK : KTAU_EDEVICE;
}

int ktau_allpairs(const float* X, int64_t m, int64_t n, ktau_pair_out out, void* ws,
                  size_t ws_bytes, void* stream) {
  return ktau_allpairs_ex(X, m, n, -1, -1, out, ws, ws_bytes, -1, 0, stream);
}

int ktau_allpairs_range(const float* X, int64_t m, int64_t n, int64_t J_begin, int64_t J_end,
                        ktau_pair_out out, void* ws, size_t ws_bytes, void* stream) {
  if (J_begin < 0) return KTAU_ERANGE;
  return ktau_allpairs_ex(X, m, n, J_begin, J_end, out, ws, ws_bytes, -1, 0, stream);
}

int ktau_status(void* ws, void* stream) {
  if (!ws) return KTAU_EINVAL;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return KTAU_EDEVICE;
  int32_t st = 0;
  if (hipMemcpy(&st, ws, sizeof(st), hipMemcpyDeviceToHost) != hipSuccess) return KTAU_EDEVICE;
  if (st != 0) {
    int32_t zero = 0;
    if (hipMemcpy(ws, &zero, sizeof(zero), hipMemcpyHostToDevice) != hipSuccess)
      return KTAU_EDEVICE;
  }
  return st;
}

}  // extern "C"
