// C ABI of libktau, plain path: argument checks, workspace layout, and the
// launches for the job mapper, the rank pre-pass and the all-pairs calls.
#include <stdlib.h>
#include <string.h>

#include "ktau_internal.h"

namespace ktau {

namespace {
__global__ void clear_words_kernel(int32_t* p, int count) {
  for (int i = threadIdx.x; i < count; i += blockDim.x) p[i] = 0;
}
}  // namespace

WsLayout ws_layout(int64_t m, int64_t n) {
  WsLayout L;
  L.ld = row_ld(n);
  const int64_t rowbytes = m * L.ld * (int64_t)sizeof(uint16_t);
  int64_t off = (int64_t)kWsHeader;
  L.perm = (size_t)off;
  off = round_up(off + rowbytes, (int64_t)kAlign);
  L.rank = (size_t)off;
  off = round_up(off + rowbytes, (int64_t)kAlign);
  L.rstart = (size_t)off;
  off = round_up(off + rowbytes, (int64_t)kAlign);
  L.n1 = (size_t)off;
  off = round_up(off + m * (int64_t)sizeof(int64_t), (int64_t)kAlign);
  L.nruns = (size_t)off;
  off = round_up(off + m * (int64_t)sizeof(int32_t), (int64_t)kAlign);
  L.nlong = (size_t)off;
  off = round_up(off + m * (int64_t)sizeof(int32_t), (int64_t)kAlign);
  L.runs = (size_t)off;
  off = round_up(off + m * (L.ld / 2) * (int64_t)sizeof(uint64_t), (int64_t)kAlign);
  L.heavy = (size_t)off;
  off = round_up(off + m * (int64_t)sizeof(int32_t), (int64_t)kAlign);
  L.sort = (size_t)off;
  off = round_up(off + (int64_t)sort_scratch_bytes(m, n), (int64_t)kAlign);
  L.total = (size_t)off;
  return L;
}

int check_shape(int64_t m, int64_t n) {
  if (m < 2 || n < 2 || m > (int64_t)0x7fffffff) return KTAU_EINVAL;
  if (n > KTAU_MAX_N) return KTAU_ERANGE;
  return KTAU_OK;
}

MatDesc matdesc(void* ws, int64_t m, int64_t n, const ktau_pair_out& out, int scheme, int q,
                int64_t J_begin, int64_t J_end, int32_t* status) {
  const WsLayout L = ws_layout(m, n);
  char* base = (char*)ws;
  MatDesc d;
  memset(&d, 0, sizeof(d));
  d.rv.perm = (const uint16_t*)(base + L.perm);
  d.rv.rank = (const uint16_t*)(base + L.rank);
  d.rv.rstart = (const uint16_t*)(base + L.rstart);
  d.rv.n1 = (const int64_t*)(base + L.n1);
  d.rv.nruns = (const int32_t*)(base + L.nruns);
  d.rv.nlong = (const int32_t*)(base + L.nlong);
  d.rv.runs = (const uint64_t*)(base + L.runs);
  d.rv.ld = L.ld;
  d.out = PairOut{out.nc, out.nd, out.n3, out.tau_b, out.tau_a};
  d.status = status ? status : (const int32_t*)base;
  d.heavy_count = (int32_t*)(base + 4);
  d.heavy = (int32_t*)(base + L.heavy);
  d.sort_tmp = (uint64_t*)(base + L.sort);
  d.m = m;
  d.n = (int32_t)n;
  d.scheme = scheme;
  d.q = q;
  d.w = (m + q - 1) / q;
  d.n_units = d.w * (d.w + 1) / 2;
  d.unit_begin = 0;
  d.J_begin = J_begin;
  d.J_end = J_end;
  return d;
}

int prepass_ws(const float* X, int64_t m, int64_t n, void* ws, int64_t* n1_out, int32_t* status,
               hipStream_t s) {
  const WsLayout L = ws_layout(m, n);
  char* base = (char*)ws;
  if (launch_prepass(X, m, n, (uint16_t*)(base + L.perm), (uint16_t*)(base + L.rank),
                     (uint16_t*)(base + L.rstart), L.ld, (int64_t*)(base + L.n1), n1_out,
                     (int32_t*)(base + L.nruns), (int32_t*)(base + L.nlong),
                     (uint64_t*)(base + L.runs),
                     status ? status : (int32_t*)base, ws_doubled(n), (uint64_t*)(base + L.sort),
                     s) != hipSuccess)
    return KTAU_EDEVICE;
  return KTAU_OK;
}

int clear_words(int32_t* p, int count, hipStream_t s) {
  hipLaunchKernelGGL(clear_words_kernel, dim3(1), dim3(64), 0, s, p, count);
  return hipGetLastError() == hipSuccess ? KTAU_OK : KTAU_EDEVICE;
}

namespace {

// Largest n for which the plain calls pick the naive bit-set count by
// default: measured faster than the network schemes up to n = 128 (5x at
// n = 32, 2.7x at 64, 1.1x at 128, 0.5x at 256 on 4096 rows).
constexpr int64_t kBitsDefaultMaxN = 128;

int plain_default_scheme(int64_t n) {
  return n <= kBitsDefaultMaxN ? KTAU_SCHEME_NAIVE : default_scheme(n);
}

// The plain workspace: the shared layout, then the bit sets (short rows).
size_t plain_ws_bytes(int64_t m, int64_t n) { return ws_layout(m, n).total + bits_bytes(m, n); }
uint32_t* plain_bits(void* ws, int64_t m, int64_t n) {
  return (uint32_t*)((char*)ws + ws_layout(m, n).total);
}

int check_ws(int64_t m, int64_t n, const void* ws, size_t ws_bytes) {
  const int rc = check_shape(m, n);
  if (rc != KTAU_OK) return rc;
  if (!ws || ((uintptr_t)ws) % kAlign != 0) return KTAU_EINVAL;
  if (ws_bytes < plain_ws_bytes(m, n)) return KTAU_ENOMEM;
  return KTAU_OK;
}

// Validates a job range and the launch options; J_begin < 0 means all jobs.
int check_pairs(int64_t m, int64_t n, int64_t& J_begin, int64_t& J_end, int& scheme, int& q,
                bool& full) {
  const int64_t P = m * (m - 1) / 2;
  full = J_begin < 0;
  if (full) {
    J_begin = 0;
    J_end = P;
  }
  if (J_begin > J_end || J_end > P) return KTAU_ERANGE;
  if (scheme < 0) scheme = plain_default_scheme(n);
  if (scheme == KTAU_SCHEME_NAIVE) {
    if (n > kBitsMaxN) return KTAU_EINVAL;
  } else if (scheme < 0 || scheme >= kNumSchemes || scheme_capacity(scheme) < n) {
    return KTAU_EINVAL;
  }
  if (q <= 0) q = scheme == KTAU_SCHEME_NAIVE ? kBitsQ : (int)plain_q(m, n);
  if (q < 1 || q > 64) return KTAU_EINVAL;
  return KTAU_OK;
}

}  // namespace
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

size_t ktau_rank_workspace_size(int64_t m, int64_t n) {
  if (m < 1 || n < 1 || n > KTAU_MAX_N) return 0;
  return sort_scratch_bytes(m, n);
}

int ktau_rank(const float* X, int64_t m, int64_t n, uint16_t* perm, uint16_t* rank,
              uint16_t* rstart, int64_t* n1, int32_t* status, void* ws, size_t ws_bytes,
              void* stream) {
  if (!X || !status || m < 1 || n < 1 || m > (int64_t)0x7fffffff) return KTAU_EINVAL;
  if (n > KTAU_MAX_N) return KTAU_ERANGE;
  const size_t need = sort_scratch_bytes(m, n);
  if (need > 0 && (!ws || ((uintptr_t)ws) % kAlign != 0)) return KTAU_EINVAL;
  if (ws_bytes < need) return KTAU_ENOMEM;
  const hipError_t e = launch_prepass(X, m, n, perm, rank, rstart, n, nullptr, n1, nullptr,
                                      nullptr, nullptr, status, false, (uint64_t*)ws,
                                      (hipStream_t)stream);
  return e == hipSuccess ? KTAU_OK : KTAU_EDEVICE;
}

size_t ktau_allpairs_workspace_size(int64_t m, int64_t n) {
  if (check_shape(m, n) != KTAU_OK) return 0;
  return plain_ws_bytes(m, n);
}

int ktau_scheme_count(void) { return kNumSchemes; }
const char* ktau_scheme_name(int scheme) {
  return scheme == KTAU_SCHEME_NAIVE ? "invalid" : scheme_name(scheme);
}
int64_t ktau_scheme_capacity(int scheme) {
  return (scheme >= 0 && scheme < kNumSchemes) ? scheme_capacity(scheme) : -1;
}
int ktau_default_scheme(int64_t n) { return default_scheme(n); }
int ktau_plain_default_scheme(int64_t n) { return plain_default_scheme(n); }
int ktau_plain_default_q(int64_t m, int64_t n) {
  return plain_default_scheme(n) == KTAU_SCHEME_NAIVE ? kBitsQ : (int)plain_q(m, n);
}

int ktau_prepare(const float* X, int64_t m, int64_t n, int64_t* out_n1, void* ws,
                 size_t ws_bytes, void* stream) {
  int rc = check_ws(m, n, ws, ws_bytes);
  if (rc != KTAU_OK) return rc;
  if (!X) return KTAU_EINVAL;
  const hipStream_t s = (hipStream_t)stream;
  if (clear_words((int32_t*)ws, 2, s) != KTAU_OK) return KTAU_EDEVICE;
  rc = prepass_ws(X, m, n, ws, out_n1, nullptr, s);
  if (rc != KTAU_OK || n > kBitsMaxN) return rc;
  const MatDesc d = matdesc(ws, m, n, ktau_pair_out{}, 0, 1, 0, 0, nullptr);
  return launch_bits_prepass(d, plain_bits(ws, m, n), s) == hipSuccess ? KTAU_OK : KTAU_EDEVICE;
}

int ktau_pairs(int64_t m, int64_t n, int64_t J_begin, int64_t J_end, ktau_pair_out out,
               void* ws, size_t ws_bytes, int scheme, int q, void* stream) {
  int rc = check_ws(m, n, ws, ws_bytes);
  if (rc != KTAU_OK) return rc;
  bool full;
  rc = check_pairs(m, n, J_begin, J_end, scheme, q, full);
  if (rc != KTAU_OK) return rc;
  const MatDesc d = matdesc(ws, m, n, out, scheme, q, J_begin, J_end, nullptr);
  const hipError_t e = scheme == KTAU_SCHEME_NAIVE
                           ? launch_bits_pairs(d, plain_bits(ws, m, n), full, (hipStream_t)stream)
                           : launch_pairs_plain(d, full, (hipStream_t)stream);
  return e == hipSuccess ? KTAU_OK : KTAU_EDEVICE;
}

int ktau_allpairs_ex(const float* X, int64_t m, int64_t n, int64_t J_begin, int64_t J_end,
                     ktau_pair_out out, void* ws, size_t ws_bytes, int scheme, int q,
                     void* stream) {
  int rc = check_ws(m, n, ws, ws_bytes);
  if (rc != KTAU_OK) return rc;
  if (!X) return KTAU_EINVAL;
  bool full;
  rc = check_pairs(m, n, J_begin, J_end, scheme, q, full);
  if (rc != KTAU_OK) return rc;
  rc = ktau_prepare(X, m, n, out.n1, ws, ws_bytes, stream);
  if (rc != KTAU_OK) return rc;
  return ktau_pairs(m, n, full ? -1 : J_begin, J_end, out, ws, ws_bytes, scheme, q, stream);
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
    const int32_t zero = 0;
    if (hipMemcpy(ws, &zero, sizeof(zero), hipMemcpyHostToDevice) != hipSuccess)
      return KTAU_EDEVICE;
  }
  return st;
}

}  // extern "C"
