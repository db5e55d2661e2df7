// Permutation-test P-values (Sec. 1: the significance of a pair's tau by a
// permutation test needs many tau of the same pair).  For every strict pair
// (y, x) and each of B caller-given permutations pi of the samples, the pair
// is counted again with x's samples permuted (x'[t] = x[pi[t]]); the output is
// the number of permutations whose |n_c - n_d| is at least the observed one
// and the P-value (1 + count) / (B + 1).  The tie terms n1 and n2 of tau_B do
// not change when one row's samples are permuted, so |tau_B| orders the
// permutations exactly as the integer |n_c - n_d| does.
//
// One group of lanes per pair, as in all-pairs: x's rank row is staged in
// LDS once, y's sorted order is loaded once, and each permutation rebuilds a
// second LDS row (slot t gets rank_x[pi[t]]) before the usual gather, direct
// in-run tie count and network count.  Every pair takes the direct tie count
// (no composite pass), which is exact for any ties; its cost follows the
// tie term of the row whose order is used, so when x has fewer ties the
// roles turn: permuting both rows' samples by pi^-1 leaves n_c - n_d alone,
// so |n_c - n_d| of (y, x o pi) is that of (x, y o pi^-1).
#include "ktau_pairdev.h"

namespace ktau {
namespace {

// Per group: x's rank row, the permuted row, and the network's cross-wave
// exchange buffer for 256-lane groups; then the block's reduction words.
template <int K, int G>
struct PermLds {
  static constexpr int kRowWords = K * G / 2;
  static constexpr int kXWords = G == 256 ? bitonic::Net<K, G>::kXChunk * 256 : 0;
  static constexpr int kWords = 2 * kRowWords + kXWords;
  static constexpr int kGroups = kBlock / G;
  static constexpr int kBlockWords = kGroups * kWords + 8;
};

// Checks that each of the B rows of perms (n entries, row stride n) is a
// permutation of 0..n-1 (else latches KTAU_EINVAL) and writes it, and its
// inverse, as byte offsets into a rank row (2 pi[t], 2 pi^-1[t]) to pad and
// inv, row stride ld, identity past n.
__global__ void __launch_bounds__(256)
perm_check_kernel(const uint16_t* __restrict__ perms, int n, int64_t ld,
                  uint16_t* __restrict__ pad, uint16_t* __restrict__ inv,
                  int32_t* __restrict__ status) {
  extern __shared__ uint32_t seen[];   // n bits
  const int64_t b = blockIdx.x;
  const int words = (n + 31) / 32;
  for (int i = threadIdx.x; i < words; i += blockDim.x) seen[i] = 0;
  __syncthreads();
  bool bad = false;
  for (int t = threadIdx.x; t < n; t += blockDim.x) {
    const uint32_t v = perms[b * n + t];
    if (v >= (uint32_t)n) {
      bad = true;
      pad[b * ld + t] = (uint16_t)(2 * t);
      continue;
    }
    const uint32_t bit = 1u << (v & 31u);
    if (atomicOr(&seen[v >> 5], bit) & bit) bad = true;
    pad[b * ld + t] = (uint16_t)(2 * v);
    inv[b * ld + v] = (uint16_t)(2 * t);   // a permutation writes every slot once
  }
  for (int64_t t = n + threadIdx.x; t < ld; t += blockDim.x) {
    pad[b * ld + t] = (uint16_t)(2 * t);
    inv[b * ld + t] = (uint16_t)(2 * t);
  }
  if (__syncthreads_or(bad) && threadIdx.x == 0) atomicExch(status, KTAU_EINVAL);
}

struct PermDesc {
  RankView rv;
  const uint16_t* pad;     // [B][ld] permutations as byte offsets
  const uint16_t* inv;     // [B][ld] their inverses
  int64_t B;
  int64_t* count_out;      // [J_end - J_begin]
  double* p_out;           // [J_end - J_begin] or NULL
  const int32_t* status;
  int64_t m;
  int32_t n;
  int64_t J_begin, J_end;
};

// The permutation test of pair (y, x); every lane of the group calls it.
template <int K, int G>
__device__ __forceinline__ int64_t pair_perm(const PermDesc& d, int64_t y, int64_t x,
                                             uint32_t* lds, uint32_t* red, int lane) {
  using PL = PermLds<K, G>;
  using Net = PairNet<K, G>;
  using bitonic::u16x2;
  constexpr int KV = K / 2;
  const RankView& rv = d.rv;
  const int64_t ld = rv.ld;
  const int64_t n = d.n;
  const int64_t n0 = n * (n - 1) / 2;
  const int64_t n1y = rv.n1[y], n1x = rv.n1[x];
  // u: the row with fewer ties, whose order is used; the other row's samples
  // are permuted (by pi if that is x, by pi^-1 if it is y)
  const bool swap = n1x < n1y;
  const int64_t u = swap ? x : y, v = swap ? y : x;
  const int64_t n1u = swap ? n1x : n1y;
  const uint16_t* table = swap ? d.inv : d.pad;
  // a constant u: every n_c - n_d is 0, every permutation counts
  if (n1u == n0) return d.B;
  const int k0 = Net::logical_lane(lane) * K;
  const bool in_row = k0 + K <= ld;   // ld is a multiple of 128
  uint16_t* row_v = (uint16_t*)lds;
  uint16_t* row_p = (uint16_t*)(lds + PL::kRowWords);
  uint32_t* xbuf = lds + 2 * PL::kRowWords;
  // v's rank row (lanes past the row: padding keys), u's order (byte offsets)
  uint32_t pw[KV];
  {
    uint32_t w[KV];
    if (in_row) {
      load_words<K>(rv.rank + v * ld + k0, w);
      load_words<K>(rv.perm + u * ld + k0, pw);
    } else {
#pragma unroll
      for (int i = 0; i < KV; ++i) {
        w[i] = 0xFFFEFFFEu;
        pw[i] = (uint32_t)(2 * (k0 + 2 * i)) | ((uint32_t)(2 * (k0 + 2 * i + 1)) << 16);
      }
    }
    store_words<K>(row_v + k0, w);
  }
  const int64_t base = n0 - n1y - n1x;   // S = base + n3 - 2 n_d
  const char* rowb = (const char*)row_v;
  int64_t s_obs = 0, count = 0;
  for (int64_t b = -1; b < d.B; ++b) {
    group_sync<G>();   // the previous pass is done with row_p (and row_v is staged)
    // row_p[t] = rank_v[sigma_b[t]] for this lane's slots (sigma = pi, or
    // pi^-1 when the roles turned; b < 0: the identity)
    uint32_t pi[KV];
    if (b >= 0 && in_row) {
      load_words<K>(table + b * ld + k0, pi);
    } else {
#pragma unroll
      for (int i = 0; i < KV; ++i)
        pi[i] = (uint32_t)(2 * (k0 + 2 * i)) | ((uint32_t)(2 * (k0 + 2 * i + 1)) << 16);
    }
    uint32_t w[KV];
#pragma unroll
    for (int i = 0; i < KV; ++i)
      w[i] = (uint32_t)*(const uint16_t*)(rowb + (pi[i] & 0xFFFFu)) |
             ((uint32_t)*(const uint16_t*)(rowb + (pi[i] >> 16)) << 16);
    store_words<K>(row_p + k0, w);
    group_sync<G>();
    u16x2 key[KV];
    gather_keys<K>(row_p, pw, key);
    uint32_t nd, n3;
    count_gathered<K, G>(key, row_p, in_row, k0, rv, u, n1u, rv, v, d.n, xbuf, red, lane,
                         nd, n3);
    int64_t s = base + (int64_t)n3 - 2 * (int64_t)nd;
    s = s < 0 ? -s : s;
    if (b < 0) s_obs = s;
    else count += s >= s_obs ? 1 : 0;
  }
  return count;
}

template <int K, int G>
__global__ void __launch_bounds__(kBlock, (fast_waves<K, G>())) perm_pairs_kernel(PermDesc d) {
  using PL = PermLds<K, G>;
  constexpr int kGroups = PL::kGroups;
  __shared__ uint32_t lds[PL::kBlockWords];
  uint32_t* red = lds + kGroups * PL::kWords;
  if (*d.status != 0) return;
  const int group = threadIdx.x / G;
  const int lane = threadIdx.x % G;
  uint32_t* buf = lds + group * PL::kWords;
  const int64_t count = d.J_end - d.J_begin;
  for (int64_t i = (int64_t)blockIdx.x * kGroups + group; i < count;
       i += (int64_t)gridDim.x * kGroups) {
    int64_t y, x;
    strict_pair(d.m, d.J_begin + i, y, x);
    const int64_t c = pair_perm<K, G>(d, y, x, buf, red, lane);
    if (lane == 0) {
      d.count_out[i] = c;
      if (d.p_out) d.p_out[i] = (double)(1 + c) / (double)(d.B + 1);
    }
  }
}

template <int K, int G>
hipError_t launch_perm_t(const PermDesc& d, hipStream_t s) {
  constexpr int kGroups = PermLds<K, G>::kGroups;
  int64_t grid = (d.J_end - d.J_begin + kGroups - 1) / kGroups;
  if (grid > kMaxPairGrid) grid = kMaxPairGrid;
  if (grid < 1) return hipSuccess;
  hipLaunchKernelGGL((perm_pairs_kernel<K, G>), dim3((unsigned)grid), dim3(kBlock), 0, s, d);
  return hipGetLastError();
}

// The network scheme of n (each capacity class's measured fastest).
hipError_t launch_perm(const PermDesc& d, hipStream_t s) {
  switch (network_scheme(d.n)) {
    case kSub8K16: return launch_perm_t<16, 8>(d, s);
    case kSub8K32: return launch_perm_t<32, 8>(d, s);
    case kSub16K32: return launch_perm_t<32, 16>(d, s);
    case kSub16K64: return launch_perm_t<64, 16>(d, s);
    case kSub32K64: return launch_perm_t<64, 32>(d, s);
    case kWaveK64: return launch_perm_t<64, 64>(d, s);
    case kBlockK32: return launch_perm_t<32, 256>(d, s);
    case kBlockK64: return launch_perm_t<64, 256>(d, s);
    case kBlockK128: return launch_perm_t<128, 256>(d, s);
    default: return hipErrorInvalidValue;
  }
}

size_t perm_pad_offset(int64_t m, int64_t n) {
  return (size_t)round_up((int64_t)ws_layout(m, n).total, (int64_t)kAlign);
}

size_t perm_table_bytes(int64_t n, int64_t B) {
  return (size_t)round_up(B * row_ld(n) * 2, (int64_t)kAlign);
}

}  // namespace
}  // namespace ktau

using namespace ktau;

extern "C" {

size_t ktau_perm_workspace_size(int64_t m, int64_t n, int64_t B) {
  if (check_shape(m, n) != KTAU_OK || n > KTAU_MAX_N_NETWORK || B < 1) return 0;
  return perm_pad_offset(m, n) + 2 * perm_table_bytes(n, B);
}

int ktau_perm_test(const float* X, int64_t m, int64_t n, const uint16_t* perms, int64_t B,
                   int64_t J_begin, int64_t J_end, int64_t* count_out, double* p_out, void* ws,
                   size_t ws_bytes, void* stream) {
  int rc = check_shape(m, n);
  if (rc != KTAU_OK) return rc;
  if (n > KTAU_MAX_N_NETWORK) return KTAU_ERANGE;
  if (!X || !perms || !count_out || B < 1 || B > (int64_t)0x7fffffff) return KTAU_EINVAL;
  if (!ws || ((uintptr_t)ws) % kAlign != 0) return KTAU_EINVAL;
  if (ws_bytes < ktau_perm_workspace_size(m, n, B)) return KTAU_ENOMEM;
  const int64_t P = m * (m - 1) / 2;
  if (J_begin < 0) {
    J_begin = 0;
    J_end = P;
  }
  if (J_begin > J_end || J_end > P) return KTAU_ERANGE;
  hipStream_t s = (hipStream_t)stream;
  int32_t* status = (int32_t*)ws;
  if (clear_words(status, 2, s) != KTAU_OK) return KTAU_EDEVICE;
  if ((rc = prepass_ws(X, m, n, ws, nullptr, nullptr, s)) != KTAU_OK) return rc;
  const WsLayout L = ws_layout(m, n);
  uint16_t* pad = (uint16_t*)((char*)ws + perm_pad_offset(m, n));
  uint16_t* inv = (uint16_t*)((char*)pad + perm_table_bytes(n, B));
  const size_t bits = (size_t)((n + 31) / 32) * sizeof(uint32_t);
  hipLaunchKernelGGL(perm_check_kernel, dim3((unsigned)B), dim3(256), bits, s, perms, (int)n,
                     L.ld, pad, inv, status);
  if (hipGetLastError() != hipSuccess) return KTAU_EDEVICE;
  if (J_end == J_begin) return KTAU_OK;
  const MatDesc md = matdesc(ws, m, n, ktau_pair_out{}, 0, 8, J_begin, J_end, status);
  PermDesc d;
  d.rv = md.rv;
  d.pad = pad;
  d.inv = inv;
  d.B = B;
  d.count_out = count_out;
  d.p_out = p_out;
  d.status = status;
  d.m = m;
  d.n = (int32_t)n;
  d.J_begin = J_begin;
  d.J_end = J_end;
  return launch_perm(d, s) == hipSuccess ? KTAU_OK : KTAU_EDEVICE;
}

}  // extern "C"
