// The naive count (Sec. 3.1, Algorithm 1: every sample pair compared, O(n^2)
// per pair of rows) for short rows, with the comparisons done once per row
// and stored as bit sets, so that a pair of rows costs one AND and one
// population count per 32 sample pairs.
//
// Per row r and sample a, two sets over the samples b of r (bit i of word k
// is sample b = 32k + i):
//   LT_r[a] = { b : rank_r(b) < rank_r(a) },   EQ_r[a] = { b : rank_r(b) = rank_r(a) }
// (b = a is in EQ_r[a]; bits of b >= n are clear).  For a pair (u, v), with
// GT_u[a] the samples above a in u (the valid bits outside LT_u[a] | EQ_u[a]):
//   n_d = sum_a |GT_u[a] & LT_v[a]|   (each discordant pair {a, b} is seen
//                                      from exactly one of its two samples)
//   n3  = (sum_a |EQ_u[a] & EQ_v[a]| - n) / 2   (both rows tied; b = a drops out)
// and n_c, tau_B, tau_A follow from n0, n1, n2 as on the other paths.  The
// counts are those of the definition (Eq. 1-3), so they equal the network's
// bit for bit.  Only samples tied with another sample of u can add to n3, so
// only their lanes read EQ sets.  Rows of at most 256 samples only: the two
// sets take 2 n w words per row (w = ceil(n/32) rounded up to 1, 2, 4 or 8),
// and the count grows as n^2/32.  Matrices of up to 2^20 pairs run one group
// per pair in job order; larger ones run q x q tiles.
#include "ktau_order.h"
#include "ktau_pairdev.h"
#include "ktau_query.h"

namespace ktau {

size_t bits_words_per_set(int64_t n) { return n <= 32 ? 1 : n <= 64 ? 2 : n <= 128 ? 4 : 8; }

size_t bits_bytes(int64_t m, int64_t n) {
  if (n > kBitsMaxN) return 0;
  return 2 * (size_t)m * (size_t)n * bits_words_per_set(n) * sizeof(uint32_t);
}

namespace {

constexpr int64_t kBitsJobsMaxPairs = 1 << 20;

// Sets of one row per workgroup: thread t builds word k = t mod nw of sample
// a = t / nw for both sets, from the row's dense ranks staged in LDS.
__global__ void __launch_bounds__(kBlock)
bits_prepass_kernel(const uint16_t* __restrict__ rank, int64_t ld, int n, int lognw,
                    uint32_t* __restrict__ lt, uint32_t* __restrict__ eq,
                    const int32_t* __restrict__ status) {
  __shared__ uint16_t s_rank[kBitsMaxN];
  if (*status != 0) return;
  const int64_t row = blockIdx.x;
  for (int b = threadIdx.x; b < n; b += kBlock) s_rank[b] = rank[row * ld + b];
  __syncthreads();
  const int nw = 1 << lognw;
  const int64_t base = row * (int64_t)n * nw;
  for (int t = threadIdx.x; t < n * nw; t += kBlock) {
    const int a = t >> lognw, k = t & (nw - 1);
    const uint32_t ra = s_rank[a];
    const int b0 = 32 * k;
    const int cnt = n - b0 < 32 ? n - b0 : 32;
    uint32_t l = 0, e = 0;
    for (int i = 0; i < cnt; ++i) {
      const uint32_t rb = s_rank[b0 + i];
      l |= (uint32_t)(rb < ra) << i;
      e |= (uint32_t)(rb == ra) << i;
    }
    lt[base + t] = l;
    eq[base + t] = e;
  }
}

// Group shape for sets of NW words: G = 8 NW lanes, four samples per lane
// (sample a = lane + G i), so a group covers n <= 32 NW; a wave of the tile
// kernel holds the sets of R rows of u at once (register blocking: every v
// set loaded serves R pairs).
template <int NW>
struct BitsShape {
  static constexpr int G = 8 * NW;
  static constexpr int A = 4;
  static constexpr int R = NW >= 8 ? 1 : NW >= 4 ? 2 : 4;   // measured best at 4 waves/SIMD
  static_assert(G * A == 32 * NW, "four samples per lane");
};

template <int NW>
__device__ __forceinline__ void load_set(const uint32_t* p, uint32_t (&w)[NW]) {
  if constexpr (NW % 4 == 0) {
#pragma unroll
    for (int k = 0; k < NW; k += 4) {
      const uint4 v = *(const uint4*)(p + k);
      w[k] = v.x;
      w[k + 1] = v.y;
      w[k + 2] = v.z;
      w[k + 3] = v.w;
    }
  } else if constexpr (NW == 2) {
    const uint2 v = *(const uint2*)p;
    w[0] = v.x;
    w[1] = v.y;
  } else {
    w[0] = *p;
  }
}

struct BitsDesc {
  MatDesc d;
  const uint32_t* lt;   // [m][n][NW]
  const uint32_t* eq;   // [m][n][NW]
};

// Row y as u: GT_u of this lane's samples (valid bits outside LT | EQ), and a
// bit per sample that is tied with another sample of the row (only those
// samples can add to n3).  lt_row / eq_row: the row's sets.
template <int NW>
__device__ __forceinline__ void load_u(const uint32_t* lt_row, const uint32_t* eq_row, int n,
                                       int lane, uint32_t (&gt)[BitsShape<NW>::A][NW],
                                       uint32_t& tied) {
  constexpr int G = BitsShape<NW>::G, A = BitsShape<NW>::A;
  tied = 0;
#pragma unroll
  for (int i = 0; i < A; ++i) {
    const int a = lane + G * i;
    if (a < n) {
      uint32_t l[NW], e[NW];
      load_set<NW>(lt_row + a * NW, l);
      load_set<NW>(eq_row + a * NW, e);
      uint32_t cnt = 0;
#pragma unroll
      for (int k = 0; k < NW; ++k) {
        const int rem = n - 32 * k;
        const uint32_t valid = rem >= 32 ? ~0u : rem > 0 ? (1u << rem) - 1u : 0u;
        gt[i][k] = ~(l[k] | e[k]) & valid;
        cnt += __builtin_popcount(e[k]);
      }
      tied |= (cnt > 1 ? 1u : 0u) << i;
    } else {
#pragma unroll
      for (int k = 0; k < NW; ++k) gt[i][k] = 0;
    }
  }
}

// Twice the joint ties of (u, v) over this lane's samples tied in u:
// |EQ_u[a] & EQ_v[a]| - 1 each (b = a is in both sets).
template <int NW>
__device__ __forceinline__ uint32_t joint_ties(const uint32_t* eq_u, const uint32_t* eq_v,
                                               uint32_t tied, int lane) {
  constexpr int G = BitsShape<NW>::G, A = BitsShape<NW>::A;
  uint32_t t2 = 0;
#pragma unroll
  for (int i = 0; i < A; ++i) {
    if ((tied >> i) & 1u) {
      const int a = lane + G * i;
      uint32_t eu[NW], ev[NW];
      load_set<NW>(eq_u + a * NW, eu);
      load_set<NW>(eq_v + a * NW, ev);
      uint32_t c = 0;
#pragma unroll
      for (int k = 0; k < NW; ++k) c += __builtin_popcount(eu[k] & ev[k]);
      t2 += c - 1u;
    }
  }
  return t2;
}

// Sum over the group of a lane's share packed as n_d in bits 0-15 and 2 n3
// in bits 16-31 (both below 2^16 for n <= 256: n_d <= n(n-1)/2 and
// 2 n3 <= n(n-1), so no carry crosses between them).
template <int G>
__device__ __forceinline__ uint32_t group_total(uint32_t v) {
#pragma unroll
  for (int d = G / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// One q x q tile per workgroup pass.  Wave w takes blocks of R consecutive
// tile rows (w R, w R + 4 R, ...) with u's sets in registers; the groups of
// the wave take the columns in turn, and each v set loaded is counted against
// all R rows.
template <int NW>
__device__ __forceinline__ void bits_tile(const BitsDesc& b, int64_t yq, int64_t xq) {
  constexpr int G = BitsShape<NW>::G, A = BitsShape<NW>::A, R = BitsShape<NW>::R;
  constexpr int kPerWave = 64 / G;
  constexpr int kWaves = kBlock / 64;
  const MatDesc& d = b.d;
  const int n = d.n;
  const int64_t row_words = (int64_t)n * NW;
  // the wave index is the same in every lane of a wave: keeping it in a
  // scalar register keeps the rows of u, their addresses and n1 there too
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int group = (threadIdx.x & 63) / G;
  const int lane = threadIdx.x % G;
  const int q = d.q;
  const int64_t xlo = xq * q;
  Deferred<G> done;
  uint32_t gt[R][A][NW];
  uint32_t tied[R];
  for (int r0 = wave * R; r0 < q; r0 += kWaves * R) {
    const int64_t y0 = yq * q + r0;
    if (y0 >= d.m) break;
    if (y0 + 1 >= xlo + q) continue;   // no column of this tile lies above these rows
    const int rows = (int)min((int64_t)min(R, q - r0), d.m - y0);   // rows of u held
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (r < rows) {
        load_u<NW>(b.lt + (y0 + r) * row_words, b.eq + (y0 + r) * row_words, n, lane, gt[r],
                   tied[r]);
      } else {
#pragma unroll
        for (int i = 0; i < A; ++i)
#pragma unroll
          for (int k = 0; k < NW; ++k) gt[r][i][k] = 0;
        tied[r] = 0;
      }
    }
    for (int c = group; c < q; c += kPerWave) {
      const int64_t x = xlo + c;
      if (x <= y0 || x >= d.m) continue;
      const uint32_t* lt_v = b.lt + x * row_words;
      uint32_t l[A][NW];
#pragma unroll
      for (int i = 0; i < A; ++i) {
        const int a = lane + G * i;
        if (a < n) {
          load_set<NW>(lt_v + a * NW, l[i]);
        } else {
#pragma unroll
          for (int k = 0; k < NW; ++k) l[i][k] = 0;
        }
      }
      const int64_t n1x = d.rv.n1[x];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int64_t y = y0 + r;
        if (r >= rows || x <= y) continue;    // group-uniform
        uint32_t nd = 0;
#pragma unroll
        for (int i = 0; i < A; ++i)
#pragma unroll
          for (int k = 0; k < NW; ++k) nd += __builtin_popcount(gt[r][i][k] & l[i][k]);
        const int64_t n1y = d.rv.n1[y];
        uint32_t t2 = 0;
        if (n1y > 0 && n1x > 0)
          t2 = joint_ties<NW>(b.eq + y * row_words, b.eq + x * row_words, tied[r], lane);
        const uint32_t v = group_total<G>(nd | (t2 << 16));
        done.add(lane, strict_job(d.m, y, x), n1y, n1x, v & 0xFFFFu, v >> 17);
        if (done.full()) done.flush(lane, d.out, d.n);
      }
    }
  }
  done.flush(lane, d.out, d.n);
}

template <int NW>
__global__ void __launch_bounds__(kBlock, 4) bits_tiles_kernel(BitsDesc b) {
  const MatDesc& d = b.d;
  if (*d.status != 0) return;
  int64_t yq, xq;
  if ((int64_t)gridDim.x == d.n_units) {
    scheduled_tile(d.w, d.n_units, blockIdx.x, yq, xq);
    bits_tile<NW>(b, yq, xq);
    return;
  }
  for (int64_t t = blockIdx.x; t < d.n_units; t += gridDim.x) {
    tile_coord(d.w, t, yq, xq);
    bits_tile<NW>(b, yq, xq);
  }
}

// Jobs [J_begin, J_end), one per group; result slot J - J_begin.
template <int NW>
__global__ void __launch_bounds__(kBlock) bits_jobs_kernel(BitsDesc b) {
  constexpr int G = BitsShape<NW>::G, A = BitsShape<NW>::A;
  constexpr int kGroups = kBlock / G;
  const MatDesc& d = b.d;
  if (*d.status != 0) return;
  const int n = d.n;
  const int group = threadIdx.x / G;
  const int lane = threadIdx.x % G;
  const int64_t count = d.J_end - d.J_begin;
  Deferred<G> done;
  const int64_t row_words = (int64_t)n * NW;
  uint32_t gt[A][NW];
  for (int64_t i = (int64_t)blockIdx.x * kGroups + group; i < count;
       i += (int64_t)gridDim.x * kGroups) {
    int64_t y, x;
    strict_pair(d.m, d.J_begin + i, y, x);
    uint32_t tied;
    load_u<NW>(b.lt + y * row_words, b.eq + y * row_words, n, lane, gt, tied);
    const uint32_t* lt_v = b.lt + x * row_words;
    uint32_t nd = 0;
#pragma unroll
    for (int j = 0; j < A; ++j) {
      const int a = lane + G * j;
      if (a < n) {
        uint32_t l[NW];
        load_set<NW>(lt_v + a * NW, l);
#pragma unroll
        for (int k = 0; k < NW; ++k) nd += __builtin_popcount(gt[j][k] & l[k]);
      }
    }
    const int64_t n1y = d.rv.n1[y], n1x = d.rv.n1[x];
    uint32_t t2 = 0;
    if (n1y > 0 && n1x > 0)
      t2 = joint_ties<NW>(b.eq + y * row_words, b.eq + x * row_words, tied, lane);
    const uint32_t v = group_total<G>(nd | (t2 << 16));
    done.add(lane, i, n1y, n1x, v & 0xFFFFu, v >> 17);
    if (done.full()) done.flush(lane, d.out, d.n);
  }
  done.flush(lane, d.out, d.n);
}

// (query row, database row) pairs i = qi m + j, one per group, for the query
// search: u = the query row, v = the database row.
template <int NW>
__global__ void __launch_bounds__(kBlock) bits_query_kernel(QueryDesc qd, const uint32_t* qlt,
                                                            const uint32_t* qeq,
                                                            const uint32_t* dlt,
                                                            const uint32_t* deq) {
  constexpr int G = BitsShape<NW>::G, A = BitsShape<NW>::A;
  constexpr int kGroups = kBlock / G;
  if (*qd.status != 0) return;
  const int n = qd.n;
  const int group = threadIdx.x / G;
  const int lane = threadIdx.x % G;
  const int64_t jobs = qd.nq * qd.m;
  const int64_t row_words = (int64_t)n * NW;
  Deferred<G> done;
  auto store = [&](int64_t slot, int64_t a, int64_t b, uint32_t d, uint32_t t) {
    store_cross(qd, slot, a, b, d, t);
  };
  uint32_t gt[A][NW];
  int64_t loaded = -1;   // query row whose sets are in gt
  uint32_t tied = 0;
  for (int64_t i = (int64_t)blockIdx.x * kGroups + group; i < jobs;
       i += (int64_t)gridDim.x * kGroups) {
    const int64_t qi = i / qd.m, j = i - qi * qd.m;
    if (qi != loaded) {
      load_u<NW>(qlt + qi * row_words, qeq + qi * row_words, n, lane, gt, tied);
      loaded = qi;
    }
    const uint32_t* lt_v = dlt + j * row_words;
    uint32_t nd = 0;
#pragma unroll
    for (int a4 = 0; a4 < A; ++a4) {
      const int a = lane + G * a4;
      if (a < n) {
        uint32_t l[NW];
        load_set<NW>(lt_v + a * NW, l);
#pragma unroll
        for (int k = 0; k < NW; ++k) nd += __builtin_popcount(gt[a4][k] & l[k]);
      }
    }
    const int64_t n1q = qd.rq.n1[qi], n1d = qd.rdb.n1[j];
    uint32_t t2 = 0;
    if (n1q > 0 && n1d > 0) t2 = joint_ties<NW>(qeq + qi * row_words, deq + j * row_words, tied, lane);
    const uint32_t v = group_total<G>(nd | (t2 << 16));
    done.add(lane, i, n1q, n1d, v & 0xFFFFu, v >> 17);
    if (done.full()) done.flush_with(lane, store);
  }
  done.flush_with(lane, store);
}

template <int NW>
hipError_t launch_bits_query_t(const QueryDesc& qd, const uint32_t* qbits, const uint32_t* dbbits,
                               hipStream_t s) {
  constexpr int kGroups = kBlock / BitsShape<NW>::G;
  const int64_t jobs = qd.nq * qd.m;
  int64_t grid = (jobs + kGroups - 1) / kGroups;
  if (grid > kMaxPairGrid) grid = kMaxPairGrid;
  if (grid < 1) return hipSuccess;
  const size_t qset = (size_t)qd.nq * qd.n * NW, dset = (size_t)qd.m * qd.n * NW;
  hipLaunchKernelGGL((bits_query_kernel<NW>), dim3((unsigned)grid), dim3(kBlock), 0, s, qd,
                     qbits, qbits + qset, dbbits, dbbits + dset);
  return hipGetLastError();
}

template <int NW>
hipError_t launch_bits_t(const BitsDesc& b, bool tiles, hipStream_t s) {
  int64_t grid;
  if (tiles) {
    grid = b.d.n_units < (1ll << 30) ? b.d.n_units : (1ll << 30);
    if (grid < 1) return hipSuccess;
    hipLaunchKernelGGL((bits_tiles_kernel<NW>), dim3((unsigned)grid), dim3(kBlock), 0, s, b);
  } else {
    constexpr int kGroups = kBlock / BitsShape<NW>::G;
    const int64_t count = b.d.J_end - b.d.J_begin;
    grid = (count + kGroups - 1) / kGroups;
    if (grid > kMaxPairGrid) grid = kMaxPairGrid;
    if (grid < 1) return hipSuccess;
    hipLaunchKernelGGL((bits_jobs_kernel<NW>), dim3((unsigned)grid), dim3(kBlock), 0, s, b);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_bits_prepass(const MatDesc& d, uint32_t* bits, hipStream_t s) {
  if (d.n > kBitsMaxN || d.m < 1) return hipErrorInvalidValue;
  const size_t nw = bits_words_per_set(d.n);
  const int lognw = nw == 1 ? 0 : nw == 2 ? 1 : nw == 4 ? 2 : 3;
  uint32_t* lt = bits;
  uint32_t* eq = bits + (size_t)d.m * d.n * nw;
  hipLaunchKernelGGL(bits_prepass_kernel, dim3((unsigned)d.m), dim3(kBlock), 0, s, d.rv.rank,
                     d.rv.ld, (int)d.n, lognw, lt, eq, d.status);
  return hipGetLastError();
}

hipError_t launch_bits_pairs(const MatDesc& d, const uint32_t* bits, bool tiles, hipStream_t s) {
  if (d.n > kBitsMaxN) return hipErrorInvalidValue;
  const size_t nw = bits_words_per_set(d.n);
  BitsDesc b;
  b.d = d;
  // Few pairs (small m): one group per pair in job order fills the GPU, where
  // the tiles would leave most of it idle; the result slots are the same.
  if (tiles && d.m * (d.m - 1) / 2 <= kBitsJobsMaxPairs) {
    tiles = false;
    b.d.J_begin = 0;
    b.d.J_end = d.m * (d.m - 1) / 2;
  }
  b.lt = bits;
  b.eq = bits + (size_t)d.m * d.n * nw;
  switch (nw) {
    case 1: return launch_bits_t<1>(b, tiles, s);
    case 2: return launch_bits_t<2>(b, tiles, s);
    case 4: return launch_bits_t<4>(b, tiles, s);
    default: return launch_bits_t<8>(b, tiles, s);
  }
}

hipError_t launch_bits_query(const QueryDesc& qd, const uint32_t* qbits, const uint32_t* dbbits,
                             hipStream_t s) {
  if (qd.n > kBitsMaxN) return hipErrorInvalidValue;
  switch (bits_words_per_set(qd.n)) {
    case 1: return launch_bits_query_t<1>(qd, qbits, dbbits, s);
    case 2: return launch_bits_query_t<2>(qd, qbits, dbbits, s);
    case 4: return launch_bits_query_t<4>(qd, qbits, dbbits, s);
    default: return launch_bits_query_t<8>(qd, qbits, dbbits, s);
  }
}

}  // namespace ktau
