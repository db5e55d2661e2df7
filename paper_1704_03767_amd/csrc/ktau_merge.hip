// Merge schemes for long rows: the Step 3 count of Sec. 3.2 (discordant
// pairs as the strict inversions of v in u's order, which Algorithm 2 counts
// with a merge sort), here with the lower merge levels done by the register
// network of ktau_bitonic.h on chunks and the upper levels as a merge path
// over 16-bit keys in LDS.
//
// One workgroup of W = ceil(n / C) waves takes one pair at a time, C = 64 K
// keys per wave (K = 32 or 64).  The samples in u's sorted order are cut into
// W chunks of C positions (the last one padded with keys above every rank),
// chunk w belonging to wave w:
//   1. v's rank row is staged in LDS; every lane gathers its K positions,
//      v'[k] = rank_v[perm_u[k]], into registers.  If u has ties the keys then
//      replace the rank row (v' in u order), where the in-run count reads them
//      exactly as in the network schemes (inversions and equal values between
//      positions of one tie run of u);
//   2. each wave sorts its chunk with the tagged bitonic network, which also
//      counts the chunk's inversions, and stores it back in LDS sorted;
//   3. level by level, neighbouring sorted runs of s = C, 2C, 4C, ... keys are
//      merged: each lane owns K consecutive output positions, finds where they
//      start on the merge path (a binary search over the two runs), merges its
//      K keys into registers and counts, for every key taken from the right
//      run, the left keys still waiting (all of them larger: on equal keys the
//      left one goes first, so ties never count); the merged keys replace the
//      runs once every lane has read them.  The top level only counts.
// n_d = all inversions - the inversions inside u's tie runs (Sec. 3.2 Step 1
// orders tied u by v; taking ties in sample order and subtracting gives the
// same count).  Padding needs no positions beyond the last chunk, unlike a
// network of the whole row (a power of two).
//
// Rows longer than 32768 samples have ranks up to 65535, whose doubled keys do
// not fit 16 bits.  Their pairs run steps 1-3 twice, on the keys
// 2 min(v', 32767) and then 2 max(v' - 32768, 0) (both at most 0xFFFE).  An
// inversion v'_j > v'_k (j < k) is seen by the first pass exactly when
// v'_k < 32767 and by the second exactly when v'_j > 32768, so
//   inv = inv_1 + inv_2 - #{j < k : v'_j > 32768, v'_k < 32767}
//                       + #{j < k : v'_j = 32768, v'_k = 32767},
// and both corrections come from one prefix scan over v' in u order.
#include "ktau_pairdev.h"

namespace ktau {
namespace {

using bitonic::u16x2;

constexpr int kMergeThreads = 64 * kMergeMaxWaves;
constexpr int kMergeHdrWords = 64;          // LDS words before the row: sums, scans
constexpr uint32_t kMergeSentinel = 0xFFFFu;  // above every key (keys <= 0xFFFE)
constexpr uint32_t kHalf = 32768;

// While sorted runs are merged the row is kept padded: 4 uint16 (two LDS
// dwords) after every 64 keys.  Each lane merges 64 consecutive outputs, so
// lanes read keys 32 to 64 positions apart; unpadded, such strides (64 or
// 128 bytes) put every lane of a wave on the same LDS bank.  Padded, a
// stride of 32 keys moves 17 dwords (a different bank per lane) and one of 64
// keys 34 dwords (two lanes per bank).  The first pad slot after each block
// holds the sentinel that a merge reads past the end of a run.  The in-order
// row of the gather and the in-run count stays unpadded.
__device__ __forceinline__ int padded(int p) { return p + ((p >> 6) << 2); }

template <int K>
struct MergeShape {
  static constexpr int kChunk = 64 * K;
  static int waves(int64_t n) { return (int)((n + kChunk - 1) / kChunk); }
  // header, padded row, and 16 bytes of slack
  static size_t lds_bytes(int waves) {
    const size_t keys = (size_t)waves * kChunk;
    return kMergeHdrWords * sizeof(uint32_t) + (keys + keys / 16) * sizeof(uint16_t) + 16;
  }
};

// Sum over the workgroup (modulo 2^32); every thread gets the total.
__device__ __forceinline__ uint32_t merge_block_sum(uint32_t v, uint32_t* red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  uint32_t t = 0;
  const int waves = (int)(blockDim.x >> 6);
  for (int w = 0; w < waves; ++w) t += red[w];
  return t;
}

// Exclusive prefix sums over threads (in thread order) of two counts.
__device__ __forceinline__ void merge_block_scan2(uint32_t& a, uint32_t& b, uint32_t* sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t ia = a, ib = b;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t ta = __shfl_up(ia, d, 64), tb = __shfl_up(ib, d, 64);
    if (lane >= d) {
      ia += ta;
      ib += tb;
    }
  }
  __syncthreads();
  if (lane == 63) {
    sh[wave] = ia;
    sh[16 + wave] = ib;
  }
  __syncthreads();
  uint32_t ba = 0, bb = 0;
  for (int w = 0; w < wave; ++w) {
    ba += sh[w];
    bb += sh[16 + w];
  }
  a = ba + ia - a;
  b = bb + ib - b;
}

// This lane's K positions k0.. of v' in u's order, packed as the network
// wants them (VGPR j holds k0 + j low and k0 + j + K/2 high), from the rank
// row staged in LDS.  perm entries are byte offsets into the row (doubled
// workspaces) or sample indices (plain); positions past the padded row get
// the padding key.
template <int K>
__device__ __forceinline__ void merge_gather(const uint16_t* row, const uint16_t* permrow, int k0,
                                             int64_t ld, bool doubled, u16x2 (&key)[K / 2]) {
  constexpr int KV = K / 2;
  if (k0 + K <= ld) {
    uint32_t pw[KV];
    load_words<K>(permrow + k0, pw);
    const char* rowb = (const char*)row;
    const uint32_t sh = doubled ? 0u : 1u;
#pragma unroll
    for (int j = 0; j < KV; ++j) {
      const uint32_t a = j % 2 ? pw[j / 2] >> 16 : pw[j / 2] & 0xFFFFu;
      const uint32_t b = (j + KV) % 2 ? pw[(j + KV) / 2] >> 16 : pw[(j + KV) / 2] & 0xFFFFu;
      u16x2 t;
      t.x = *(const uint16_t*)(rowb + (a << sh));
      t.y = *(const uint16_t*)(rowb + (b << sh));
      key[j] = t;
    }
  } else {
    const uint16_t pad = doubled ? 0xFFFEu : 0xFFFFu;
#pragma unroll
    for (int j = 0; j < KV; ++j) {
      key[j].x = pad;
      key[j].y = pad;
    }
  }
}

// K consecutive uint16 packed in K/2 words (element 2i low, 2i+1 high) to an
// 8-byte aligned address, two words per store.
template <int K>
__device__ __forceinline__ void store_words8(uint16_t* p, const uint32_t (&w)[K / 2]) {
#pragma unroll
  for (int i = 0; i < K / 4; ++i) ((uint2*)p)[i] = make_uint2(w[2 * i], w[2 * i + 1]);
}

// Keys in the network's packing, as K consecutive words in position order.
template <int K>
__device__ __forceinline__ void unpack_keys(const u16x2 (&key)[K / 2], uint32_t mask,
                                            uint32_t (&w)[K / 2]) {
  constexpr int KV = K / 2;
#pragma unroll
  for (int i = 0; i < KV / 2; ++i) {
    const uint32_t lo = bitonic::bits(key[2 * i]) & mask;
    const uint32_t hi = bitonic::bits(key[2 * i + 1]) & mask;
    // positions k0 + 2i, 2i + 1 (low halves), k0 + KV + 2i, 2i + 1 (high)
    w[i] = __builtin_amdgcn_perm(hi, lo, 0x05040100u);
    w[KV / 2 + i] = __builtin_amdgcn_perm(hi, lo, 0x07060302u);
  }
}

// Stores keys in the network's packing at positions k0 .. k0+K-1 of the
// unpadded row.
template <int K>
__device__ __forceinline__ void merge_store_keys(uint16_t* row, int k0, const u16x2 (&key)[K / 2],
                                                 uint32_t mask) {
  uint32_t w[K / 2];
  unpack_keys<K>(key, mask, w);
  store_words<K>(row + k0, w);
}

// Byte offset in the padded row of the key at doubled position i2 = 2 p.
// (one shift and one shift-add; left to itself the compiler used three)
__device__ __forceinline__ uint32_t padded_byte(uint32_t i2) {
  uint32_t o;
  asm("v_lshl_add_u32 %0, %1, 3, %2" : "=v"(o) : "v"(i2 >> 7), "v"(i2));
  return o;
}

// One lane's K outputs of the merge of sorted runs A (positions l0 ..
// l0 + lenA - 1 of the padded row) and B (l0 + s .. l0 + s + lenB - 1),
// starting at output position diag; returns the number of (A, B) pairs among
// them with the A key strictly larger (for each B key taken, the A keys not
// yet taken).  With kStore the merged keys are packed into w (output 2i low,
// 2i + 1 high).  Every run ends at a 64-key boundary, and the first slot of
// the pad after it holds the sentinel: a head past the end of its run reads
// that slot, since the byte offset of a position only grows with it and the
// load takes the smaller of the head's offset and the run's pad slot.  The
// lane keeps the doubled positions of both heads; each step loads the next
// key of the run it took from.
//
// The count needs no work per B key: with nB(t) the B keys taken before step
// t and lo the A keys before the segment, the B key taken at step t finds
// lenA - lo - (t - nB(t)) A keys waiting, and the j-th B key taken has
// nB(t) = j, so the count is nB (lenA - lo) - sum_{B steps} t + nB (nB - 1) / 2,
// where sum_{B steps} t = nB (K - 1) - sum_t nB(t): a plain running sum of
// B's head position.
template <int K, bool kStore>
__device__ __forceinline__ uint32_t merge_segment(const uint16_t* row, int l0, int s, int lenA,
                                                  int lenB, int diag, uint32_t (&w)[K / 2]) {
  auto at = [&](int p) { return (uint32_t)row[padded(l0 + p)]; };
  // merge path: the number of A keys among the first diag outputs
  int lo = diag > lenB ? diag - lenB : 0;
  int hi = diag < lenA ? diag : lenA;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (at(mid) <= at(s + diag - 1 - mid)) lo = mid + 1;
    else hi = mid;
  }
  const char* base = (const char*)row;
  const uint32_t limA = padded_byte(2u * (uint32_t)(l0 + lenA - 1)) + 2u;
  const uint32_t limB = padded_byte(2u * (uint32_t)(l0 + s + lenB - 1)) + 2u;
  auto load = [&](uint32_t i2, uint32_t lim) {
    const uint32_t o = padded_byte(i2);
    return (uint32_t)*(const uint16_t*)(base + (o < lim ? o : lim));
  };
  uint32_t ia2 = 2u * (uint32_t)(l0 + lo);               // A's head
  uint32_t ib2 = 2u * (uint32_t)(l0 + s + diag - lo);    // B's head
  const uint32_t ib0 = ib2;
  uint32_t a = load(ia2, limA), b = load(ib2, limB);
  uint32_t heads = 0, low = 0;   // heads: sum over steps of B's head
  bool tb = false;
#pragma unroll
  for (int t = 0; t < K; ++t) {
    heads += ib2;
    // keep the sum a chain: reassociated, it held every step's terms live
    asm volatile("" : "+v"(heads));
    tb = b < a;
    if constexpr (kStore) {
      const uint32_t o = tb ? b : a;
      if (t & 1) w[t / 2] = low | (o << 16);
      else low = o;
    }
    if (t + 1 < K) {
      const uint32_t nxt = (tb ? ib2 : ia2) + 2u;
      ia2 = tb ? ia2 : nxt;
      ib2 = tb ? nxt : ib2;
      const uint32_t nv = load(nxt, tb ? limB : limA);
      a = tb ? a : nv;
      b = tb ? nv : b;
    }
  }
  const uint32_t nb = ((ib2 - ib0) >> 1) + (tb ? 1u : 0u);
  const uint32_t sum_nb = (heads - (uint32_t)K * ib0) >> 1;
  const uint32_t sum_t = nb * (uint32_t)(K - 1) - sum_nb;
  return nb * (uint32_t)(lenA - lo) - sum_t + nb * (nb - 1u) / 2u;
}

// The inverse of merge_store_keys: positions k0 .. k0+K-1 of the row, in the
// network's packing.
template <int K>
__device__ __forceinline__ void merge_load_keys(const uint16_t* row, int k0, u16x2 (&key)[K / 2]) {
  constexpr int KV = K / 2;
  uint32_t w[KV];
  load_words<K>(row + k0, w);
#pragma unroll
  for (int i = 0; i < KV / 2; ++i) {
    key[2 * i] = bitonic::vec(__builtin_amdgcn_perm(w[KV / 2 + i], w[i], 0x05040100u));
    key[2 * i + 1] = bitonic::vec(__builtin_amdgcn_perm(w[KV / 2 + i], w[i], 0x07060302u));
  }
}

// The first `total` pairs of positions inside one tie run of u (in the order
// of u's run list), split evenly into 2 nthreads stretches, two walked side
// by side per thread; returns this thread's inversions inside runs and adds
// its equal pairs to tie.
__device__ __forceinline__ uint32_t merge_tie_walk(const RankView& ru_v, int64_t u, uint32_t total,
                                                   const uint16_t* row, uint32_t& tie) {
  uint32_t xin = 0;
  const int64_t ld = ru_v.ld;
  const int tid = threadIdx.x, nthreads = blockDim.x;
  const uint64_t* rl = ru_v.runs + u * (ld / 2);
  const int nr = ru_v.nruns[u];
  const uint32_t per = (uint32_t)(((uint64_t)total + 2u * nthreads - 1u) / (2u * nthreads));
  const uint64_t p0 = (uint64_t)tid * per, p1 = (uint64_t)(tid + nthreads) * per;
  const uint32_t c0 = p0 < total ? (uint32_t)(total - p0 < per ? total - p0 : per) : 0u;
  const uint32_t c1 = p1 < total ? (uint32_t)(total - p1 < per ? total - p1 : per) : 0u;
  if (c0 > 0) {
    TieWalk w0, w1;
    w0.init(rl, nr, (uint32_t)p0, row);
    if (c1 > 0) w1.init(rl, nr, (uint32_t)p1, row);
    for (uint32_t i = 0; i < c0; ++i) {
      w0.step(row, i + 1 < c0, xin, tie);
      if (i < c1) w1.step(row, i + 1 < c1, xin, tie);
    }
  }
  return xin;
}

// One long tie run of u (len keys 2 v' from position start of the in-order
// row) on one wave's network of 64 K >= len keys: the strict inversions inside
// it (desc) and, on the keys reflected (0xFFFE - key, the padding kept last),
// its strict ascents (asc); its pairs with equal v' (joint ties) are the rest,
// len (len - 1) / 2 - desc - asc.  Adds this lane's parts to xin and tie.
template <int K>
__device__ __forceinline__ void long_run_count(const uint16_t* row, int start, int len, int plane,
                                               uint32_t& xin, uint32_t& tie) {
  using Net = bitonic::Net<K, 64>;
  constexpr int KV = K / 2;
  const int e0 = Net::logical_lane(plane) * K;
  // keys of the run (reflected or not), the padding 0xFFFE last either way
  auto load = [&](u16x2 (&key)[KV], uint32_t flip) {
#pragma unroll
    for (int j = 0; j < KV; ++j) {
      const int ex = e0 + j, ey = e0 + j + KV;
      key[j].x = (unsigned short)(ex < len ? (uint32_t)row[start + ex] ^ flip : 0xFFFEu);
      key[j].y = (unsigned short)(ey < len ? (uint32_t)row[start + ey] ^ flip : 0xFFFEu);
    }
  };
  u16x2 key[KV];
  load(key, 0u);
  const uint32_t desc = Net::count(key, plane, nullptr);
  // 0xFFFE - k = k ^ 0xFFFE for even k <= 0xFFFE
  load(key, 0xFFFEu);
  const uint32_t asc = Net::count(key, plane, nullptr);
  xin += desc;
  tie += (plane == 0 ? (uint32_t)(len * (len - 1) / 2) : 0u) - desc - asc;
}

// The long runs of u (the last nl entries of its run list), wave w taking
// runs w, w + W, ...; returns this lane's inversions inside them and adds
// its part of their joint ties to tie.
__device__ __forceinline__ uint32_t merge_long_runs(const uint64_t* rl, int nl, const uint16_t* row,
                                                    uint32_t& tie) {
  const int wave = threadIdx.x >> 6, plane = threadIdx.x & 63, waves = blockDim.x >> 6;
  uint32_t xin = 0;
  for (int r = wave; r < nl; r += waves) {
    const uint64_t e = rl[r];
    const int start = (int)(e & 0xFFFFu), len = (int)((e >> 16) & 0xFFFFu) + 1;
    // one network size for every long run: larger or several sizes made the
    // kernel spill registers
    long_run_count<8>(row, start, len, plane, xin, tie);
  }
  return xin;
}

// The two cross terms of the split of 16-bit ranks into halves (file
// comment), from v' in u order in the row: thread t owns positions
// t K .. t K + K - 1 of the NR.  Returns this thread's part of
// #{v'_j = 32768, v'_k = 32767} - #{v'_j > 32768, v'_k < 32767}, j < k.
template <int K>
__device__ __forceinline__ uint32_t merge_cross_terms(const uint16_t* row, int NR, uint32_t* scan) {
  const int p = threadIdx.x * K;
  const bool mine = p < NR;
  uint32_t h = 0, e = 0;
  if (mine)
    for (int i = 0; i < K; ++i) {
      const uint32_t r = row[p + i];
      h += r > kHalf ? 1u : 0u;
      e += r == kHalf ? 1u : 0u;
    }
  merge_block_scan2(h, e, scan);
  uint32_t plus = 0, minus = 0;
  if (mine)
    for (int i = 0; i < K; ++i) {
      const uint32_t r = row[p + i];
      minus += r < kHalf - 1 ? h : 0u;
      plus += r == kHalf - 1 ? e : 0u;
      h += r > kHalf ? 1u : 0u;
      e += r == kHalf ? 1u : 0u;
    }
  return plus - minus;
}

// Sorts and counts this wave's chunk (network), stores it sorted, then runs
// the merge levels over the row; returns this lane's part of the inversion
// count.  Every thread of the workgroup calls it.
template <int K>
__device__ __forceinline__ uint32_t merge_count(u16x2 (&key)[K / 2], uint16_t* row, int NR,
                                                bool active, int k0, int plane, bool skip_top) {
  using Net = bitonic::Net<K, 64>;
  constexpr int KV = K / 2;
  constexpr int C = 64 * K;
  uint32_t share = 0;
  if (active) share += Net::count(key, plane, nullptr);
  // the row may still be the staged rank row that other waves gather from
  __syncthreads();
  if (active) {
    // sorted, tags cleared, into the padded row
    uint32_t w[KV];
    unpack_keys<K>(key, 0xFFFEFFFEu, w);
    store_words8<K>(row + padded(k0), w);
    // the pad after each 64-key block holds the merge's sentinel
    if (((k0 + K) & 63) == 0)
      *(uint2*)(row + padded(k0 + K - 1) + 1) =
          make_uint2(kMergeSentinel * 0x10001u, kMergeSentinel * 0x10001u);
  }
  __syncthreads();
  for (int s = C; s < NR; s <<= 1) {
    const bool top = 2 * s >= NR;
    if (top && skip_top) break;
    const int l0 = k0 & ~(2 * s - 1);
    const int lenA = NR - l0 < s ? NR - l0 : s;
    const int restB = NR - l0 - s;
    const int lenB = restB <= 0 ? 0 : restB < s ? restB : s;
    const bool work = active && lenB > 0;
    uint32_t w[KV];
    if (top) {
      if (work) share += merge_segment<K, false>(row, l0, s, lenA, lenB, k0 - l0, w);
    } else {
      if (work) share += merge_segment<K, true>(row, l0, s, lenA, lenB, k0 - l0, w);
      __syncthreads();
      if (work) store_words8<K>(row + padded(k0), w);
      __syncthreads();
    }
  }
  return share;
}

// n_d and n3 of rows (y, x), computed by the whole workgroup (blockDim.x =
// 64 W' with W' >= ceil(n / C)); false, with nothing computed, if both rows
// exceed the tie budget (the composite pass takes the pair).  lds: header
// words, then a row of W C uint16 and slack.  kWide: rows longer than
// kDoubledMaxN (plain ranks and sample indices, two counting passes).
template <int K, bool kWide>
__device__ bool pair_merge(const RankView& ry, int64_t y, const RankView& rx, int64_t x, int n,
                           int64_t budget, uint32_t* lds, uint32_t& nd, uint32_t& n3) {
  using Net = bitonic::Net<K, 64>;
  constexpr int KV = K / 2;
  constexpr int C = 64 * K;
  const int64_t n1y = ry.n1[y], n1x = rx.n1[x];
  if (n1y > budget && n1x > budget) return false;
  const bool swap = n1x < n1y;
  const RankView& ru_v = swap ? rx : ry;
  const RankView& rv_v = swap ? ry : rx;
  const int64_t u = swap ? x : y, v = swap ? y : x;
  const int64_t n1u = swap ? n1x : n1y;
  if (n1u == (int64_t)n * (n - 1) / 2) {
    // u constant (then so is v, u being the lighter row): every sample pair
    // is tied in u, none discordant, and the joint ties are v's ties
    nd = 0;
    n3 = (uint32_t)(swap ? n1y : n1x);
    return true;
  }
  const int64_t ld = ry.ld;
  uint32_t* red = lds;
  uint32_t* scan = lds + 16;
  uint16_t* row = (uint16_t*)(lds + kMergeHdrWords);
  const int tid = threadIdx.x, nthreads = blockDim.x;
  const int wave = tid >> 6, plane = tid & 63;
  const int nw = (n + C - 1) / C;
  const int NR = nw * C;
  const bool active = wave < nw;
  const int k0 = wave * C + Net::logical_lane(plane) * K;
  uint32_t share = 0;        // inversions (mod 2^32), this lane's part
  uint32_t tie = 0;
  // The top merge (first s_top positions against the rest) is counted from
  // v's global ranks when v has at most kTopGroups tie groups, as for the
  // network's last merge (top_share): the first s_top positions are all
  // samples, s_top <= (nw - 1) C < n.  Rows of the wide form, whose two
  // passes clamp the keys, always merge.
  int s_top = C;
  while (2 * s_top < NR) s_top <<= 1;
  const int ngroups = (kWide || nw < 2) ? kTopGroups + 1 : rv_v.nruns[v];
  const bool closed = ngroups <= kTopGroups;
  uint32_t eqs = 0;
  for (int pass = 0; pass < (kWide ? 2 : 1); ++pass) {
    // the previous pair (or pass) has finished with the row
    __syncthreads();
    {
      const uint4* src = (const uint4*)(rv_v.rank + v * ld);
      uint4* dst = (uint4*)row;
      for (int i = tid; i < (int)(ld / 8); i += nthreads) dst[i] = src[i];
    }
    __syncthreads();
    u16x2 key[KV];
    if (active) merge_gather<K>(row, ru_v.perm + u * ld, k0, ld, !kWide, key);
    if (closed && active && k0 < s_top) {
      TopGroups tg;
      top_groups(rv_v, v, ngroups, n, 0u, 1, tg);
      share += top_share<K, 0u, 1>(key, ngroups, tg, eqs);
    }
    if (pass == 0 && (kWide || n1u != 0)) {
      // v' in u order replaces the rank row
      __syncthreads();
      if (active) merge_store_keys<K>(row, k0, key, 0xFFFFFFFFu);
      __syncthreads();
      if (n1u != 0) {
        // pairs inside u's tie runs: the long runs (listed last) by
        // networks, the others by the walk (rows longer than kDoubledMaxN,
        // whose plain ranks do not fit the network's keys, walk all runs)
        const uint64_t* rl = ru_v.runs + u * (ld / 2);
        const int nr = ru_v.nruns[u];
        const int nl = kWide ? 0 : ru_v.nlong[u];
        const uint32_t walked = nl > 0 ? (uint32_t)(rl[nr - nl] >> 32) : (uint32_t)n1u;
        share -= merge_tie_walk(ru_v, u, walked, row, tie);
        if (nl > 0) share -= merge_long_runs(rl + (nr - nl), nl, row, tie);
      }
      if constexpr (kWide) share += merge_cross_terms<K>(row, NR, scan);
      // the keys again from the row (not kept live across the in-run counts)
      if (active) merge_load_keys<K>(row, k0, key);
      // every walk and scan has read the row
      __syncthreads();
    }
    if constexpr (kWide) {
      // plain ranks r (0xFFFF past n) -> keys 2 min(r, 32767) in the first
      // pass, 2 max(r - 32768, 0) in the second
      const u16x2 lim = {(unsigned short)(kHalf - 1), (unsigned short)(kHalf - 1)};
      const u16x2 off = {(unsigned short)kHalf, (unsigned short)kHalf};
#pragma unroll
      for (int j = 0; j < KV; ++j) {
        const u16x2 r = pass == 0 ? __builtin_elementwise_min(key[j], lim)
                                  : __builtin_elementwise_sub_sat(key[j], off);
        key[j] = r + r;
      }
    }
    share += merge_count<K>(key, row, NR, active, k0, plane, closed);
  }
  nd = merge_block_sum(share, red);
  if (closed) {
    const uint32_t e = ngroups > 0 ? merge_block_sum(eqs, red) : 0u;
    const uint32_t c0 = e & 0xFFFFu, c1 = e >> 16, h = (uint32_t)s_top;
    nd += c0 * (c0 - 1u) / 2u + c1 * (c1 - 1u) / 2u - h * (h - 1u) / 2u;
  }
  n3 = n1u != 0 ? merge_block_sum(tie, red) : 0u;
  return true;
}

// Jobs [J_begin, J_end) of one matrix, one pair at a time per workgroup,
// grid-strided in job order (consecutive workgroups share u's row).
template <int K, bool kWide>
__global__ void __launch_bounds__(kMergeThreads) merge_jobs_kernel(MatDesc d) {
  extern __shared__ uint32_t merge_lds[];
  if (*d.status != 0) return;
  const int64_t count = d.J_end - d.J_begin;
  const int64_t budget = direct_budget(d.n);
  for (int64_t i = blockIdx.x; i < count; i += gridDim.x) {
    int64_t y, x;
    strict_pair(d.m, d.J_begin + i, y, x);
    uint32_t nd, n3;
    if (!pair_merge<K, kWide>(d.rv, y, d.rv, x, d.n, budget, merge_lds, nd, n3)) continue;
    if (threadIdx.x == 0) store_pair(d.out, i, d.n, d.rv.n1[y], d.rv.n1[x], nd, n3);
  }
}

// Workgroups a CU holds at once for each workgroup size (occupancy query,
// cached), and the number of CUs.  A launch has twice as many workgroups as
// the device holds, each striding over the jobs: the second half fills CUs
// whose first workgroups finish early (pair costs vary with their ties);
// measured 0-7% faster than exactly one full device.
template <int K, bool kWide>
struct MergeOccupancy {
  int per_cu[kMergeMaxWaves + 1] = {};
  int cus = 0;
  hipError_t err = hipSuccess;
  MergeOccupancy() {
    int dev = 0;
    err = hipGetDevice(&dev);
    if (err == hipSuccess)
      err = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (err == hipSuccess)
      err = hipFuncSetAttribute(reinterpret_cast<const void*>(merge_jobs_kernel<K, kWide>),
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)MergeShape<K>::lds_bytes(kMergeMaxWaves));
    for (int w = 1; w <= kMergeMaxWaves && err == hipSuccess; ++w) {
      int v = 0;
      err = hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &v, merge_jobs_kernel<K, kWide>, 64 * w, MergeShape<K>::lds_bytes(w));
      per_cu[w] = v < 1 ? 1 : v;
    }
  }
};

// Set up on the first use, outside any graph capture (prepare_pairs_merge).
template <int K, bool kWide>
const MergeOccupancy<K, kWide>& merge_occupancy() {
  static const MergeOccupancy<K, kWide> occ;
  return occ;
}

template <int K, bool kWide>
hipError_t merge_prepare_t() {
  return merge_occupancy<K, kWide>().err;
}

template <int K, bool kWide>
hipError_t merge_launch_t(const MatDesc& d, hipStream_t s) {
  using Shape = MergeShape<K>;
  const MergeOccupancy<K, kWide>& occ = merge_occupancy<K, kWide>();
  if (occ.err != hipSuccess) return occ.err;
  const int64_t count = d.J_end - d.J_begin;
  if (count < 1) return hipSuccess;
  const int waves = Shape::waves(d.n);
  if (waves < 1 || waves > kMergeMaxWaves) return hipErrorInvalidValue;
  const int64_t fill = 2 * (int64_t)occ.cus * occ.per_cu[waves];
  const int64_t grid = count < fill ? count : fill;
  hipLaunchKernelGGL((merge_jobs_kernel<K, kWide>), dim3((unsigned)grid), dim3(64 * waves),
                     Shape::lds_bytes(waves), s, d);
  return hipGetLastError();
}

}  // namespace

hipError_t prepare_pairs_merge(int scheme) {
  switch (scheme) {
    case kMergeK32: return merge_prepare_t<32, false>();
    case kMergeK64: {
      const hipError_t e = merge_prepare_t<64, false>();
      return e != hipSuccess ? e : merge_prepare_t<64, true>();
    }
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_pairs_merge(const MatDesc& d, hipStream_t s) {
  const bool wide = !ws_doubled(d.n);
  switch (d.scheme) {
    case kMergeK32:
      return wide ? hipErrorInvalidValue : merge_launch_t<32, false>(d, s);
    case kMergeK64:
      return wide ? merge_launch_t<64, true>(d, s) : merge_launch_t<64, false>(d, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ktau
