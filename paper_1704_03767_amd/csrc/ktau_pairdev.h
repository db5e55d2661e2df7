// Device routines shared by the pair kernels of every form (all-pairs,
// batched, query-vs-database): group primitives, the per-pair fast path
// (tagged bitonic count with the direct in-run tie correction), the
// composite path for two heavily tied rows, and the Step 5 / Eq. 1, 3 store.
// Internal to libktau.
#pragma once

#include <type_traits>

#include "ktau_bitonic.h"
#include "ktau_internal.h"

namespace ktau {
namespace {

constexpr int kBlock = 256;      // threads per workgroup for every pair kernel
constexpr int kWavesPerBlock = kBlock / 64;
// Grid cap of the job-order launches (256 CUs x 32 workgroups).
constexpr int64_t kMaxPairGrid = 8192;

// ---------------------------------------------------------------- utilities

template <int G>
__device__ __forceinline__ void group_sync() {
  if constexpr (G <= 64) {
    // inside one wave: LDS operations of a wave complete in order; this only
    // stops the compiler from moving LDS accesses across the point
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// Sum over the group; every lane of the group gets the total.
template <int G>
__device__ __forceinline__ uint32_t group_sum(uint32_t v, uint32_t* red) {
  if constexpr (G < 64) {
#pragma unroll
    for (int d = G / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
  } else {
    v = wave_sum(v);
    if constexpr (G == 64) {
      return v;
    } else {
      const int wave = threadIdx.x >> 6;
      __syncthreads();
      if ((threadIdx.x & 63) == 0) red[wave] = v;
      __syncthreads();
      uint32_t t = 0;
#pragma unroll
      for (int w = 0; w < G / 64; ++w) t += red[w];
      return t;
    }
  }
}

// K consecutive uint16 from a 2K-byte aligned address, by vector loads.
template <int K>
__device__ __forceinline__ void load_u16(const uint16_t* p, uint16_t (&out)[K]) {
  if constexpr (K == 2) {
    const uint32_t w = *(const uint32_t*)p;
    out[0] = (uint16_t)w;
    out[1] = (uint16_t)(w >> 16);
  } else if constexpr (K == 4) {
    const uint2 w = *(const uint2*)p;
    out[0] = (uint16_t)w.x;
    out[1] = (uint16_t)(w.x >> 16);
    out[2] = (uint16_t)w.y;
    out[3] = (uint16_t)(w.y >> 16);
  } else {
#pragma unroll
    for (int i = 0; i < K / 8; ++i) {
      const uint4 w = ((const uint4*)p)[i];
      const uint32_t a[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        out[8 * i + 2 * c] = (uint16_t)a[c];
        out[8 * i + 2 * c + 1] = (uint16_t)(a[c] >> 16);
      }
    }
  }
}

template <int K>
__device__ __forceinline__ void store_u16(uint16_t* p, const uint16_t (&in)[K]) {
#pragma unroll
  for (int i = 0; i < K / 2; ++i)
    ((uint32_t*)p)[i] = (uint32_t)in[2 * i] | ((uint32_t)in[2 * i + 1] << 16);
}

// K consecutive uint16 as K/2 packed words (element 2i low, 2i+1 high), from
// a 2K-byte aligned address.
template <int K>
__device__ __forceinline__ void load_words(const uint16_t* p, uint32_t (&w)[K / 2]) {
  if constexpr (K == 2) {
    w[0] = *(const uint32_t*)p;
  } else if constexpr (K == 4) {
    const uint2 a = *(const uint2*)p;
    w[0] = a.x;
    w[1] = a.y;
  } else {
#pragma unroll
    for (int i = 0; i < K / 8; ++i) {
      const uint4 a = ((const uint4*)p)[i];
      w[4 * i] = a.x;
      w[4 * i + 1] = a.y;
      w[4 * i + 2] = a.z;
      w[4 * i + 3] = a.w;
    }
  }
}

template <int K>
__device__ __forceinline__ void store_words(uint16_t* p, const uint32_t (&w)[K / 2]) {
  if constexpr (K == 2) {
    *(uint32_t*)p = w[0];
  } else if constexpr (K == 4) {
    *(uint2*)p = make_uint2(w[0], w[1]);
  } else {
#pragma unroll
    for (int i = 0; i < K / 8; ++i)
      ((uint4*)p)[i] = make_uint4(w[4 * i], w[4 * i + 1], w[4 * i + 2], w[4 * i + 3]);
  }
}

// Step 5 and Eq. 1/3: store the counts and tau of job slot `slot`.
__device__ __forceinline__ void store_pair(const PairOut& o, int64_t slot, int64_t n, int64_t n1y,
                                           int64_t n1x, uint32_t nd32, uint32_t n332) {
  const int64_t n0 = n * (n - 1) / 2;
  const int64_t nd = nd32, n3 = n332;
  const int64_t nc = n0 - n1y - n1x + n3 - nd;
  if (o.nc) o.nc[slot] = nc;
  if (o.nd) o.nd[slot] = nd;
  if (o.n3) o.n3[slot] = n3;
  const double num = (double)(nc - nd);
  if (o.tau_b) {
    const double d1 = (double)(n0 - n1y);
    const double d2 = (double)(n0 - n1x);
    const double prod = d1 * d2;
    const double den = sqrt(prod);
    o.tau_b[slot] = den == 0.0 ? __builtin_nan("") : num / den;
  }
  if (o.tau_a) o.tau_a[slot] = num / (double)n0;
}

// Counts of up to G finished pairs of one group, one pair per lane, so that
// the FP64 tau of Eq. 3 and the stores are issued once for all of them
// instead of once per pair.
template <int G>
struct Deferred {
  int cnt = 0;
  int64_t slot = 0, n1y = 0, n1x = 0;
  uint32_t nd = 0, n3 = 0;
  __device__ __forceinline__ void add(int lane, int64_t s, int64_t a, int64_t b, uint32_t d,
                                      uint32_t t) {
    if (lane == cnt) {
      slot = s;
      n1y = a;
      n1x = b;
      nd = d;
      n3 = t;
    }
    ++cnt;
  }
  __device__ __forceinline__ bool full() const { return cnt == G; }
  __device__ __forceinline__ void flush(int lane, const PairOut& o, int64_t n) {
    if (lane < cnt) store_pair(o, slot, n, n1y, n1x, nd, n3);
    cnt = 0;
  }
  template <class Store>
  __device__ __forceinline__ void flush_with(int lane, Store&& store) {
    if (lane < cnt) store(slot, n1y, n1x, nd, n3);
    cnt = 0;
  }
};

// ======================================================= main (fast) path

// One lane's walk over a stretch of the within-run pairs of u (positions in
// u's sorted order, values 2 v' in an LDS row).  Pairs of a run are numbered
// by the later position b, then the earlier a (index b(b-1)/2 + a), run after
// run; a pair adds to xin when the earlier value is larger and to tie when
// they are equal.
struct TieWalk {
  const uint64_t* rl;
  int lo;                                  // current run
  const uint16_t *pa, *pb, *ps, *pe;       // earlier, later, run start, run end
  uint32_t me, o;                          // values at pb and pa

  // Positions the walk at pair p (< the total number of pairs).
  __device__ __forceinline__ void init(const uint64_t* runs, int nruns, uint32_t p,
                                       const uint16_t* row) {
    rl = runs;
    int l = 0, h = nruns - 1;
    while (l < h) {   // the last run whose pair prefix is <= p
      const int mid = (l + h + 1) >> 1;
      if ((uint32_t)(rl[mid] >> 32) <= p) l = mid;
      else h = mid - 1;
    }
    lo = l;
    const uint64_t e = rl[l];
    const uint32_t start = (uint32_t)e & 0xFFFFu, len = ((uint32_t)(e >> 16) & 0xFFFFu) + 1u;
    const uint32_t qi = p - (uint32_t)(e >> 32);
    // b(b-1)/2 <= qi < b(b+1)/2 (a float estimate, then exact integer
    // fix-up).  In 32 bits: qi < 2^31 (a run of at most 65536 samples) keeps
    // the estimate at most 65536, whose b(b-1) still fits, and the first loop
    // leaves b <= 65535, so b(b+1) fits too.
    uint32_t b = (uint32_t)((1.0f + __fsqrt_rn(8.0f * (float)qi + 1.0f)) * 0.5f);
    while (b * (b - 1) / 2 > qi) --b;
    while (b * (b + 1) / 2 <= qi) ++b;
    const uint32_t a = qi - b * (b - 1) / 2;
    ps = row + start;
    pe = ps + len;
    pa = ps + a;
    pb = ps + b;
    me = *pb;
    o = *pa;
  }

  // Counts the current pair and moves to the next; `more` tells whether
  // another pair follows (then the next run exists when this one ends).  The
  // move to the next later position is branch-free (it happens every few
  // steps in some lane); only the end of a run branches.
  __device__ __forceinline__ void step(const uint16_t* row, bool more, uint32_t& xin,
                                       uint32_t& tie) {
    const uint32_t cur = o;
    xin += cur > me ? 1u : 0u;
    tie += cur == me ? 1u : 0u;
    ++pa;
    const bool wrap = pa == pb;
    pb = wrap ? pb + 1 : pb;
    pa = wrap ? ps : pa;
    if (pb == pe) {
      if (more) {
        const uint64_t e = rl[++lo];
        ps = row + ((uint32_t)e & 0xFFFFu);
        pe = ps + ((uint32_t)(e >> 16) & 0xFFFFu) + 1;
      }
      pa = ps;
      pb = ps + 1;
    }
    me = *pb;
    o = *pa;   // pa < pb: inside the row
  }
};

// Waves per SIMD that the register allocation of a fast-path kernel must
// allow (the second launch bound; the VGPR file holds 512 per lane): keys and
// gather indices take K VGPRs, so K = 128 is held to two waves, K = 64 to
// four, smaller K to five.
template <int K, int G>
constexpr int fast_waves() {
  return K >= 128 ? 2 : K >= 64 ? 4 : 5;
}

// LDS words per group: the v rank row (uint16), reused for v' on the tie
// path, plus the network's exchange buffer for 256-lane groups.  A
// workgroup's LDS is exactly its groups' words (so that, e.g., 16 groups of
// 1024 keys take 32 KB and five workgroups fit a CU), then for 256-lane groups
// the cross-wave reduction words and a 64-bit work-unit slot.
template <int K, int G>
struct FastLds {
  static constexpr int kRowWords = K * G / 2;
  static constexpr int kXWords = G == 256 ? bitonic::Net<K, G>::kXChunk * 256 : 0;
  static constexpr int kWords = kRowWords + kXWords;
  static constexpr int kGroups = kBlock / G;
  static constexpr int kBlockWords = kGroups * kWords + (G == 256 ? 8 : 0);
  static __device__ __forceinline__ uint32_t* red(uint32_t* lds) { return lds + kGroups * kWords; }
  static __device__ __forceinline__ int64_t* unit(uint32_t* lds) {
    return (int64_t*)(lds + kGroups * kWords + 4);
  }
};

// v'[k] = rank_v[perm_u[k]] for this lane's K sorted positions, from a rank
// row staged in LDS (row) and the lane's perm words (pw, byte offsets).
template <int K>
__device__ __forceinline__ void gather_keys(const uint16_t* row, const uint32_t (&pw)[K / 2],
                                            bitonic::u16x2 (&key)[K / 2]) {
  using bitonic::u16x2;
  constexpr int KV = K / 2;
  // v'[k] = rank_v[perm_u[k]], packed: VGPR j holds k0 + j and k0 + j + KV.
  // Workspace ranks are stored doubled, so the gathered values are already
  // the network's keys 2 v' (its tag goes in bit 0); row tails past n hold
  // perm[k] = 2k and 0xFFFE, the padding key.
  const char* rowb = (const char*)row;
#pragma unroll
  for (int j = 0; j < KV; ++j) {
    const uint32_t a = j % 2 ? pw[j / 2] >> 16 : pw[j / 2] & 0xFFFFu;
    const uint32_t b = (j + KV) % 2 ? pw[(j + KV) / 2] >> 16 : pw[(j + KV) / 2] & 0xFFFFu;
    u16x2 t;
    t.x = *(const uint16_t*)(rowb + a);
    t.y = *(const uint16_t*)(rowb + b);
    key[j] = t;
    // with 128 keys per lane, keep the scheduler from putting every gather
    // load in flight at once (each needs a register until it is packed)
    if constexpr (K >= 128)
      if (j % 16 == 15) __builtin_amdgcn_sched_barrier(0);
  }
}

// The counting network of a scheme: the half-precision one for groups of up
// to one wave (256-lane blocks, whose exchanges between waves go through
// LDS, keep the integer one).  Its lane mapping assigns each lane its K
// sorted positions.
template <int K, int G>
constexpr bool kHalfNet = G <= 64 && K >= 4 && K * G <= 8192;
template <int K, int G>
using PairNet = std::conditional_t<kHalfNet<K, G>, bitonic::NetS<K, G>, bitonic::Net<K, G>>;

// Tie groups of v up to which the top level's count is taken from global
// ranks instead of the network's last merge.
constexpr int kTopGroups = 2;
// Tie runs of u up to which a lane checks whether its positions meet one
// before writing them for the in-run walk.
constexpr int kFewRuns = 4;

// The last merge's count without the merge.  With A the first N/2 positions
// of u's order and B the rest, the last merge counts the pairs (a in A, b in
// B) with v_a > v_b.  A and B together are all of v, so with
// minrank(a) = #{x : v_x < v_a},
//     #{b in B : v_b < v_a} = minrank(a) - #{a' in A : v_a' < v_a},
// and summed over A the count is
//     sum over A of minrank(a) - C(|A|, 2) + ties(A),
// ties(A) being the pairs of A with equal v.  The keys of A are 2d (d the
// dense rank); for the tie groups of v (dense rank d_g, size m_g),
// minrank(a) = d(a) + sum_g (m_g - 1) [d(a) > d_g] and
// ties(A) = sum_g C(#{a in A : d(a) = d_g}, 2).  This returns the lane's
// share of the first sum (0 outside A) and, in eqs, its per-group counts of
// d(a) = d_g (16 bits per group).  The keys are kBias + d * 2^kShift
// (kShift >= 1), and the lane's K keys all belong to samples (no padding).
//
// Per group, with g = kBias + d_g * 2^kShift (keys differ from it by
// multiples of at least 2): at the lowest dense rank no key lies below the
// group, so sat(g + 1 - key) is 1 at the group and 0 above it and
// #above = K - #at; at the highest none lies above, and sat(key - (g - 1)) is
// 1 at the group and 0 below it; otherwise f = min(sat(key - (g - 1)), 2) is
// 0 below, 1 at and 2 above, and sum f = #at + 2 #above,
// sum f^2 = #at + 4 #above.
enum : int { kGroupInner = 0, kGroupLowest = 1, kGroupHighest = 2 };
struct TopGroups {
  uint32_t op[kTopGroups] = {};     // the comparison operand above, both halves
  uint32_t gm[kTopGroups] = {};     // m_g - 1
  int edge[kTopGroups] = {};        // kGroupInner / kGroupLowest / kGroupHighest
};

template <int K, uint32_t kBias, int kShift>
__device__ __forceinline__ uint32_t top_share(const bitonic::u16x2 (&key)[K / 2], int ngroups,
                                              const TopGroups& tg, uint32_t& eqs) {
  using bitonic::u16x2;
  using bitonic::vec;
  constexpr int KV = K / 2;
  constexpr uint32_t kOnes = 0x00010001u;
  uint32_t s2 = 0;
#pragma unroll
  for (int j = 0; j < KV; ++j) s2 = __builtin_amdgcn_udot2(key[j], vec(kOnes), s2, false);
  uint32_t share = (s2 - (uint32_t)K * kBias) >> kShift;
  eqs = 0;
#pragma unroll
  for (int g = 0; g < kTopGroups; ++g) {
    if (g >= ngroups) break;
    const u16x2 op = vec(tg.op[g]);
    uint32_t at = 0, above = 0;
    if (tg.edge[g] == kGroupLowest) {
#pragma unroll
      for (int j = 0; j < KV; ++j)
        at = __builtin_amdgcn_udot2(__builtin_elementwise_sub_sat(op, key[j]), vec(kOnes), at,
                                    false);
      above = (uint32_t)K - at;
    } else if (tg.edge[g] == kGroupHighest) {
#pragma unroll
      for (int j = 0; j < KV; ++j)
        at = __builtin_amdgcn_udot2(__builtin_elementwise_sub_sat(key[j], op), vec(kOnes), at,
                                    false);
    } else {
      uint32_t a1 = 0, a2 = 0;
#pragma unroll
      for (int j = 0; j < KV; ++j) {
        const u16x2 f = bitonic::pmin(__builtin_elementwise_sub_sat(key[j], op),
                                      vec(0x00020002u));
        a1 = __builtin_amdgcn_udot2(f, vec(kOnes), a1, false);   // at + 2 above
        a2 = __builtin_amdgcn_udot2(f, f, a2, false);            // at + 4 above
      }
      at = 2 * a1 - a2;
      above = (a2 - a1) >> 1;
    }
    share += tg.gm[g] * above;
    eqs |= at << (16 * g);
  }
  return share;
}

// The tie groups of row v (at most kTopGroups of them, ngroups in all, n
// samples) as top_share takes them: d_g is the group's dense rank (its run
// start less the surplus m - 1 of the runs before it); the highest dense
// rank is n - 1 less the surplus of all runs.
__device__ __forceinline__ void top_groups(const RankView& rv_v, int64_t v, int ngroups, int n,
                                           uint32_t kBias, int kShift, TopGroups& tg) {
  if (ngroups <= 0) return;
  const uint64_t* rl = rv_v.runs + v * (rv_v.ld / 2);
  uint32_t st[kTopGroups], ln[kTopGroups];
#pragma unroll
  for (int g = 0; g < kTopGroups; ++g) {
    const uint64_t e = g < ngroups ? rl[g] : 0ull;
    st[g] = (uint32_t)e & 0xFFFFu;
    ln[g] = ((uint32_t)(e >> 16) & 0xFFFFu) + 1u;
  }
  if (ngroups == 2 && st[1] < st[0]) {
    const uint32_t ts = st[0], tl = ln[0];
    st[0] = st[1];
    ln[0] = ln[1];
    st[1] = ts;
    ln[1] = tl;
  }
  const uint32_t d[kTopGroups] = {st[0], st[1] - (ln[0] - 1u)};
  const uint32_t dmax = (uint32_t)n - 1u - (ln[0] - 1u) - (ln[1] - 1u);
#pragma unroll
  for (int g = 0; g < kTopGroups; ++g) {
    const uint32_t k = kBias + (d[g] << kShift);
    tg.gm[g] = ln[g] - 1u;
    tg.edge[g] = d[g] == 0u ? kGroupLowest : d[g] == dmax ? kGroupHighest : kGroupInner;
    tg.op[g] = (tg.edge[g] == kGroupLowest ? k + 1u : k - 1u) * 0x00010001u;
  }
}

// n_d and n3 of one pair from its gathered keys: the direct in-run tie count
// over u's runs (when u has ties: the LDS row is overwritten with 2 v' in u
// order), then the network's inversion count less the inversions inside u
// runs.  The network's last merge is skipped when its count follows from
// v's global ranks (v has at most kTopGroups tie groups), or when the second
// half holds only padding (nothing to count).  Called by every lane of the
// group; rv_v / v / n give v's row and the number of samples.
template <int K, int G>
__device__ __forceinline__ void count_gathered(bitonic::u16x2 (&key)[K / 2], uint16_t* row,
                                               bool in_row, int k0, const RankView& ru_v,
                                               int64_t u, int64_t n1u, const RankView& rv_v,
                                               int64_t v, int n, uint32_t* xbuf,
                                               uint32_t* red, int lane, uint32_t& nd,
                                               uint32_t& n3) {
  constexpr bool kHalf = kHalfNet<K, G>;
  using Net = PairNet<K, G>;
  constexpr uint32_t kBias = kHalf ? bitonic::kHalfKeyBias : 0u;
  constexpr int kShift = kHalf ? bitonic::half_tag_bits(K * G) : 1;
  constexpr int KV = K / 2;
  const int64_t ld = ru_v.ld;
  uint32_t xin = 0, tie = 0;
  if (n1u != 0) {
    // 2 v' in u order replaces the rank row once every lane has gathered;
    // only the in-run positions are read from it, so with few runs a lane
    // whose positions meet none of them skips its store (the lanes' blocks
    // are 2K bytes apart, so their stores contend for the same LDS banks)
    const uint64_t* rl = ru_v.runs + u * (ld / 2);
    const int nr = ru_v.nruns[u];
    bool meets = true;
    if (nr <= kFewRuns) {
      meets = false;
#pragma unroll
      for (int r = 0; r < kFewRuns; ++r) {
        if (r < nr) {
          const uint64_t e = rl[r];
          const int st = (int)(e & 0xFFFFu), len = (int)((e >> 16) & 0xFFFFu) + 1;
          meets |= st < k0 + K && st + len > k0;
        }
      }
    }
    group_sync<G>();
    if (in_row && meets) {
      uint32_t w[KV];
      if constexpr (KV == 1) {
        w[0] = bitonic::bits(key[0]);
      } else {
#pragma unroll
        for (int i = 0; i < KV / 2; ++i) {
          // positions k0 + 2i, 2i + 1 (low halves), k0 + KV + 2i, 2i + 1 (high)
          w[i] = __builtin_amdgcn_perm(bitonic::bits(key[2 * i + 1]), bitonic::bits(key[2 * i]),
                                       0x05040100u);
          w[KV / 2 + i] = __builtin_amdgcn_perm(bitonic::bits(key[2 * i + 1]),
                                                bitonic::bits(key[2 * i]), 0x07060302u);
        }
      }
      store_words<K>(row + k0, w);
    }
    group_sync<G>();
    // The n1_u pairs of positions inside one tie run of u (Step 2), split
    // evenly into 2G stretches; lane l walks stretches l and l + G side by
    // side so that the LDS loads of the two walks overlap.
    const uint32_t total = (uint32_t)n1u;
    const uint32_t per = (total + 2 * G - 1) / (2 * G);
    const uint32_t p0 = (uint32_t)lane * per, p1 = (uint32_t)(lane + G) * per;
    const uint32_t c0 = p0 < total ? (total - p0 < per ? total - p0 : per) : 0u;
    const uint32_t c1 = p1 < total ? (total - p1 < per ? total - p1 : per) : 0u;
    if (c0 > 0) {
      TieWalk w0, w1;
      w0.init(rl, nr, p0, row);
      if (c1 > 0) w1.init(rl, nr, p1, row);
      for (uint32_t i = 0; i < c0; ++i) {
        w0.step(row, i + 1 < c0, xin, tie);
        if (i < c1) w1.step(row, i + 1 < c1, xin, tie);
      }
    }
  }
  // the last merge: counted by the network, from global ranks, or empty
  const bool pad_half = 2 * n <= Net::N;
  const int ngroups = pad_half ? 0 : rv_v.nruns[v];
  const bool closed = !pad_half && ngroups <= kTopGroups;
  // n_d = inversions - inversions inside u runs, summed in one reduction
  // (exact modulo 2^32)
  uint32_t share, eqs = 0;
  if (pad_half || closed) share = Net::template count_split<false>(key, lane, xbuf) - xin;
  else share = Net::template count_split<true>(key, lane, xbuf) - xin;
  if (closed) {
    TopGroups tg;
    top_groups(rv_v, v, ngroups, n, kBias, kShift, tg);
    const uint32_t t = top_share<K, kBias, kShift>(key, ngroups, tg, eqs);
    if (Net::logical_lane(lane) < G / 2) share += t;
    else eqs = 0;
  }
  nd = group_sum<G>(share, red);
  if (closed) {
    const uint32_t e = ngroups > 0 ? group_sum<G>(eqs, red) : 0u;
    const uint32_t c0 = e & 0xFFFFu, c1 = e >> 16, h = (uint32_t)Net::N / 2;
    nd += c0 * (c0 - 1u) / 2u + c1 * (c1 - 1u) / 2u - h * (h - 1u) / 2u;
  }
  n3 = n1u != 0 ? group_sum<G>(tie, red) : 0u;
}


// n_d and n3 of rows (y, x) unless both rows exceed the tie budget (then
// returns false and the composite pass handles the pair).  Called by every
// lane of the group with the same arguments.
template <int K, int G>
__device__ __forceinline__ bool pair_fast(const RankView& ry, int64_t y, const RankView& rx,
                                          int64_t x, int n, int64_t budget, uint32_t* lds,
                                          uint32_t* red, int lane, uint32_t& nd, uint32_t& n3) {
  using FL = FastLds<K, G>;
  using Net = PairNet<K, G>;
  using bitonic::u16x2;
  constexpr int KV = K / 2;
  const int64_t n1y = ry.n1[y], n1x = rx.n1[x];
  if (n1y > budget && n1x > budget) return false;
  // u: the row with fewer ties; both views share the row stride
  const bool swap = n1x < n1y;
  const RankView& ru_v = swap ? rx : ry;
  const RankView& rv_v = swap ? ry : rx;
  const int64_t u = swap ? x : y, v = swap ? y : x;
  const int64_t n1u = swap ? n1x : n1y;
  const int64_t ld = ry.ld;
  // this lane holds sorted positions k0 .. k0+K-1 (the network's element lane);
  // k0 passes through an empty asm so that the addresses formed from it are
  // formed for each pair, not held (or spilled) across the loop of pairs
  int k0 = Net::logical_lane(lane) * K;
  asm volatile("" : "+v"(k0));
  // vector loads stay inside the row (ld is a multiple of 128, so a lane is
  // either wholly inside or wholly past n)
  const bool in_row = k0 + K <= ld;
  uint16_t* row = (uint16_t*)lds;
  uint32_t* xbuf = lds + FL::kRowWords;
  // stage v's rank row in LDS (slots past the row get the padding key)
  if constexpr (K >= 8) {
    // 16-byte chunks dealt round-robin to the group's lanes, so that one
    // store instruction covers consecutive chunks (no bank conflicts)
    const uint4* src = (const uint4*)(rv_v.rank + v * ld);
    uint4* dst = (uint4*)row;
    if (K * G <= ld) {
      // every chunk inside the row: all loads in flight, then the stores
      uint4 w[K / 8];
#pragma unroll
      for (int i = 0; i < K / 8; ++i) w[i] = src[lane + G * i];
#pragma unroll
      for (int i = 0; i < K / 8; ++i) dst[lane + G * i] = w[i];
    } else {
#pragma unroll
      for (int i = 0; i < K / 8; ++i) {
        const int c = lane + G * i;
        dst[c] = 8 * c < ld ? src[c]
                            : make_uint4(0xFFFEFFFEu, 0xFFFEFFFEu, 0xFFFEFFFEu, 0xFFFEFFFEu);
      }
    }
  } else {
    uint32_t w[KV];
    if (in_row) {
      load_words<K>(rv_v.rank + v * ld + k0, w);
    } else {
#pragma unroll
      for (int i = 0; i < KV; ++i) w[i] = 0xFFFEFFFEu;
    }
    store_words<K>(row + k0, w);
  }
  // workspace perm entries are byte offsets into a rank row (2 x sample); a
  // lane wholly past the row gathers its own (padding) slots
  uint32_t pw[KV];
  if (in_row) {
    load_words<K>(ru_v.perm + u * ld + k0, pw);
  } else {
#pragma unroll
    for (int i = 0; i < KV; ++i)
      pw[i] = (uint32_t)(2 * (k0 + 2 * i)) | ((uint32_t)(2 * (k0 + 2 * i + 1)) << 16);
  }
  group_sync<G>();
  u16x2 key[KV];
  gather_keys<K>(row, pw, key);
  count_gathered<K, G>(key, row, in_row, k0, ru_v, u, n1u, rv_v, v, n, xbuf, red, lane, nd, n3);
  return true;
}

// ============================================ composite pass (LDS merge)

// In-lane: strict inversions among the lane's K keys, then a bitonic sorting
// network leaves them ascending (indices are compile-time, keys stay in
// registers).
template <int K>
__device__ __forceinline__ uint32_t lane_sort_count(uint32_t (&key)[K]) {
  uint32_t c = 0;
#pragma unroll
  for (int i = 0; i < K; ++i)
#pragma unroll
    for (int j = i + 1; j < K; ++j) c += key[i] > key[j] ? 1u : 0u;
#pragma unroll
  for (int size = 2; size <= K; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
#pragma unroll
      for (int i = 0; i < K; ++i) {
        const int j = i ^ stride;
        if (j > i) {
          const bool up = (i & size) == 0;
          uint32_t a = key[i], b = key[j];
          uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
          key[i] = up ? lo : hi;
          key[j] = up ? hi : lo;
        }
      }
    }
  }
  return c;
}

// buf holds 2*G*K + 16 keys.  On entry every lane's K keys are sorted; on exit
// the group's keys are sorted (lane-blocked) and the return value is this
// lane's share of the cross-lane inversions (Algorithm 2: a right-run key
// taken before left-run keys adds the number of left keys still waiting).
template <int K, int G>
__device__ __forceinline__ uint32_t merge_levels(uint32_t (&key)[K], uint32_t* buf, int lane) {
  constexpr int N = G * K;
  uint32_t cnt = 0;
  int cur = 0;
#pragma unroll 1
  for (int s = K; s < N; s <<= 1) {
    uint32_t* b = buf + cur * N;
#pragma unroll
    for (int r = 0; r < K; ++r) b[lane * K + r] = key[r];
    group_sync<G>();
    const int pos = lane * K;
    const int l0 = pos & ~(2 * s - 1);
    const int diag = pos - l0;
    const uint32_t* A = b + l0;
    // merge path: number of A keys among the first `diag` outputs, A first
    // on equal keys
    int lo = diag > s ? diag - s : 0;
    int hi = diag < s ? diag : s;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (A[mid] <= A[s + diag - 1 - mid]) lo = mid + 1;
      else hi = mid;
    }
    int ia = lo, ib = diag - lo;
    uint32_t a = ia < s ? A[ia] : kSentinel;
    uint32_t bb = ib < s ? A[s + ib] : kSentinel;
#pragma unroll
    for (int t = 0; t < K; ++t) {
      const bool takeB = bb < a;   // strict: equal keys are not discordant
      key[t] = takeB ? bb : a;
      cnt += takeB ? (uint32_t)(s - ia) : 0u;
      ia += takeB ? 0 : 1;
      ib += takeB ? 1 : 0;
      const int idx = takeB ? ib : ia;
      const uint32_t raw = A[takeB ? s + ib : ia];
      const uint32_t nv = idx < s ? raw : kSentinel;
      a = takeB ? a : nv;
      bb = takeB ? nv : bb;
    }
    cur ^= 1;
  }
  return cnt;
}

template <int K, int G>
__device__ __forceinline__ uint32_t sort_count(uint32_t (&key)[K], uint32_t* buf, int lane,
                                               uint32_t* red) {
  uint32_t c = lane_sort_count<K>(key);
  c += merge_levels<K, G>(key, buf, lane);
  return group_sum<G>(c, red);
}

template <int K, int G>
struct CompLds {
  static constexpr int kWords = 2 * G * K + 16;
};

// Both rows heavy: Step 1 literally (sort by (u run, v')), joint ties from
// equal composite keys, then Step 3 on v' alone.
template <int K, int G>
__device__ void pair_composite(const RankView& ry, int64_t y, const RankView& rx, int64_t x,
                               int n, uint32_t* buf, uint32_t* red, int lane, uint32_t& nd,
                               uint32_t& n3) {
  const bool swap = rx.n1[x] < ry.n1[y];
  const RankView& ru_v = swap ? rx : ry;
  const RankView& rv_v = swap ? ry : rx;
  const int64_t u = swap ? x : y, v = swap ? y : x;
  const int64_t ld = ry.ld;
  const uint16_t* pu = ru_v.perm + u * ld;
  const uint16_t* rk = rv_v.rank + v * ld;
  const uint16_t* ru = ru_v.rstart + u * ld;
  const int k0 = lane * K;
  uint32_t key[K];
#pragma unroll
  for (int r = 0; r < K; ++r) {
    const int k = k0 + r;
    key[r] = k < n ? ((uint32_t)ru[k] << 16) | (uint32_t)rk[pu[k] >> 1] : kPadKey;
  }
  (void)sort_count<K, G>(key, buf, lane, red);
  // joint ties: in the (u, v)-sorted sequence, sum over positions of the
  // number of earlier positions holding an equal composite key.  The last
  // merge level (log2 G of them, an even number) read region 1, so region 0
  // is free.
  uint32_t* sb = buf;
#pragma unroll
  for (int r = 0; r < K; ++r) sb[k0 + r] = key[r];
  group_sync<G>();
  uint32_t tie = 0;
#pragma unroll
  for (int r = 0; r < K; ++r) {
    const int k = k0 + r;
    if (k < n) {
      int lo = 0, hi = k;   // first position holding a key equal to key[r]
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (sb[mid] < key[r]) lo = mid + 1;
        else hi = mid;
      }
      tie += (uint32_t)(k - lo);
    }
  }
  n3 = group_sum<G>(tie, red);
#pragma unroll
  for (int r = 0; r < K; ++r)
    if (key[r] != kPadKey) key[r] &= 0xFFFFu;
  group_sync<G>();
  nd = sort_count<K, G>(key, buf, lane, red);
}

}  // namespace
}  // namespace ktau
