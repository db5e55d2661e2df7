// Register-resident inversion count for the pair kernels (the Step 3 count of
// Sec. 3.2, Algorithm 2, computed with a different merge schedule).
//
// A group of G lanes (8, 16 or 32 lanes of a wave, a whole wave, or a
// 256-lane workgroup) holds N = G*K keys, K per lane, lane-blocked (element
// e = lane*K + r).  Keys are 16-bit, twice a dense rank, packed two per VGPR:
// VGPR j holds elements r = j (low half) and r = j + K/2 (high half).
//
// The sort is a bitonic network, level L merging sorted blocks of s = 2^L
// into blocks of 2s.  Exactly as in Algorithm 2, the count of a level is, over
// every block, the number of (left-half element, right-half element) pairs
// whose left element is strictly larger.  It is read off the merged block
// without comparing pairs: before the level every key is tagged in its least
// significant bit with the half it comes from (key' = 2*rank + tag), so the
// network sorts equal ranks left-half first; a right-half element that lands
// at ascending position p of its merged block, as the j-th of its half, has
// exactly p - j left elements at or below it.  Summing over the block,
//     inversions = s*s + s(s-1)/2 - (sum of positions of right-half elements),
// and one v_dot2_u32_u16 per VGPR accumulates that position sum.
//
// Bitonic merging needs every other block sorted descending.  Instead of
// selecting min or max per lane, keys of a descending block are stored
// complemented, so every comparator of every stage keeps the minimum at the
// lower position; a complemented block's physical position q is ascending
// position 2s-1-q, which flips the sign of its term (see levels).
//
// Partners at distance d:  d < K/2 -> another VGPR of the same lane (one
// v_pk_min_u16 + one v_pk_max_u16 for two comparators);  d = K/2 -> the two
// halves of one VGPR;  d >= K: another lane.  Physical lane bits 0-3 use
// ds_swizzle plus a masked select; bits 4 and 5 use v_permlane16_swap /
// v_permlane32_swap, which exchange half the lanes of two VGPRs so that the
// comparison becomes a plain min/max between the two registers (swapped back
// afterwards); waves of a 256-lane group exchange through LDS.  In whole-wave
// groups the two most used element lane bits (the lowest) are placed on
// physical bits 4 and 5, which saves LDS swizzles.
#pragma once

#include "ktau_internal.h"

namespace ktau {
namespace bitonic {

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t bits(u16x2 v) { return __builtin_bit_cast(uint32_t, v); }
__device__ __forceinline__ u16x2 vec(uint32_t v) { return __builtin_bit_cast(u16x2, v); }
__device__ __forceinline__ u16x2 pmin(u16x2 a, u16x2 b) { return __builtin_elementwise_min(a, b); }
__device__ __forceinline__ u16x2 pmax(u16x2 a, u16x2 b) { return __builtin_elementwise_max(a, b); }

constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v >> 1); }

// Value of lane ^ M (M < 32) by ds_swizzle in bit-mask mode.
template <int M>
__device__ __forceinline__ uint32_t lane_xor(uint32_t v) {
  static_assert(M > 0 && M < 32, "swizzle reaches 32 lanes");
  return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, (M << 10) | 0x1F);
}

// a ^ b ^ c in one v_bitop3_b32 (the compiler folds a ^ (a & m) into an AND
// with a literal and then spends a second instruction on c); c is a scalar
// operand where it is the same in every lane.
template <bool kScalarC>
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t r;
  if constexpr (kScalarC)
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(c));
  else
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}

template <int K, int G>
struct Net {
  static constexpr int KV = K / 2;            // VGPRs per lane
  static constexpr int LOGK = ilog2(K);
  static constexpr int LOGKV = ilog2(KV);
  static constexpr int LOGG = ilog2(G);
  static constexpr int LOGN = LOGK + LOGG;
  static constexpr int N = K * G;
  // VGPRs exchanged per LDS round across the waves of a 256-lane group (the
  // exchange buffer holds kXChunk * G words)
  static constexpr int kXChunk = KV < 16 ? KV : K >= 128 ? 8 : 16;
  static_assert(K >= 2 && K <= 128 && (K & (K - 1)) == 0, "K is a power of two <= 128");
  // Lane-spanning levels accumulate sum(raw * r) below bit kWShift and the
  // number of raw tags above it (sum of r < K is at most K(K-1)/2).
  static constexpr int kWShift = K <= 64 ? 12 : 14;
  static_assert(K * (K - 1) / 2 < (1 << kWShift), "weight field");
  static_assert(G == 8 || G == 16 || G == 32 || G == 64 || G == 256,
                "part of a wave, a wave or a 256-lane workgroup");

  // Physical lane bit of element lane bit lb (measured: worth it for whole
  // waves, not for 32-lane groups).
  static constexpr int phys_bit(int lb) {
    if constexpr (G >= 64) return lb == 0 ? 4 : lb == 1 ? 5 : lb < 6 ? lb - 2 : lb;
    return lb;
  }
  // The element lane (the group's K-key block) held by physical lane `lane`.
  static __device__ __forceinline__ int logical_lane(int lane) {
    if constexpr (G < 64) {
      return lane;
    } else {
      int l = 0;
#pragma unroll
      for (int b = 0; b < LOGG; ++b) l |= ((lane >> phys_bit(b)) & 1) << b;
      return l;
    }
  }

  // Bit b of element (lane, j, h); `lane` is the element lane.
  static __device__ __forceinline__ uint32_t ebit(int lane, int j, int h, int b) {
    const uint32_t e = ((uint32_t)lane << LOGK) | ((uint32_t)h << LOGKV) | (uint32_t)j;
    return (e >> b) & 1u;
  }
  // All ones in lanes whose bit lb is clear (the lower partner of a stage).
  static __device__ __forceinline__ uint32_t lane_mask(int lane, int lb) {
    return (uint32_t)(((lane >> lb) & 1) - 1);
  }
  static __device__ __forceinline__ uint32_t half_mask(uint32_t lo, uint32_t hi) {
    return (lo ? 0xFFFFu : 0u) | (hi ? 0xFFFF0000u : 0u);
  }

  // One comparator stage on element bit k (partners e and e ^ 2^k); `lane`
  // is the element lane, `plane` the physical lane.
  template <int k>
  static __device__ __forceinline__ void stage(u16x2 (&v)[KV], int lane, int plane,
                                               uint32_t* xbuf) {
    if constexpr (k < LOGKV) {
#pragma unroll
      for (int j = 0; j < KV; ++j) {
        if ((j >> k) & 1) continue;
        const int p = j | (1 << k);
        const u16x2 a = v[j], b = v[p];
        v[j] = pmin(a, b);
        v[p] = pmax(a, b);
      }
    } else if constexpr (k == LOGKV) {
#pragma unroll
      for (int j = 0; j < KV; ++j) {
        const u16x2 t = __builtin_shufflevector(v[j], v[j], 1, 0);
        const u16x2 mn = pmin(v[j], t), mx = pmax(v[j], t);
        v[j] = __builtin_shufflevector(mn, mx, 0, 3);
      }
    } else {
      constexpr int lb = k - LOGK;            // element lane bit
      constexpr int pb = phys_bit(lb);        // physical lane bit
      if constexpr (pb < 4) {
        // the lower lane keeps the minimum; a bit mask in a VGPR selects it
        // (no per-lane condition has to live in scalar registers)
        const uint32_t keep_min = lane_mask(lane, lb);
#pragma unroll
        for (int j = 0; j < KV; ++j) {
          const u16x2 p = vec(lane_xor<(1 << pb)>(bits(v[j])));
          const u16x2 mn = pmin(v[j], p), mx = pmax(v[j], p);
          v[j] = vec((bits(mn) & keep_min) | (bits(mx) & ~keep_min));
        }
      } else if constexpr (pb == 4 || pb == 5) {
        if constexpr (KV >= 2) {
#pragma unroll
          for (int j = 0; j < KV; j += 2) {
            uint32_t a = bits(v[j]), b = bits(v[j + 1]);
            if constexpr (pb == 4) {
              auto s = __builtin_amdgcn_permlane16_swap(a, b, false, false);
              a = s[0];
              b = s[1];
            } else {
              auto s = __builtin_amdgcn_permlane32_swap(a, b, false, false);
              a = s[0];
              b = s[1];
            }
            const u16x2 mn = pmin(vec(a), vec(b)), mx = pmax(vec(a), vec(b));
            a = bits(mn);
            b = bits(mx);
            if constexpr (pb == 4) {
              auto s = __builtin_amdgcn_permlane16_swap(a, b, false, false);
              v[j] = vec(s[0]);
              v[j + 1] = vec(s[1]);
            } else {
              auto s = __builtin_amdgcn_permlane32_swap(a, b, false, false);
              v[j] = vec(s[0]);
              v[j + 1] = vec(s[1]);
            }
          }
        } else {
          // a single VGPR: exchange with itself, keep the partner's copy
          const bool lower = ((lane >> lb) & 1) == 0;
          uint32_t a = bits(v[0]);
          uint32_t part;
          if constexpr (pb == 4) {
            auto s = __builtin_amdgcn_permlane16_swap(a, a, false, false);
            part = lower ? (uint32_t)s[1] : (uint32_t)s[0];
          } else {
            auto s = __builtin_amdgcn_permlane32_swap(a, a, false, false);
            part = lower ? (uint32_t)s[1] : (uint32_t)s[0];
          }
          const uint32_t keep_min = lane_mask(lane, lb);
          const u16x2 mn = pmin(v[0], vec(part)), mx = pmax(v[0], vec(part));
          v[0] = vec((bits(mn) & keep_min) | (bits(mx) & ~keep_min));
        }
      } else {
        // across the waves of a 256-lane group, through LDS, kXChunk VGPRs
        // at a time
        const uint32_t keep_min = lane_mask(lane, lb);
#pragma unroll
        for (int j0 = 0; j0 < KV; j0 += kXChunk) {
#pragma unroll
          for (int j = 0; j < kXChunk; ++j) xbuf[j * G + plane] = bits(v[j0 + j]);
          __syncthreads();
#pragma unroll
          for (int j = 0; j < kXChunk; ++j) {
            const u16x2 p = vec(xbuf[j * G + (plane ^ (1 << pb))]);
            const u16x2 mn = pmin(v[j0 + j], p), mx = pmax(v[j0 + j], p);
            v[j0 + j] = vec((bits(mn) & keep_min) | (bits(mx) & ~keep_min));
          }
          __syncthreads();
        }
      }
    }
  }

  template <int L, int k>
  static __device__ __forceinline__ void stages_down(u16x2 (&v)[KV], int lane, int plane,
                                                     uint32_t* xbuf) {
    stage<k>(v, lane, plane, xbuf);
    if constexpr (k > 0) stages_down<L, k - 1>(v, lane, plane, xbuf);
  }

  // Tag-and-orientation constant of level L for VGPR j: tag = bit L of e (the
  // half of the 2s block), complemented iff bit L+1 of e (a descending
  // block).  The previous level stored key' ^ orient(bit L); working the
  // cases through, the new key is (old & 0xFFFE) ^ c with
  // c = (bit L != bit L+1 ? 0xFFFF : 0) per half, and level 0 starts from
  // untagged ascending keys 2*rank with c = tag ^ orient.
  template <int L>
  static __device__ __forceinline__ uint32_t tag_const(int lane, int j) {
    if constexpr (L == 0) {
      const uint32_t t0 = ebit(lane, j, 0, 0), t1 = ebit(lane, j, 1, 0);
      return (t0 | (t1 << 16)) ^ half_mask(ebit(lane, j, 0, 1), ebit(lane, j, 1, 1));
    } else {
      return half_mask(ebit(lane, j, 0, L) ^ (L + 1 < LOGN ? ebit(lane, j, 0, L + 1) : 0u),
                       ebit(lane, j, 1, L) ^ (L + 1 < LOGN ? ebit(lane, j, 1, L + 1) : 0u));
    }
  }

  // The count of level L is a sum over right-half elements of their
  // ascending position in the merged block (see the top of this file).  With
  // raw = the stored tag bit after the merge and q the physical position in
  // the 2s block, a complemented block's elements have tag 1 - raw and
  // ascending position 2s-1-q, and the level's term works out to
  //   (sum of q over the lane's elements of complemented blocks) - sum raw*q,
  // i.e. a per-lane constant minus one dot product of the raw tag bits.
  // Blocks inside a lane: q depends on (j, half) only, so the constants and
  // weights are compile-time.  Blocks spanning lanes: q = base + r (r = index
  // in the lane, base the lane's offset in its block); the weights
  // r + 2^kWShift give sum raw*r (below bit kWShift) and the number of raw
  // tags (above it) in one accumulator.
  static constexpr uint32_t in_lane_weight(int L, int j) {
    const uint32_t m2s = (2u << L) - 1u;
    return ((uint32_t)j & m2s) | (((uint32_t)(j + KV) & m2s) << 16);
  }
  static constexpr uint32_t in_lane_const() {
    // sum over in-lane levels of the positions of complemented elements
    uint32_t c = 0;
    for (int L = 0; L + 1 < LOGK; ++L)
      for (int r = 0; r < K; ++r)
        if ((r >> (L + 1)) & 1) c += (uint32_t)r & ((2u << L) - 1u);
    return c;
  }

  // Level L: its comparator stages, its count, and the re-tag for level L+1
  // (one AND, one dot product and one XOR per VGPR).
  template <int L, int kEnd = LOGN>
  static __device__ __forceinline__ void levels(u16x2 (&v)[KV], int lane, int plane,
                                                uint32_t* xbuf, uint32_t& acc_in,
                                                uint32_t& total) {
    stages_down<L, L>(v, lane, plane, xbuf);
    uint32_t acc = 0;
#pragma unroll
    for (int j = 0; j < KV; ++j) {
      const uint32_t t = bits(v[j]) & 0x00010001u;
      if constexpr (L + 1 < LOGK) {
        const uint32_t w = in_lane_weight(L, j);
        if (w != 0u) acc_in = __builtin_amdgcn_udot2(vec(t), vec(w), acc_in, false);
      } else {
        constexpr uint32_t kW = 1u << kWShift;
        const uint32_t w = ((uint32_t)j + kW) | (((uint32_t)(j + KV) + kW) << 16);
        acc = __builtin_amdgcn_udot2(vec(t), vec(w), acc, false);
      }
      // the re-tag word depends on the lane once bit L+2 is a lane bit
      if constexpr (L + 1 < LOGN)
        v[j] = vec(xor3<(L + 2 < LOGK)>(bits(v[j]), t, tag_const<L + 1>(lane, j)));
    }
    if constexpr (L + 1 >= LOGK) {
      // the lane lies inside one block of 2s: its offset and orientation
      const uint32_t base = ((uint32_t)lane & ((1u << (L + 1 - LOGK)) - 1u)) << LOGK;
      const uint32_t raw = (acc & ((1u << kWShift) - 1u)) + base * (acc >> kWShift);
      const uint32_t desc =
          (L + 1 < LOGN) ? (uint32_t)(lane >> (L + 1 - LOGK)) & 1u : 0u;
      const uint32_t all = (uint32_t)K * base + (uint32_t)(K * (K - 1) / 2);
      total += (all & (0u - desc)) - raw;
    }
    if constexpr (L + 1 < kEnd) levels<L + 1, kEnd>(v, lane, plane, xbuf, acc_in, total);
  }

  // Constant part of all levels: a level with nb >= 2 blocks of 2s adds
  // (nb/2) * s^2 (half the blocks ascending, half descending); the top level
  // (one ascending block) adds s^2 + s(s-1)/2.
  static constexpr uint32_t constant_part() {
    uint64_t c = 0;
    for (int L = 0; L < LOGN; ++L) {
      const uint64_t s = 1ull << L;
      const uint64_t nb = (uint64_t)N / (2 * s);
      c += nb >= 2 ? (nb / 2) * s * s : s * s + s * (s - 1) / 2;
    }
    return (uint32_t)c;
  }

  // The top level's term in constant_part (one ascending block of 2s = N).
  static constexpr uint32_t top_const() {
    const uint64_t s = (uint64_t)N / 2;
    return (uint32_t)(s * s + s * (s - 1) / 2);
  }

  // As count, with the top level (the merge of the two halves of N/2) run
  // only when kTop is set.  Without it the share leaves out that level's
  // count, and the keys end as the two sorted halves re-tagged for the top
  // level: the first half (element lanes below G/2) ascending and untagged,
  // i.e. exactly 2*rank.
  template <bool kTop>
  static __device__ __forceinline__ uint32_t count_split(u16x2 (&v)[KV], int plane,
                                                         uint32_t* xbuf) {
    asm volatile("" : "+v"(plane));   // per-lane words formed here, not hoisted
    const int lane = logical_lane(plane);
#pragma unroll
    for (int j = 0; j < KV; ++j) v[j] = vec(bits(v[j]) ^ tag_const<0>(lane, j));
    uint32_t acc_in = 0, total = in_lane_const();
    levels<0, kTop ? LOGN : LOGN - 1>(v, lane, plane, xbuf, acc_in, total);
    total -= acc_in;
    if (plane == 0) total += kTop ? constant_part() : constant_part() - top_const();
    return total;
  }

  // v: packed keys 2*rank (padding 0xFFFE) of element lane logical_lane(plane),
  // sorted in place; plane is the lane's index in the group.  Returns this
  // lane's share of the group's strict inversion count (the constant part is
  // added by lane 0 of the group), modulo 2^32.
  static __device__ __forceinline__ uint32_t count(u16x2 (&v)[KV], int plane, uint32_t* xbuf) {
    const int lane = logical_lane(plane);
#pragma unroll
    for (int j = 0; j < KV; ++j) v[j] = vec(bits(v[j]) ^ tag_const<0>(lane, j));
    uint32_t acc_in = 0, total = in_lane_const();
    levels<0>(v, lane, plane, xbuf, acc_in, total);
    total -= acc_in;
    if (plane == 0) total += constant_part();
    return total;
  }
};


// Bias of the half-precision keys: the smallest normal f16 pattern.
constexpr uint32_t kHalfKeyBias = 0x0400u;

// Tag bits held below the rank in the half-precision keys of an N-key
// network: the most (up to 5) for which padding with a full field,
// 0x0400 + (N + 1) 2^T - 1, is still a finite f16 pattern (4 for 1024 keys,
// 1 for 8192).
constexpr int half_tag_bits(int N) {
  int t = 1;
  while (t < 5 && (uint32_t)(N + 1) * (2u << t) + kHalfKeyBias - 1u <= 0x7BFFu) ++t;
  return t;
}

// (a & b) ^ c in one v_bitop3_b32, b in a scalar register.
__device__ __forceinline__ uint32_t and_xor(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t r;
  asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x6a" : "=v"(r) : "v"(a), "s"(b), "v"(c));
  return r;
}

// The same count with keys held as half-precision bit patterns, for groups of
// at most 8192 keys.  A key is the positive normal f16 pattern
// 0x0400 + rank * 2^T + field, T = half_tag_bits(N): the rank decides every
// comparison between different ranks, and the T-bit field below it holds the
// tags of T levels at once (a tag epoch): bit i is the element's position bit
// of the epoch's i-th level, taken at the epoch's first level (bits at and
// above a level's stay fixed until that level's merge).  Equal ranks are then
// ordered by the current level's tag: earlier levels' tags sit below it, and
// later levels' tags are equal across a block.  So keys are re-tagged once per
// epoch, not once per level.  The packed f16 minimum orders the keys as
// integers do, and flipping the sign bit reverses the order.
//
// Level 0 is counted directly (each pair compared before its exchange).  The
// other levels inside one half of a lane's VGPRs (register stages only) keep
// every block ascending: a level's first stage pairs each position with its
// mirror in the block, the rest are half-cleaners, and no sign is used.  From
// the half stage's level on (its first stage mirrored as well) the sign bit
// carries two things:
//   * the orientation of a descending block (in place of the complement);
//   * a per-stage pattern: in a stage whose partner sits in another lane or
//     in the other half of the VGPR, the upper partner is held negated, so
//     that both partners compute min(own, -partner) -- the lower one gets the
//     minimum, the upper one minus the maximum -- in one v_pk_minimum3_f16
//     with the negation (and, within a VGPR, the half swap) folded into the
//     operand modifiers.  Changing the pattern between two such stages costs
//     one XOR per VGPR, against the two extra operations (max and select) of
//     the plain form.
// Register stages keep min/max pairs and need both partners' signs equal;
// the permlane stages need them equal and positive.  After the half stage the
// high halves stay negated, so the register stages sort them descending: from
// that level on, a lane's high halves hold its upper K/2 elements in reverse
// order (element K-1-j in VGPR j).  Register and lane stages pair the same
// VGPRs under that numbering; half stages pair VGPR j with VGPR KV-1-j (at the
// half stage's own level that is the mirror of an ascending 64-element
// block), and the count's position weights follow it.

template <int K, int G>
struct NetS {
  using B = Net<K, G>;
  static constexpr int KV = B::KV, LOGK = B::LOGK, LOGKV = B::LOGKV, LOGG = B::LOGG;
  static constexpr int LOGN = B::LOGN, N = B::N, kXChunk = B::kXChunk, kWShift = B::kWShift;
  static_assert(N <= 8192, "keys 0x0400 + rank * 2^T + field stay finite");
  static_assert(KV >= 2, "level 0 pairs two VGPRs");
  static constexpr int kT = half_tag_bits(N);
  static constexpr uint32_t kField = ((1u << kT) - 1u) * 0x00010001u;
  static constexpr uint32_t kSign = 0x80008000u;
  typedef _Float16 h2 __attribute__((ext_vector_type(2)));

  static __device__ __forceinline__ h2 hv(uint32_t x) { return __builtin_bit_cast(h2, x); }
  static __device__ __forceinline__ uint32_t hu(h2 x) { return __builtin_bit_cast(uint32_t, x); }
  // IEEE minimum / maximum: one instruction each, no quieting of the inputs
  // (every key is a finite normal number)
  static __device__ __forceinline__ uint32_t fmn(uint32_t a, uint32_t b) {
    return hu(__builtin_elementwise_minimum(hv(a), hv(b)));
  }
  static __device__ __forceinline__ uint32_t fmx(uint32_t a, uint32_t b) {
    return hu(__builtin_elementwise_maximum(hv(a), hv(b)));
  }
  // min(a, -b); min(a, -(b with its halves swapped))
  static __device__ __forceinline__ uint32_t fmn_neg(uint32_t a, uint32_t b) {
    return hu(__builtin_elementwise_minimum(hv(a), -hv(b)));
  }
  static __device__ __forceinline__ uint32_t fmn_neg_swapped(uint32_t a, uint32_t b) {
    const h2 y = hv(b);
    return hu(__builtin_elementwise_minimum(hv(a), -__builtin_shufflevector(y, y, 1, 0)));
  }

  // Tag epochs start at level 1, every kT levels inside a half, at the half
  // stage's level LOGKV, and every kT levels after it.
  static constexpr bool epoch_start(int L) {
    if (L == 1 || L == LOGKV) return true;
    return L < LOGKV ? (L - 1) % kT == 0 : (L - LOGKV) % kT == 0;
  }
  static constexpr int epoch_of(int L) {
    int s = L;
    while (!epoch_start(s)) --s;
    return s;
  }
  // Field of an epoch starting at level S < LOGKV (tags inside a half only:
  // the same in both halves and every lane).
  static constexpr uint32_t half_field(int S, int j) {
    const int w = kT < LOGKV - S ? kT : LOGKV - S;
    return (((uint32_t)j >> S) & ((1u << w) - 1u)) * 0x00010001u;
  }
  // Field of an epoch starting at level S >= LOGKV, both halves.
  static __device__ __forceinline__ uint32_t field_word(int S, int lane, int j) {
    uint32_t c = 0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint32_t e = ((uint32_t)lane << LOGK) | ((uint32_t)h << LOGKV) | (uint32_t)j;
      c |= ((e >> S) & ((1u << kT) - 1u)) << (16 * h);
    }
    return c;
  }

  // Element lane bit lb sits on physical lane bit lb: bits 0-4 exchange by
  // ds_swizzle (one minimum per VGPR under a sign pattern), bit 5 of a whole
  // wave by v_permlane32_swap (a minimum and a maximum per two VGPRs, signs
  // plain); bit 5 is the top level's, which is mostly taken from global
  // ranks.  (The integer network puts its most used lane bits on the permlane
  // swaps instead.)
  static constexpr int phys_bit(int lb) { return lb; }
  static __device__ __forceinline__ int logical_lane(int plane) { return plane; }

  // Stage on element bit k: takes a sign pattern (the upper partner negated)
  // or needs both partners positive (permlane stages); register stages take
  // whatever signs their partners share.
  static constexpr bool patterned(int k) {
    return k == LOGKV || (k >= LOGK && phys_bit(k - LOGK) != 5);
  }
  static constexpr bool wants_plain(int k) { return k >= LOGK && !patterned(k); }

  // Sign bits of the pattern keyed on element bit b (b < 0: none), for the
  // element lane `lane`; b is the half bit or a lane bit.
  static __device__ __forceinline__ uint32_t pattern(int lane, int b) {
    if (b < 0) return 0u;
    if (b == LOGKV) return 0x80000000u;
    return ((lane >> (b - LOGK)) & 1) ? kSign : 0u;
  }

  // A stage of a level L >= LOGKV.
  template <int L, int k>
  static __device__ __forceinline__ void stage(uint32_t (&v)[KV], int lane, int plane,
                                               uint32_t* xbuf) {
    if constexpr (k < LOGKV) {
#pragma unroll
      for (int j = 0; j < KV; ++j) {
        if ((j >> k) & 1) continue;
        const int p = j | (1 << k);
        const uint32_t a = v[j], b = v[p];
        v[j] = fmn(a, b);
        v[p] = fmx(a, b);
      }
    } else if constexpr (k == LOGKV) {
      // VGPR j's low half meets VGPR KV-1-j's high half and the reverse
#pragma unroll
      for (int j = 0; j < KV / 2; ++j) {
        const uint32_t a = v[j], b = v[KV - 1 - j];
        v[j] = fmn_neg_swapped(a, b);
        v[KV - 1 - j] = fmn_neg_swapped(b, a);
      }
    } else {
      constexpr int lb = k - LOGK;
      constexpr int pb = phys_bit(lb);
      if constexpr (pb < 5) {
#pragma unroll
        for (int j = 0; j < KV; ++j) v[j] = fmn_neg(v[j], lane_xor<(1 << pb)>(v[j]));
      } else if constexpr (pb == 5) {
        // two VGPRs at a time: the swap brings both partners into one lane,
        // which keeps the minimum in one VGPR and the maximum in the other,
        // and the swap back returns them (signs plain: both positive or both
        // negated by the block's orientation)
#pragma unroll
        for (int j = 0; j < KV; j += 2) {
          auto s = __builtin_amdgcn_permlane32_swap(v[j], v[j + 1], false, false);
          const uint32_t a = s[0], b = s[1];
          auto r = __builtin_amdgcn_permlane32_swap(fmn(a, b), fmx(a, b), false, false);
          v[j] = r[0];
          v[j + 1] = r[1];
        }
      } else {
#pragma unroll
        for (int j0 = 0; j0 < KV; j0 += kXChunk) {
#pragma unroll
          for (int j = 0; j < kXChunk; ++j) xbuf[j * G + plane] = v[j0 + j];
          __syncthreads();
#pragma unroll
          for (int j = 0; j < kXChunk; ++j)
            v[j0 + j] = fmn_neg(v[j0 + j], xbuf[j * G + (plane ^ (1 << pb))]);
          __syncthreads();
        }
      }
    }
  }

  // Stages k .. 0 of a level L >= LOGKV; `cur` is the element bit the current
  // sign pattern is keyed on (-1: none).
  template <int L, int k, int cur>
  static __device__ __forceinline__ void stages_down(uint32_t (&v)[KV], int lane, int plane,
                                                     uint32_t* xbuf) {
    constexpr int want = patterned(k) ? k : wants_plain(k) ? -1 : cur;
    if constexpr (want != cur) {
      const uint32_t m = pattern(lane, cur) ^ pattern(lane, want);
#pragma unroll
      for (int j = 0; j < KV; ++j) v[j] ^= m;
    }
    stage<L, k>(v, lane, plane, xbuf);
    if constexpr (k > 0) stages_down<L, k - 1, want>(v, lane, plane, xbuf);
  }

  // Sign bit of element (lane, j, h) at the start of level L >= LOGKV
  // (orientation, bit L+1, xor the pattern of the level's first stage) and
  // at its end (the half stage leaves the high halves negated).
  template <int L>
  static __device__ __forceinline__ uint32_t sign_start(int lane, int j, int h) {
    const uint32_t desc = L + 1 < LOGN ? B::ebit(lane, j, h, L + 1) : 0u;
    return desc ^ (patterned(L) ? B::ebit(lane, j, h, L) : 0u);
  }
  template <int L>
  static __device__ __forceinline__ uint32_t sign_end(int lane, int j, int h) {
    const uint32_t desc = L + 1 < LOGN ? B::ebit(lane, j, h, L + 1) : 0u;
    return desc ^ (uint32_t)h;
  }
  // Sign words: at the start of level LOGKV (from unsigned keys), and the
  // flips from the end of level L to the start of level L+1.
  static __device__ __forceinline__ uint32_t entry_signs(int lane, int j) {
    return (sign_start<LOGKV>(lane, j, 0) << 15) | (sign_start<LOGKV>(lane, j, 1) << 31);
  }
  template <int L>
  static __device__ __forceinline__ uint32_t flips(int lane, int j) {
    uint32_t c = 0;
#pragma unroll
    for (int h = 0; h < 2; ++h)
      c |= (sign_end<L>(lane, j, h) ^ sign_start<L + 1>(lane, j, h)) << (15 + 16 * h);
    return c;
  }

  // Level 0: each pair (VGPRs j, j+1, both halves) counted, then exchanged.
  static __device__ __forceinline__ uint32_t level0(uint32_t (&v)[KV]) {
    constexpr uint32_t kOnes = 0x00010001u;
    uint32_t c = 0;
#pragma unroll
    for (int j = 0; j < KV; j += 2) {
      const u16x2 a = vec(v[j]), b = vec(v[j + 1]);
      c = __builtin_amdgcn_udot2(pmin(__builtin_elementwise_sub_sat(a, b), vec(kOnes)), vec(kOnes),
                                 c, false);
      asm volatile("" : "+v"(c));
      v[j] = bits(pmin(a, b));
      v[j + 1] = bits(pmax(a, b));
    }
    return c;
  }

  // Levels 1 .. LOGKV-1, inside a half: ascending blocks of 2^(L+1) VGPRs.
  // In an ascending block of 2s merged from two of s, the pairs counted are
  // s*s + s(s-1)/2 less the sum of the positions of the second block's
  // elements (added in constant_part).
  template <int L>
  static __device__ __forceinline__ void half_levels(uint32_t (&v)[KV], uint32_t& total) {
    if constexpr (L < LOGKV) {
      if constexpr (L > 1 && epoch_start(L)) {
#pragma unroll
        for (int j = 0; j < KV; ++j) v[j] = (v[j] & ~kField) | half_field(L, j);
      }
      constexpr int m = (2 << L) - 1;
#pragma unroll
      for (int j = 0; j < KV; ++j) {
        if ((j >> L) & 1) continue;
        const u16x2 a = vec(v[j]), b = vec(v[j ^ m]);
        v[j] = bits(pmin(a, b));
        v[j ^ m] = bits(pmax(a, b));
      }
#pragma unroll
      for (int k = L - 1; k >= 0; --k) {
#pragma unroll
        for (int j = 0; j < KV; ++j) {
          if ((j >> k) & 1) continue;
          const u16x2 a = vec(v[j]), b = vec(v[j | (1 << k)]);
          v[j] = bits(pmin(a, b));
          v[j | (1 << k)] = bits(pmax(a, b));
        }
      }
      constexpr int tb = L - epoch_of(L);
      uint32_t acc = 0;
#pragma unroll
      for (int j = 0; j < KV; ++j) {
        const uint32_t w = (uint32_t)(j & m);
        if (w == 0u) continue;
        acc = __builtin_amdgcn_udot2(vec(v[j] & (0x00010001u << tb)), vec(w * 0x00010001u), acc,
                                     false);
        asm volatile("" : "+v"(acc));
      }
      total -= acc >> tb;
      half_levels<L + 1>(v, total);
    }
  }

  // Levels L .. kEnd-1 (L >= LOGKV): stages, count, and the step to the next
  // level (sign flips, and a new field where an epoch starts).  Without the
  // top level the first half's keys end with field and sign cleared.
  template <int L, int kEnd>
  static __device__ __forceinline__ void levels(uint32_t (&v)[KV], int lane, int plane,
                                                uint32_t* xbuf, uint32_t& total) {
    stages_down<L, L, patterned(L) ? L : -1>(v, lane, plane, xbuf);
    constexpr int tb = L - epoch_of(L);
    uint32_t acc = 0;
#pragma unroll
    for (int j = 0; j < KV; ++j) {
      // the half stage left the high halves negated: descending over j
      constexpr uint32_t kW = 1u << kWShift;
      const uint32_t w = ((uint32_t)j + kW) | (((uint32_t)(K - 1 - j) + kW) << 16);
      acc = __builtin_amdgcn_udot2(vec(v[j] & (0x00010001u << tb)), vec(w), acc, false);
      asm volatile("" : "+v"(acc));
    }
    acc >>= tb;
    {
      // the lane lies inside one block of 2s, at ascending offset base of
      // its oriented keys; a descending block's key order is the reverse
      constexpr uint32_t m2s = (2u << L) - 1u;
      const uint32_t base = ((uint32_t)lane & ((1u << (L + 1 - LOGK)) - 1u)) << LOGK;
      const uint32_t rsum = acc & ((1u << kWShift) - 1u), nraw = acc >> kWShift;
      const uint32_t desc = (L + 1 < LOGN) ? (uint32_t)(lane >> (L + 1 - LOGK)) & 1u : 0u;
      total -= desc ? (m2s - base) * nraw - rsum : base * nraw + rsum;
    }
    if constexpr (L + 1 < kEnd) {
#pragma unroll
      for (int j = 0; j < KV; ++j) {
        if constexpr (epoch_start(L + 1))
          v[j] = and_xor(v[j], ~kField, field_word(L + 1, lane, j) | flips<L>(lane, j));
        else
          v[j] ^= flips<L>(lane, j);
      }
      levels<L + 1, kEnd>(v, lane, plane, xbuf, total);
    } else if constexpr (L + 1 < LOGN) {
#pragma unroll
      for (int j = 0; j < KV; ++j) v[j] &= ~(kField | kSign);
    }
  }

  // Over levels 1 .. LOGN-1, sum over blocks of s*s + s(s-1)/2 (level 0 is
  // counted directly).
  static constexpr uint32_t constant_part() {
    uint64_t c = 0;
    for (int L = 1; L < LOGN; ++L) {
      const uint64_t s = 1ull << L;
      c += ((uint64_t)N / (2 * s)) * (s * s + s * (s - 1) / 2);
    }
    return (uint32_t)c;
  }
  static constexpr uint32_t top_const() { return B::top_const(); }

  // As Net::count_split, from the same packed keys 2*rank (padding 0xFFFE);
  // without the top level the first half's keys end as 0x0400 + rank * 2^kT.
  template <bool kTop>
  static __device__ __forceinline__ uint32_t count_split(u16x2 (&key)[KV], int plane,
                                                         uint32_t* xbuf) {
    // the lane's per-level sign and tag words are formed where they are used
    // (an empty asm keeps them from being hoisted out of the loop of pairs
    // and held, or spilled, across it)
    asm volatile("" : "+v"(plane));
    const int lane = logical_lane(plane);
    constexpr uint32_t kScale = (1u << (kT - 1)) * 0x00010001u;
    uint32_t v[KV];
#pragma unroll
    for (int j = 0; j < KV; ++j) {
      // 0x0400 + rank * 2^kT + the first epoch's field, padding at rank N
      const u16x2 r = pmin(key[j], vec((uint32_t)(2 * N) * 0x00010001u));
      v[j] = bits(r * vec(kScale) + vec(0x04000400u | half_field(1, j)));
    }
    uint32_t total = level0(v);
    half_levels<1>(v, total);
    {
      // into the half stage's level: its epoch's field and the signs
#pragma unroll
      for (int j = 0; j < KV; ++j)
        v[j] = and_xor(v[j], ~kField, field_word(LOGKV, lane, j) | entry_signs(lane, j));
    }
    levels<LOGKV, kTop ? LOGN : LOGN - 1>(v, lane, plane, xbuf, total);
    if (plane == 0) total += kTop ? constant_part() : constant_part() - top_const();
#pragma unroll
    for (int j = 0; j < KV; ++j) key[j] = vec(v[j]);
    return total;
  }
};

}  // namespace bitonic
}  // namespace ktau
