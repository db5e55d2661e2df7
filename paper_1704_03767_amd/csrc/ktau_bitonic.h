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
        acc_in = __builtin_amdgcn_udot2(vec(t), vec(in_lane_weight(L, j)), acc_in, false);
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

// The same count with keys held as half-precision bit patterns, for groups of
// at most 8192 keys.  A key 2*rank + tag becomes the positive normal f16
// pattern 0x0400 + 2*rank + tag (padding 0x7BFE), so that the packed f16
// minimum orders keys as integers do, and flipping the sign bit reverses the
// order.  The sign bit then carries two things:
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
// VGPRs under that numbering; later half stages pair VGPR j with VGPR KV-1-j,
// and the count's position weights follow it.

template <int K, int G>
struct NetS {
  using B = Net<K, G>;
  static constexpr int KV = B::KV, LOGK = B::LOGK, LOGKV = B::LOGKV, LOGG = B::LOGG;
  static constexpr int LOGN = B::LOGN, N = B::N, kXChunk = B::kXChunk, kWShift = B::kWShift;
  static_assert(N <= 8192, "keys 0x0400 + 2*rank + tag stay below the padding key 0x7BFE");
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
  // min(a, -b); min(a, -(a with its halves swapped)); min(a, -(b with its
  // halves swapped))
  static __device__ __forceinline__ uint32_t fmn_neg(uint32_t a, uint32_t b) {
    return hu(__builtin_elementwise_minimum(hv(a), -hv(b)));
  }
  static __device__ __forceinline__ uint32_t fmn_neg_swap(uint32_t a) {
    const h2 x = hv(a);
    return hu(__builtin_elementwise_minimum(x, -__builtin_shufflevector(x, x, 1, 0)));
  }
  static __device__ __forceinline__ uint32_t fmn_neg_swapped(uint32_t a, uint32_t b) {
    const h2 y = hv(b);
    return hu(__builtin_elementwise_minimum(hv(a), -__builtin_shufflevector(y, y, 1, 0)));
  }

  // Stage on element bit k: takes a sign pattern (the upper partner negated)
  // or needs both partners positive (permlane stages); register stages take
  // whatever signs their partners share.
  static constexpr bool patterned(int k) {
    return k == LOGKV || (k >= LOGK && (B::phys_bit(k - LOGK) < 4 || B::phys_bit(k - LOGK) > 5));
  }
  static constexpr bool wants_plain(int k) { return k >= LOGK && !patterned(k); }

  // Sign bits of the pattern keyed on element bit b (b < 0: none), for the
  // element lane `lane`; b is the half bit or a lane bit.
  static __device__ __forceinline__ uint32_t pattern(int lane, int b) {
    if (b < 0) return 0u;
    if (b == LOGKV) return 0x80000000u;
    return ((lane >> (b - LOGK)) & 1) ? kSign : 0u;
  }

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
    } else if constexpr (k == LOGKV && (L == LOGKV || KV == 1)) {
#pragma unroll
      for (int j = 0; j < KV; ++j) v[j] = fmn_neg_swap(v[j]);
    } else if constexpr (k == LOGKV) {
      // the high halves hold their elements in reverse order: VGPR j's low
      // half meets VGPR KV-1-j's high half and the reverse
#pragma unroll
      for (int j = 0; j < KV / 2; ++j) {
        const uint32_t a = v[j], b = v[KV - 1 - j];
        v[j] = fmn_neg_swapped(a, b);
        v[KV - 1 - j] = fmn_neg_swapped(b, a);
      }
    } else {
      constexpr int lb = k - LOGK;
      constexpr int pb = B::phys_bit(lb);
      if constexpr (pb < 4) {
#pragma unroll
        for (int j = 0; j < KV; ++j) v[j] = fmn_neg(v[j], lane_xor<(1 << pb)>(v[j]));
      } else if constexpr (pb == 4 || pb == 5) {
        if constexpr (KV >= 2) {
#pragma unroll
          for (int j = 0; j < KV; j += 2) {
            uint32_t a = v[j], b = v[j + 1];
            if constexpr (pb == 4) {
              auto s = __builtin_amdgcn_permlane16_swap(a, b, false, false);
              a = s[0];
              b = s[1];
            } else {
              auto s = __builtin_amdgcn_permlane32_swap(a, b, false, false);
              a = s[0];
              b = s[1];
            }
            const uint32_t mn = fmn(a, b), mx = fmx(a, b);
            if constexpr (pb == 4) {
              auto s = __builtin_amdgcn_permlane16_swap(mn, mx, false, false);
              v[j] = s[0];
              v[j + 1] = s[1];
            } else {
              auto s = __builtin_amdgcn_permlane32_swap(mn, mx, false, false);
              v[j] = s[0];
              v[j + 1] = s[1];
            }
          }
        } else {
          const bool lower = ((lane >> lb) & 1) == 0;
          const uint32_t a = v[0];
          uint32_t part;
          if constexpr (pb == 4) {
            auto s = __builtin_amdgcn_permlane16_swap(a, a, false, false);
            part = lower ? (uint32_t)s[1] : (uint32_t)s[0];
          } else {
            auto s = __builtin_amdgcn_permlane32_swap(a, a, false, false);
            part = lower ? (uint32_t)s[1] : (uint32_t)s[0];
          }
          v[0] = lower ? fmn(a, part) : fmx(a, part);
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

  // Stages k .. 0 of a level; `cur` is the element bit the current sign
  // pattern is keyed on (-1: none).
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

  // Sign bit of element (lane, j, h) at the start of level L (orientation,
  // bit L+1, xor the pattern of the level's first stage) and at its end (the
  // half stage of levels L >= LOGKV leaves the high halves negated).
  template <int L>
  static __device__ __forceinline__ uint32_t sign_start(int lane, int j, int h) {
    const uint32_t desc = L + 1 < LOGN ? B::ebit(lane, j, h, L + 1) : 0u;
    return desc ^ (patterned(L) ? B::ebit(lane, j, h, L) : 0u);
  }
  template <int L>
  static __device__ __forceinline__ uint32_t sign_end(int lane, int j, int h) {
    const uint32_t desc = L + 1 < LOGN ? B::ebit(lane, j, h, L + 1) : 0u;
    return desc ^ (L >= LOGKV ? (uint32_t)h : 0u);
  }
  // Tag (bit 0) and sign (bit 15) of each half of VGPR j at the start of
  // level 0, the keys carrying neither.
  static __device__ __forceinline__ uint32_t start_const(int lane, int j) {
    uint32_t c = 0;
#pragma unroll
    for (int h = 0; h < 2; ++h)
      c |= (B::ebit(lane, j, h, 0) | (sign_start<0>(lane, j, h) << 15)) << (16 * h);
    return c;
  }
  // From the end of level L to the start of L+1: with t the current tag
  // bits, v ^ t ^ retag_const sets tag bit L+1 and flips the sign where it
  // changes.
  template <int L>
  static __device__ __forceinline__ uint32_t retag_const(int lane, int j) {
    uint32_t c = 0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint32_t flip = sign_end<L>(lane, j, h) ^ sign_start<L + 1>(lane, j, h);
      c |= (B::ebit(lane, j, h, L + 1) | (flip << 15)) << (16 * h);
    }
    return c;
  }

  // Key position weights of the count (see Net): inside a lane, VGPR j's
  // halves at ascending positions of their merged block.
  static constexpr uint32_t in_lane_weight(int L, int j) {
    uint32_t w = 0;
    for (int h = 0; h < 2; ++h) {
      const uint32_t e = ((uint32_t)h << LOGKV) | (uint32_t)j;
      const uint32_t m2s = (2u << L) - 1u;
      const uint32_t pos = e & m2s;
      const uint32_t desc = (e >> (L + 1)) & 1u;
      w |= (desc ? m2s - pos : pos) << (16 * h);
    }
    return w;
  }

  template <int L, int kEnd>
  static __device__ __forceinline__ void levels(uint32_t (&v)[KV], int lane, int plane,
                                                uint32_t* xbuf, uint32_t& acc_in,
                                                uint32_t& total) {
    stages_down<L, L, patterned(L) ? L : -1>(v, lane, plane, xbuf);
    uint32_t acc = 0;
#pragma unroll
    for (int j = 0; j < KV; ++j) {
      const uint32_t t = v[j] & 0x00010001u;
      if constexpr (L + 1 < LOGK) {
        acc_in = __builtin_amdgcn_udot2(vec(t), vec(in_lane_weight(L, j)), acc_in, false);
        asm volatile("" : "+v"(acc_in));
      } else {
        // the half stage left the high halves negated: descending over j
        constexpr uint32_t kW = 1u << kWShift;
        const uint32_t w = ((uint32_t)j + kW) | (((uint32_t)(K - 1 - j) + kW) << 16);
        acc = __builtin_amdgcn_udot2(vec(t), vec(w), acc, false);
        asm volatile("" : "+v"(acc));
      }
      // the re-tag word depends on the lane once bit L+2 is a lane bit
      if constexpr (L + 1 < LOGN) v[j] = xor3<(L + 2 < LOGK)>(v[j], t, retag_const<L>(lane, j));
    }
    if constexpr (L + 1 >= LOGK) {
      // the lane lies inside one block of 2s, at ascending offset base of
      // its oriented keys; a descending block's key order is the reverse
      constexpr uint32_t m2s = (2u << L) - 1u;
      const uint32_t base = ((uint32_t)lane & ((1u << (L + 1 - LOGK)) - 1u)) << LOGK;
      const uint32_t rsum = acc & ((1u << kWShift) - 1u), nraw = acc >> kWShift;
      const uint32_t desc = (L + 1 < LOGN) ? (uint32_t)(lane >> (L + 1 - LOGK)) & 1u : 0u;
      total -= desc ? (m2s - base) * nraw - rsum : base * nraw + rsum;
    }
    if constexpr (L + 1 < kEnd) levels<L + 1, kEnd>(v, lane, plane, xbuf, acc_in, total);
  }

  // Over all levels, sum over blocks of s*s + s(s-1)/2.
  static constexpr uint32_t constant_part() {
    uint64_t c = 0;
    for (int L = 0; L < LOGN; ++L) {
      const uint64_t s = 1ull << L;
      c += ((uint64_t)N / (2 * s)) * (s * s + s * (s - 1) / 2);
    }
    return (uint32_t)c;
  }
  static constexpr uint32_t top_const() { return B::top_const(); }

  // Bias of the first half's keys after the network without its top level:
  // they are 0x0400 + 2*rank.
  static constexpr uint32_t kKeyBias = kHalfKeyBias;

  // As Net::count_split, from the same packed keys 2*rank (padding 0xFFFE).
  template <bool kTop>
  static __device__ __forceinline__ uint32_t count_split(u16x2 (&key)[KV], int plane,
                                                         uint32_t* xbuf) {
    // the lane's per-level sign and tag words are formed where they are used
    // (an empty asm keeps them from being hoisted out of the loop of pairs
    // and held, or spilled, across it)
    asm volatile("" : "+v"(plane));
    const int lane = B::logical_lane(plane);
    uint32_t v[KV];
#pragma unroll
    for (int j = 0; j < KV; ++j) {
      // the bias and the level-0 tag and sign bits (all clear in the clamped
      // key) in one packed add
      v[j] = bits(pmin(key[j], vec(0x77FE77FEu)) + vec(0x04000400u | start_const(lane, j)));
    }
    uint32_t acc_in = 0, total = 0;
    levels<0, kTop ? LOGN : LOGN - 1>(v, lane, plane, xbuf, acc_in, total);
    total -= acc_in;
    if (plane == 0) total += kTop ? constant_part() : constant_part() - top_const();
#pragma unroll
    for (int j = 0; j < KV; ++j) key[j] = vec(v[j]);
    return total;
  }
};

}  // namespace bitonic
}  // namespace ktau
