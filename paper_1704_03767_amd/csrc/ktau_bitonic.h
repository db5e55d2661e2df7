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
      if constexpr (L + 1 < LOGN) v[j] = vec(bits(v[j]) ^ t ^ tag_const<L + 1>(lane, j));
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

}  // namespace bitonic
}  // namespace ktau
