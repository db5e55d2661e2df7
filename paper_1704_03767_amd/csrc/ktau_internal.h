// Internal declarations shared by the HIP translation units of libktau.
// Nothing here is part of the public interface (include/ktau.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ktau.h"

namespace ktau {

// Rows of every per-variable array are padded to a multiple of 128 uint16
// elements (a 256-byte boundary), so that a pair kernel lane's block of
// K <= 128 sorted positions is either wholly inside the padded row or wholly
// past it.
constexpr int64_t kRowAlign = 128;
constexpr size_t kWsHeader = 256;       // bytes: status word + reserved
constexpr size_t kAlign = 256;

// Longest row whose 64-bit sort keys one workgroup sorts in LDS (128 KB);
// longer rows (up to KTAU_MAX_N) finish their sort in global scratch, one
// slot of sort_slot_words(n) words (n rounded up to a power of two) per
// workgroup of at most kSortSlots.
constexpr int kLdsSortMax = 16384;
constexpr int64_t kSortSlots = 256;

// Rows of up to kDoubledMaxN samples keep doubled 16-bit ranks and sample
// byte offsets in a pair workspace (2 rank + tag fits 16 bits); longer rows
// keep them plain (16-bit ranks and sample indices up to 65535).
constexpr int64_t kDoubledMaxN = 32768;
__host__ __device__ inline bool ws_doubled(int64_t n) { return n <= kDoubledMaxN; }

__host__ __device__ inline int64_t row_ld(int64_t n) {
  return (n + kRowAlign - 1) / kRowAlign * kRowAlign;
}

__host__ __device__ inline int64_t sort_slot_words(int64_t n) {
  int64_t w = 2 * kLdsSortMax;
  while (w < n) w <<= 1;
  return w;
}

// Bytes of sort scratch the pre-pass of m rows of length n needs.
inline size_t sort_scratch_bytes(int64_t m, int64_t n) {
  if (n <= kLdsSortMax) return 0;
  return (size_t)(m < kSortSlots ? m : kSortSlots) * (size_t)sort_slot_words(n) * sizeof(uint64_t);
}

// Tie runs longer than kLongRunMin and at most kLongRunMax samples are
// "long": the merge schemes count the inversions and joint ties inside them
// with a sorting network per run instead of comparing every pair in them.
constexpr int kLongRunMin = 64;
constexpr int kLongRunMax = 512;

// Sort keys: padding slots beyond n, and the sentinel read past a run end.
// Real keys are at most 0x7FFFFFFE (15-bit tie-run start << 16 | doubled
// rank, with n <= 16384 on that pass), so both compare above every real key
// and the sentinel above the padding.
constexpr uint32_t kPadKey = 0xFFFFFFFEu;
constexpr uint32_t kSentinel = 0xFFFFFFFFu;

__host__ __device__ inline int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

// ---- job-id bijection (Sec. 4.1, Eq. 4-10) and tiles (Sec. 4.2, Eq. 11-14)

// Cells before row y of the inclusive upper triangle of a d x d matrix (Eq. 5).
__host__ __device__ inline int64_t tri_row_start(int64_t d, int64_t y) {
  return y * (2 * d - y + 1) / 2;
}

// Row of inclusive-triangle id t in a d x d matrix: Eq. 9 in FP64, then an
// exact integer correction so rounding in sqrt can never pick the wrong row.
__host__ __device__ inline int64_t tri_row_of(int64_t d, int64_t t) {
  double dd = (double)d;
  double z = dd - 0.5 - sqrt(dd * dd + dd + 0.25 - 2.0 * (double)(t + 1));
  int64_t y = (int64_t)ceil(z);
  if (y < 0) y = 0;
  if (y > d - 1) y = d - 1;
  while (y > 0 && tri_row_start(d, y) > t) --y;
  while (y + 1 < d && tri_row_start(d, y + 1) <= t) ++y;
  return y;
}

// Strict triangle of an m x m matrix = inclusive triangle of dimension m-1
// with x shifted by one: J = F_{m-1}(y) + (x - 1 - y).
__host__ __device__ inline int64_t strict_job(int64_t m, int64_t y, int64_t x) {
  return tri_row_start(m - 1, y) + (x - 1 - y);
}

__host__ __device__ inline void strict_pair(int64_t m, int64_t J, int64_t& y, int64_t& x) {
  y = tri_row_of(m - 1, J);
  x = J - tri_row_start(m - 1, y) + y + 1;
}

__host__ __device__ inline void tile_coord(int64_t w, int64_t t, int64_t& yq, int64_t& xq) {
  yq = tri_row_of(w, t);
  xq = t - tri_row_start(w, yq) + yq;
}

// ---- device views

struct RankView {
  // [rows][ld] sorted position -> 2 x sample (byte offset in a rank row), or
  // the sample itself in rows longer than kDoubledMaxN
  const uint16_t* perm;
  // [rows][ld] sample -> 2 x dense rank, or the rank itself in rows longer
  // than kDoubledMaxN
  const uint16_t* rank;
  const uint16_t* rstart;   // [rows][ld] sorted position -> first position of its tie run
  const int64_t* n1;        // [rows]
  const int32_t* nruns;     // [rows] number of tie runs of length >= 2
  const int32_t* nlong;     // [rows] how many of them are long (listed last)
  // [rows][ld/2] tie runs of length >= 2 in sorted order, the long ones
  // (kLongRunMin < length <= kLongRunMax) after the others: bits 0-15
  // start, 16-31 length - 1, 32-63 number of within-run pairs of the runs
  // listed before it
  const uint64_t* runs;
  int64_t ld;               // row stride in elements (runs: ld/2 per row)
};

struct PairOut {
  int64_t* nc;
  int64_t* nd;
  int64_t* n3;
  double* tau_b;
  double* tau_a;
};

// Per-pair schemes.  A "group" of G lanes (8, 16 or 32 lanes of a wave, a
// whole wave, or a 256-lane block) sorts one pair's n <= G*K keys, K keys per
// lane.  Smaller groups keep more of the network inside each lane's
// registers; the list below is (enum, K, G) of every scheme.
#define KTAU_FOR_EACH_SCHEME(X) \
  X(kWaveK2, 2, 64)             \
  X(kWaveK4, 4, 64)             \
  X(kWaveK8, 8, 64)             \
  X(kWaveK16, 16, 64)           \
  X(kBlockK4, 4, 256)           \
  X(kBlockK8, 8, 256)           \
  X(kBlockK16, 16, 256)         \
  X(kSub8K16, 16, 8)            \
  X(kSub16K16, 16, 16)          \
  X(kSub16K32, 32, 16)          \
  X(kSub16K64, 64, 16)          \
  X(kSub32K32, 32, 32)          \
  X(kSub32K64, 64, 32)          \
  X(kWaveK32, 32, 64)           \
  X(kWaveK64, 64, 64)           \
  X(kSub8K32, 32, 8)            \
  X(kSub8K64, 64, 8)            \
  X(kBlockK32, 32, 256)         \
  X(kBlockK64, 64, 256)         \
  X(kBlockK128, 128, 256)

// After the network schemes come the merge schemes for long rows
// (ktau_merge.hip): one workgroup of up to 16 waves per pair, each wave
// sorting and counting a chunk of 64 K keys with the network above (K = 32 or
// 64), the levels above the chunks counted by a merge path over the keys in
// LDS.  Capacity 16 chunks (32768 or 65536 samples).
enum Scheme : int32_t {
#define KTAU_ENUM(S, K, G) S,
  KTAU_FOR_EACH_SCHEME(KTAU_ENUM)
#undef KTAU_ENUM
  kNumNetSchemes,
  kMergeK32 = kNumNetSchemes,
  kMergeK64,
  kNumSchemes
};
constexpr int kMergeMaxWaves = 16;

__host__ __device__ inline bool is_merge(int s) { return s == kMergeK32 || s == kMergeK64; }
inline int scheme_lanes(int s) {
  static const int g[] = {
#define KTAU_G(S, K, G) G,
      KTAU_FOR_EACH_SCHEME(KTAU_G)
#undef KTAU_G
      64 * kMergeMaxWaves, 64 * kMergeMaxWaves,
  };
  return g[s];
}
inline int scheme_k(int s) {
  static const int k[] = {
#define KTAU_K(S, K, G) K,
      KTAU_FOR_EACH_SCHEME(KTAU_K)
#undef KTAU_K
      32, 64,
  };
  return k[s];
}
inline int64_t scheme_capacity(int s) { return (int64_t)scheme_lanes(s) * scheme_k(s); }
// Name of a numbered scheme or of KTAU_SCHEME_NAIVE ("naive_bits").
const char* scheme_name(int s);
int default_scheme(int64_t n);
// The fastest network scheme that holds n (n <= 32768): the scheme of the
// query and permutation-test kernels, which have no merge form.
int network_scheme(int64_t n);
// Default tile edge: 8 up to n = 4096; longer rows take one 256-lane block per
// pair and are few (m is small next to n), so smaller tiles spread them.
int default_q(int64_t n);
// Tile edge of a plain launch of m rows (default_q, or 16 for large m).
int plain_q(int64_t m, int64_t n);

// Comparisons the direct in-run tie count may spend on one pair (about the
// cost of a second sort); rows whose n1 exceeds it are "heavy", and pairs of
// two heavy rows go to the composite pass.  The composite pass keeps 32-bit
// keys of a whole pair in LDS, which holds up to kCompositeMaxN of them;
// beyond that every pair counts its ties directly (exact, slower only when
// both rows are heavily tied).
constexpr int64_t kCompositeMaxN = 16384;
__host__ __device__ inline int64_t direct_budget(int64_t n) {
  if (n > kCompositeMaxN) return INT64_MAX;
  int64_t lg = 0;
  while ((1ll << lg) < n) ++lg;
  return 4 * n * lg;
}

// Rows of at most kBitsMaxN samples can also be counted by the naive
// comparison of every sample pair, with each row's comparisons stored once as
// bit sets (ktau_bits.hip): bits_words_per_set(n) words per set, two sets per
// sample, bits_bytes(m, n) bytes behind the plain workspace.
constexpr int64_t kBitsMaxN = 256;
constexpr int kBitsQ = 16;              // default tile edge of that path
size_t bits_words_per_set(int64_t n);
size_t bits_bytes(int64_t m, int64_t n);

// One matrix as seen by the pair kernels.
struct MatDesc {
  RankView rv;
  PairOut out;
  const float* X;         // input rows (batched pre-pass)
  int64_t* n1_out;        // optional copy of n1 for the caller
  const int32_t* status;  // device status word (non-zero: skip all work)
  int32_t* heavy;         // [m] list of heavy rows (written by the heavy pass)
  int32_t* heavy_count;   // device scalar
  uint64_t* sort_tmp;     // pre-pass sort scratch (rows longer than kLdsSortMax)
  uint32_t* bits;         // bit sets of KTAU_SCHEME_NAIVE (batches; NULL otherwise)
  int64_t m;
  int32_t n;
  int32_t scheme;
  int32_t q;              // tile edge
  int32_t pad;
  int64_t w;              // tiles per side
  int64_t n_units;        // w (w + 1) / 2 tiles
  int64_t unit_begin;     // first global unit id of this matrix (batched)
  int64_t J_begin, J_end; // jobs of this call; results at J - J_begin
};

// ---- launchers (stream-ordered; return hipError_t)

// sort_tmp: sort_scratch_bytes(m, n) bytes (unused, may be NULL, when n <=
// kLdsSortMax).
hipError_t launch_prepass(const float* X, int64_t m, int64_t n, uint16_t* perm, uint16_t* rank,
                          uint16_t* rstart, int64_t ld, int64_t* n1_ws, int64_t* n1_out,
                          int32_t* nruns, int32_t* nlong, uint64_t* runs, int32_t* status,
                          bool doubled, uint64_t* sort_tmp, hipStream_t s);

// Rank pre-pass of every row of every matrix of a descriptor table whose n is
// at most kLdsSortMax (max_n: the largest such n); longer matrices go
// through launch_prepass one by one.
hipError_t launch_prepass_batch(const MatDesc* descs_dev, int64_t count, int64_t total_rows,
                                const int64_t* row_prefix_dev, int max_n, hipStream_t s);

// Main pair kernel over all tiles (tiles = true) or over jobs
// [J_begin, J_end), then the heavy-row pass and the composite pass.
hipError_t launch_pairs_plain(const MatDesc& d, bool tiles, hipStream_t s);
// The tile kernel alone (one workgroup per tile, band schedule) of a network
// scheme: its pairs past the tie budget are left to the composite pass.
hipError_t launch_pair_tiles(const MatDesc& d, hipStream_t s);

// Merge-scheme pair kernel over jobs [J_begin, J_end) of one matrix (pairs of
// two heavy rows are left to the composite pass, as in the network schemes).
hipError_t launch_pairs_merge(const MatDesc& d, hipStream_t s);
// Sets a merge scheme kernel's LDS limit (done by its first launch too; call
// it before capturing a launch into a graph).
hipError_t prepare_pairs_merge(int scheme);

// Persistent launch of one scheme over the tiles of the matrices of a
// descriptor table (all of that scheme), taking tiles from the kXcds (8)
// zeroed int64 counters at counters_dev.
hipError_t launch_pairs_persistent(int scheme, const MatDesc* descs_dev, int64_t count,
                                   int64_t total_units, const int64_t* unit_prefix_dev,
                                   int64_t* counters_dev, const int32_t* status, hipStream_t s);

// Bit sets of every row of a prepared matrix (n <= kBitsMaxN), and the naive
// pair count from them over all tiles or over jobs [J_begin, J_end).
hipError_t launch_bits_prepass(const MatDesc& d, uint32_t* bits, hipStream_t s);
hipError_t launch_bits_pairs(const MatDesc& d, const uint32_t* bits, bool tiles, hipStream_t s);

// Heavy-row lists and the composite pass for every matrix of a table.
hipError_t launch_tie_passes_batch(const MatDesc* descs_dev, int64_t count, int max_n,
                                   hipStream_t s);

// ---- host helpers shared by the API units (ktau_api.hip)

struct WsLayout {
  size_t perm, rank, rstart, n1, nruns, nlong, runs, heavy, sort, total;
  int64_t ld;
};
WsLayout ws_layout(int64_t m, int64_t n);
int check_shape(int64_t m, int64_t n);
// Descriptor of a matrix whose rank pre-pass lives in `ws`; status NULL means
// the status word at the start of ws.
MatDesc matdesc(void* ws, int64_t m, int64_t n, const ktau_pair_out& out, int scheme, int q,
                int64_t J_begin, int64_t J_end, int32_t* status);
int prepass_ws(const float* X, int64_t m, int64_t n, void* ws, int64_t* n1_out, int32_t* status,
               hipStream_t s);
// Zeroes `count` int32 words with a kernel (never a memset node in a graph).
int clear_words(int32_t* p, int count, hipStream_t s);

}  // namespace ktau
