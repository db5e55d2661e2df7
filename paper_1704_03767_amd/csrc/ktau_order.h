// Order in which a plain launch visits the q x q tiles of one matrix (the
// tile triangle of Eq. 11-14).  Integer arithmetic only, usable on the host
// (tests) and the device.  Internal to libktau.
//
// Workgroup b of a launch runs on XCD b mod 8 (the hardware hands
// workgroups to the 8 XCDs round-robin; each XCD has its own L2).  The
// schedule gives every XCD one contiguous stretch of a "band" order: bands
// of kBand tile rows, and inside a band, tile columns left to right, the
// band's tiles of one column top to bottom.  The rows of a band (perm and
// rank of kBand * q variables) stay in the XCD's L2 while the band's columns
// stream through it, so each input row is fetched about once per band
// instead of once per tile.
#pragma once

#include <stdint.h>

#ifdef __HIPCC__
#define KTAU_HD __host__ __device__
#else
#define KTAU_HD
#endif

namespace ktau {

constexpr int64_t kBand = 16;   // tile rows per band
constexpr int64_t kXcds = 8;

// Tiles of the bands before band B (all of them full, kBand rows).
KTAU_HD inline int64_t band_prefix(int64_t w, int64_t B) {
  return B * (kBand * w - kBand * (kBand - 1) / 2) - kBand * kBand * (B * (B - 1) / 2);
}

// Tile coordinates of the i-th tile of the band order (0 <= i < w(w+1)/2).
KTAU_HD inline void band_tile(int64_t w, int64_t i, int64_t& yq, int64_t& xq) {
  int64_t lo = 0, hi = (w - 1) / kBand;   // the last band with prefix <= i
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (band_prefix(w, mid) <= i) lo = mid;
    else hi = mid - 1;
  }
  const int64_t y0 = lo * kBand;
  const int64_t h = (w - y0) < kBand ? (w - y0) : kBand;
  int64_t off = i - band_prefix(w, lo);
  const int64_t diag = h * (h + 1) / 2;   // the band's triangle on the diagonal
  if (off < diag) {
    int64_t c = 0;                        // column y0 + c holds c + 1 tiles
    while ((c + 1) * (c + 2) / 2 <= off) ++c;
    xq = y0 + c;
    yq = y0 + (off - c * (c + 1) / 2);
  } else {
    // off < kBand * w < 2^32 for every w the library accepts
    const uint32_t o = (uint32_t)(off - diag), hh = (uint32_t)h;
    xq = y0 + h + (int64_t)(o / hh);
    yq = y0 + (int64_t)(o % hh);
  }
}

// Tile run by workgroup b of a launch with one workgroup per tile (T tiles,
// w tiles per side).
KTAU_HD inline void scheduled_tile(int64_t w, int64_t T, int64_t b, int64_t& yq, int64_t& xq) {
  const int64_t x = b % kXcds, k = b / kXcds;
  const int64_t r = T % kXcds;
  const int64_t start = x * (T / kXcds) + (x < r ? x : r);
  band_tile(w, start + k, yq, xq);
}

}  // namespace ktau
