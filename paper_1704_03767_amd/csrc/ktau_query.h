// Internal declarations of the query-vs-database path (ktau_query.hip and
// the serving loop in ktau_server.hip).
#pragma once

#include "ktau_internal.h"

namespace ktau {

// A resident, ranked database.
struct DbView {
  RankView rv;
  int64_t m = 0, n = 0;
  int scheme = 0;
  uint32_t* bits = nullptr;        // bit sets of the rows (KTAU_SCHEME_NAIVE only)
  int32_t* heavy = nullptr;        // heavy-row list of the database
  int32_t* heavy_count = nullptr;
  int32_t heavy_rows = -1;         // its length, read back once (-1: unknown)
};

// One query launch: nq query rows against all m database rows.
struct QueryDesc {
  RankView rq;                     // query rows (same row stride as rdb)
  RankView rdb;
  int64_t nq, m;
  int32_t n, pad;
  double* tau;                     // [nq][m]
  int64_t* nd;                     // [nq][m]
  const int32_t* status;
  const int32_t* q_heavy;
  const int32_t* q_heavy_count;
  const int32_t* db_heavy;
  const int32_t* db_heavy_count;
};

// Step 5 and Eq. 3 for a (query, database row) pair: the same expression,
// in the same order, as the all-pairs store.
__device__ __forceinline__ void store_cross(const QueryDesc& qd, int64_t slot, int64_t n1q,
                                            int64_t n1d, uint32_t nd32, uint32_t n332) {
  const int64_t n = qd.n;
  const int64_t n0 = n * (n - 1) / 2;
  const int64_t nd = nd32, n3 = n332;
  const int64_t nc = n0 - n1q - n1d + n3 - nd;
  const double num = (double)(nc - nd);
  const double d1 = (double)(n0 - n1q);
  const double d2 = (double)(n0 - n1d);
  const double prod = d1 * d2;
  const double den = sqrt(prod);
  qd.tau[slot] = den == 0.0 ? __builtin_nan("") : num / den;
  qd.nd[slot] = nd;
}

hipError_t launch_heavy(const MatDesc& d, hipStream_t s);

// The naive count (bit sets, ktau_bits.hip) of every (query, database row)
// pair into qd.tau / qd.nd: qbits and dbbits hold the sets of the query rows
// and of the database rows.
hipError_t launch_bits_query(const QueryDesc& qd, const uint32_t* qbits, const uint32_t* dbbits,
                             hipStream_t s);

// Device bytes a query launch needs beyond the status header (naive: the
// database uses KTAU_SCHEME_NAIVE, so the query rows need bit sets too).
size_t query_scratch_bytes(int64_t nq, int64_t m, int64_t n, int k, bool naive);

// Enqueues a full query (rank, pairs, composite, top-k, write) on s; scratch
// holds query_scratch_bytes(nq, db.m, db.n, k) bytes (256-byte aligned);
// status is the device word that collects NaN reports.
int launch_query(const DbView& db, const float* Q, int64_t nq, int k, void* scratch,
                 int64_t* idx_out, double* tau_out, int64_t* nd_out, int32_t* status,
                 hipStream_t s);

}  // namespace ktau

struct ktau_db {
  ktau::DbView v;
  void* ws = nullptr;              // library-owned rank workspace of the database
};
