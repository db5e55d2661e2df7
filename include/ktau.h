/*
 * ktau.h -- exact all-pairs Kendall's tau on AMD Instinct MI355X (gfx950).
 *
 * Paper: Liu, Pan, Green, Aluru, "Parallelized Kendall's Tau Coefficient
 * Computation via SIMD Vectorized Sorting on Many-Integrated-Core Processors".
 *
 * Given m variables observed on n samples (a row-major m x n float32 matrix,
 * one row per variable), the library computes for every strict pair of rows
 * y < x the exact integer counts of Sec. 1 and Table 1 -- concordant n_c,
 * discordant n_d, joint ties n3 -- and the per-row tie term n1 (n2 of a pair is
 * n1 of its second row), and from them tau_B (Eq. 3) and optionally tau_A
 * (Eq. 1) in FP64:
 *     tau_B = (double)(nc - nd) / sqrt((double)(n0 - n1) * (double)(n0 - n2))
 * with n0 = n(n-1)/2, round-to-nearest, no contraction; a constant row gives
 * tau_B = NaN (0/0) while its counts stay exact.  Ties are IEEE float32
 * equality (-0.0 ties +0.0).  NaN inputs are refused (KTAU_ENAN).
 *
 * Counts come from the sorting method of Sec. 3.2: samples ordered by u (a
 * per-row rank pre-pass done once per row, Sec. 3), v permuted into that order,
 * discordant pairs counted as strict inversions (Step 3; Algorithm 2 counts
 * them by merge sort, the kernels here by a bitonic network that yields the
 * same count, and for rows of more than 4096 samples by networks on chunks
 * with merge levels above them), tie runs scanned.  The plain calls count rows of up to 128
 * samples by default with the naive comparison of every sample pair instead
 * (Sec. 3.1), done as per-row bit sets (KTAU_SCHEME_NAIVE below), which gives
 * the same counts.  Pairs are numbered by the job-id bijection of Sec. 4.1
 * (Eq. 4-10) restricted to the strict upper triangle: row-major, y < x,
 *     J(y, x) = F(y) + (x - y - 1),  F(y) = y (2(m-1) - y + 1) / 2,
 * J in [0, m(m-1)/2).  Work is spread in q x q tiles numbered by Eq. 11-14.
 *
 * Conventions for every call:
 *   - Pointers named *_dev are device (HBM) pointers owned by the caller unless
 *     stated; host pointers are named *_host.  The library never frees caller
 *     memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Calls that take a stream are asynchronous and stream-ordered: they
 *     return after validating arguments and enqueueing kernels.
 *   - Every call returns an int status: KTAU_OK (0) or a negative KTAU_E*.
 *     Host-detectable errors are returned before anything is enqueued; NaN in
 *     the input is found on the device, latched in the workspace header and
 *     reported by ktau_status().  No C++ exception crosses this interface.
 *   - Sizes: 2 <= n <= KTAU_MAX_N (KTAU_MAX_N_NETWORK for the query and
 *     permutation-test calls), m >= 2 (m < 2^31).
 */
#ifndef KTAU_H
#define KTAU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KTAU_OK 0
#define KTAU_EINVAL -1    /* bad argument: null pointer, m < 2, n < 2, bad range */
#define KTAU_ERANGE -2    /* n > KTAU_MAX_N, or a job range outside [0, P]      */
#define KTAU_ENOMEM -3    /* workspace too small or a device allocation failed  */
#define KTAU_EDEVICE -4   /* a HIP runtime call failed                          */
#define KTAU_EBUSY -5     /* server: non-blocking submit refused by admission   */
#define KTAU_ENAN -6      /* a NaN was found in the input (latched on device)   */
#define KTAU_ECANCELED -7 /* server: request cancelled or failed in its slot    */
#define KTAU_ETIMEDOUT -8 /* server: wait timed out                             */

/* Largest sample count n of the all-pairs, rank and batch calls.  Ranks and
 * sample indices are 16-bit.  Up to KTAU_MAX_N_NETWORK samples the pair
 * kernels key every sample by twice its rank in 16 bits (the spare bit carries
 * the sort network's tag); longer rows, whose ranks need all 16 bits, are
 * counted twice on two clamped 15-bit halves of the rank range with an exact
 * correction for the pairs that straddle them (the paper packs ranks into
 * 16-bit halves for n <= 32767 and names wider keys as the remedy for longer
 * vectors, Sec. 3.3). */
#define KTAU_MAX_N 65536
/* Largest n of the calls that only have the 16-bit network kernels: the
 * query search and the permutation test (KTAU_ERANGE above it). */
#define KTAU_MAX_N_NETWORK 32768

/* Human-readable name of a status code (static storage). */
const char* ktau_status_string(int status);

/* ---------------------------------------------------------------------------
 * Job-id bijection (Sec. 4.1, Eq. 4-10; tiles Sec. 4.2, Eq. 11-14).  Host
 * functions; the kernels use the same arithmetic on the device.
 * ------------------------------------------------------------------------- */

/* Strict job id of pair (y, x), 0 <= y < x < m; -1 if the pair is invalid. */
int64_t ktau_pair_to_job(int64_t m, int64_t y, int64_t x);

/* Inverse of ktau_pair_to_job: Eq. 9 on dimension m-1 evaluated in FP64,
 * then an exact integer fix-up.  KTAU_ERANGE if J is not in [0, m(m-1)/2). */
int ktau_job_to_pair(int64_t m, int64_t J, int64_t* y_host, int64_t* x_host);

/* Inclusive tile triangle of a w x w tile matrix (Eq. 11-14): tile id t in
 * [0, w(w+1)/2) -> tile coordinate yq <= xq.  KTAU_ERANGE if t is outside. */
int ktau_tile_to_coord(int64_t w, int64_t t, int64_t* yq_host, int64_t* xq_host);

/* ---------------------------------------------------------------------------
 * Rank pre-pass (Sec. 3: every vector is replaced by its ranks once).
 * ------------------------------------------------------------------------- */

/* For each row r of X_dev (m x n float32, row-major, contiguous):
 *   perm_dev[r*n + k]   = sample at sorted position k (ascending value, equal
 *                         values by sample index), uint16;
 *   rank_dev[r*n + i]   = dense rank of sample i (number of distinct values
 *                         below it), uint16;
 *   rstart_dev[r*n + k] = first sorted position of the tie run holding
 *                         position k, uint16;
 *   n1_dev[r]           = sum over tie runs of t(t-1)/2, int64.
 * Any output may be NULL.  status_dev (int32, device) receives KTAU_ENAN if a
 * NaN is present (written only on error; the caller clears it).
 * ws_dev: device scratch of at least ktau_rank_workspace_size(m, n) bytes,
 * 256-byte aligned, owned by the caller and free again when the stream has
 * passed the call; rows longer than 16384 finish their sort there.  It may be
 * NULL when that size is 0 (n <= 16384).  Errors: KTAU_EINVAL (null X or
 * status, m or n < 1, missing or misaligned scratch), KTAU_ERANGE
 * (n > KTAU_MAX_N), KTAU_ENOMEM (ws_bytes too small). */
size_t ktau_rank_workspace_size(int64_t m, int64_t n);
int ktau_rank(const float* X_dev, int64_t m, int64_t n, uint16_t* perm_dev,
              uint16_t* rank_dev, uint16_t* rstart_dev, int64_t* n1_dev,
              int32_t* status_dev, void* ws_dev, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Plain all-pairs.
 * ------------------------------------------------------------------------- */

/* Result arrays, all device pointers; any may be NULL to skip it.  Pair
 * arrays hold one entry per strict job id (J - J_begin for range calls). */
typedef struct ktau_pair_out {
  int64_t* nc;     /* concordant pairs                       [P]  */
  int64_t* nd;     /* discordant pairs                       [P]  */
  int64_t* n3;     /* pairs tied in both rows                [P]  */
  double* tau_b;   /* tau_B (Eq. 3)                          [P]  */
  double* tau_a;   /* tau_A (Eq. 1)                          [P]  */
  int64_t* n1;     /* per-row tie term; n2 of (y, x) = n1[x] [m]  */
} ktau_pair_out;

/* Bytes of device workspace the all-pairs calls need for (m, n): the rank
 * pre-pass of every row (Sec. 3: each vector ranked once beforehand), about
 * 10 m ceil128(n) bytes; for n <= 256 also the bit sets of
 * KTAU_SCHEME_NAIVE, 8 n ceil(n/32) bytes per row rounded up to 1, 2, 4 or 8
 * words per set; for n > 16384 a sort scratch of up to 256 rows.  0 for an
 * invalid shape. */
size_t ktau_allpairs_workspace_size(int64_t m, int64_t n);

/* All m(m-1)/2 strict pairs of X_dev (m x n float32, row-major): the
 * all-pairs correlation matrix of Sec. 1 (Eq. 1-3 for every pair of rows),
 * counted by the sorting method of Sec. 3.2 and numbered by the strict job
 * bijection (Sec. 4.1).  out's arrays (device, caller-owned, NULL to skip)
 * receive one entry per job id.  The workspace (>= ktau_allpairs_workspace_size
 * bytes, 256-byte aligned, owned by the caller) receives the rank pre-pass and
 * the status word; it may be reused once the previous call on it has
 * completed.  Errors: KTAU_EINVAL (null X, bad shape, misaligned workspace),
 * KTAU_ERANGE (n > KTAU_MAX_N), KTAU_ENOMEM (workspace too small),
 * KTAU_EDEVICE (a launch failed); a NaN is latched for ktau_status. */
int ktau_allpairs(const float* X_dev, int64_t m, int64_t n, ktau_pair_out out,
                  void* workspace_dev, size_t ws_bytes, void* stream);

/* Jobs J in [J_begin, J_end) only: the correlation matrix computed in
 * job-id sub-ranges over several passes (Sec. 4.3, offload in passes); the
 * result slot of job J is J - J_begin.  Any prefix of the job range can be
 * resumed from its end.  Errors as ktau_allpairs, plus KTAU_ERANGE if
 * 0 <= J_begin <= J_end <= m(m-1)/2 does not hold. */
int ktau_allpairs_range(const float* X_dev, int64_t m, int64_t n,
                        int64_t J_begin, int64_t J_end, ktau_pair_out out,
                        void* workspace_dev, size_t ws_bytes, void* stream);

/* ktau_allpairs for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same computation and results, with the workspace in a fixed static
 * device array of 64 MiB inside the library (one per GPU, held until the
 * process ends) instead of caller memory; the call makes no allocation.
 * Shapes whose ktau_allpairs_workspace_size exceeds 64 MiB are refused with
 * KTAU_ENOMEM before anything is enqueued (for example m = 4096, n = 1024
 * fits; m = 16384, n = 1024 does not).  status_dev (device int32, may be
 * NULL) receives the call's latched status (KTAU_ENAN for a NaN input, else
 * KTAU_OK) in stream order.  Every call on one GPU shares that GPU's array:
 * calls that overlap on one GPU (several streams or threads) race and must be
 * serialised by the caller.  Other errors as ktau_allpairs. */
int ktau_allpairs_noalloc(const float* X_dev, int64_t m, int64_t n, ktau_pair_out out,
                          int32_t* status_dev, void* stream);

/* The two halves of ktau_allpairs, for callers that rank once and then make
 * several passes over job sub-ranges (Sec. 4.3) or time the halves apart.
 * ktau_prepare clears the workspace status and runs the rank pre-pass of X
 * into the workspace (Sec. 3: ranks, order, tie runs and n1 of every row,
 * once; writing out_n1_dev[m] too if it is not NULL), and for n <= 256 the
 * bit sets of KTAU_SCHEME_NAIVE.
 * ktau_pairs computes jobs [J_begin, J_end) (J_begin < 0: all jobs, in tile
 * order) from a workspace prepared for the same (m, n): Sec. 3.2 Steps 1-5
 * per pair with the per-row halves taken from the workspace; scheme < 0 and
 * q <= 0 pick the defaults (ktau_plain_default_scheme(n); tile edge 16 for
 * KTAU_SCHEME_NAIVE, else for n <= 4096 16 from m = 8192 rows on and 8 below,
 * 4 for n <= 16384, 2 beyond; the merge schemes take pairs in job order and
 * ignore q).  Errors as
 * ktau_allpairs_range, plus KTAU_EINVAL for a scheme that cannot hold n. */
int ktau_prepare(const float* X_dev, int64_t m, int64_t n, int64_t* out_n1_dev,
                 void* workspace_dev, size_t ws_bytes, void* stream);
int ktau_pairs(int64_t m, int64_t n, int64_t J_begin, int64_t J_end,
               ktau_pair_out out, void* workspace_dev, size_t ws_bytes,
               int scheme, int q, void* stream);

/* Waits for `stream`, then returns the status latched in a workspace by the
 * last call that used it (KTAU_ENAN if the input held a NaN: a NaN has no
 * order, so the ranks of Sec. 3 do not exist; KTAU_EINVAL if a permutation
 * given to ktau_perm_test was not one; else KTAU_OK), and clears it.
 * KTAU_EDEVICE if the synchronisation or the copy fails. */
int ktau_status(void* workspace_dev, void* stream);


/* ---------------------------------------------------------------------------
 * Per-pair schemes and an explicit-scheme entry point (for tuning and tests).
 * Network schemes (numbers 0 .. 19) are a group size (8, 16 or 32 lanes of a
 * wave, a whole 64-lane wave, or a 256-lane workgroup) and a number K of keys
 * per lane; they sort and count a whole pair in registers and handle
 * n <= lanes * K (at most 32768).  The merge schemes "merge_k32" and
 * "merge_k64" (the two numbers after them) give each pair a workgroup of
 * ceil(n / 64K) waves: each wave sorts and counts a chunk of 64 K samples
 * with the network, and the merge levels above the chunks are counted by a
 * merge path in LDS (Algorithm 2's count of right elements taken before
 * waiting left ones); they handle n <= 32768 and n <= 65536 and are the
 * default above 4096 samples.
 * ------------------------------------------------------------------------- */

/* The naive count of Sec. 3.1 (Algorithm 1: all n(n-1)/2 sample pairs of a
 * pair of rows compared), as a scheme of the plain entry points (ktau_pairs,
 * ktau_allpairs_ex) for n <= 256.  The comparisons are made once
 * per row by ktau_prepare and kept in the workspace as bit sets (for every
 * sample, the samples ranked below it and those tied with it), so a pair
 * costs an AND and a population count per 32 sample pairs; counts and tau are
 * the same, bit for bit, as the network schemes'.  Its default tile edge is
 * 16.  Not a member of the numbered schemes (ktau_scheme_count).  Batches
 * take it too (ktau_batch_opts.force_scheme, or the autotuner's choice for
 * sample-count classes up to 256), and so do queries against a database
 * created with it (ktau_db_create_ex; the default of ktau_db_create up to 128
 * samples); the permutation test does not. */
#define KTAU_SCHEME_NAIVE 100

/* The numbered pair schemes: ways of running Sec. 3.2 Steps 1-5 for one pair
 * on a group of lanes (Step 3's count on a tagged sorting network, or on a
 * network per chunk and merge paths above it for long rows). */
int ktau_scheme_count(void);
const char* ktau_scheme_name(int scheme);      /* "invalid" if out of range   */
int64_t ktau_scheme_capacity(int scheme);      /* largest n; -1 if invalid    */
int ktau_default_scheme(int64_t n);
/* The scheme the plain calls pick for n: KTAU_SCHEME_NAIVE where it measured
 * faster than the network, else ktau_default_scheme(n). */
int ktau_plain_default_scheme(int64_t n);
/* The tile edge the plain calls pick for m rows of n samples with scheme
 * ktau_plain_default_scheme(n) (Sec. 4.2, Eq. 11-14: q x q tiles of pairs). */
int ktau_plain_default_q(int64_t m, int64_t n);

/* ktau_allpairs (J_begin < 0) or ktau_allpairs_range (J_begin >= 0) with the
 * scheme (a numbered scheme or KTAU_SCHEME_NAIVE) and tile edge q (1..64,
 * the q x q tiles of Sec. 4.2) chosen by the caller; scheme < 0 or q <= 0 pick
 * the defaults.  KTAU_EINVAL if the scheme cannot hold n. */
int ktau_allpairs_ex(const float* X_dev, int64_t m, int64_t n, int64_t J_begin,
                     int64_t J_end, ktau_pair_out out, void* workspace_dev,
                     size_t ws_bytes, int scheme, int q, void* stream);
/* ---------------------------------------------------------------------------
 * Batched all-pairs: many independent matrices of uneven (m, n) in one
 * persistent launch per scheme class.  Workgroups take q x q tiles (Sec. 4.2)
 * of any matrix of the class from atomic counters -- the shared-counter
 * distribution that Sec. 4.1 names for jobs of varied cost; one counter per
 * XCD's stretch of the tiles, with stealing between stretches -- so small
 * matrices do not leave the device idle.  A matrix of 8192 rows or more on a
 * network scheme runs instead as a plain tile launch of its own (a workgroup
 * per tile; a tuned tile edge of 8 or more becomes 16).  The launch sequence (status clear, one pre-pass over
 * all rows, the pair kernels, the heavy-tie composite pass) is captured in a
 * hipGraph on the first ktau_batch_run and replayed afterwards.
 * ------------------------------------------------------------------------- */

typedef struct ktau_matrix {
  const float* X_dev;   /* m x n float32, row-major; read by every run        */
  int64_t m, n;         /* 2 <= m, 2 <= n <= KTAU_MAX_N                        */
  ktau_pair_out out;    /* device results for all m(m-1)/2 strict jobs; NULLs ok */
} ktau_matrix;

typedef struct ktau_batch_opts {
  int32_t use_graph;      /* 1 (default): capture once in a hipGraph, replay   */
  int32_t autotune;       /* 1 (default): (scheme, q) per sample-count class by
                             measurement on this device; 0: built-in defaults   */
  int32_t force_scheme;   /* >= 0: this scheme (a numbered one or
                             KTAU_SCHEME_NAIVE) for every matrix (-1 default) */
  int32_t force_q;        /* > 0: this tile edge for every matrix (0 default)  */
  const char* tune_cache; /* autotune cache file (NULL: $KTAU_TUNE_CACHE, else
                             in-process only)                                   */
} ktau_batch_opts;

typedef struct ktau_batch ktau_batch;   /* opaque plan, owned by the library */

void ktau_batch_default_opts(ktau_batch_opts* opts_host);

/* Validates every matrix, chooses each one's (scheme, q), and allocates the
 * plan's device arena (rank workspaces for all matrices plus descriptors;
 * about 10 m ceil128(n) bytes per matrix, plus 256 KB per row, for at most
 * 256 rows, of sort scratch where n > 16384).  The matrices' X_dev and output
 * arrays are the caller's and must stay valid while the plan is used.
 * Autotuning, when a sample-count class is not yet tuned, times the
 * candidates on the first rows of the class's matrix with the most rows
 * (launches on `stream`, blocking until they finish). */
int ktau_batch_create(const ktau_matrix* mats_host, int64_t count,
                      const ktau_batch_opts* opts_host, void* stream,
                      ktau_batch** plan_out);

/* Enqueues one full run of the plan on `stream` (asynchronous). */
int ktau_batch_run(ktau_batch* plan, void* stream);

/* Waits for `stream`; KTAU_ENAN if any matrix of the last run held a NaN. */
int ktau_batch_status(ktau_batch* plan, void* stream);

/* The (scheme, q) chosen for matrix i. */
int ktau_batch_plan(const ktau_batch* plan, int64_t i, int32_t* scheme_host,
                    int32_t* q_host);

void ktau_batch_destroy(ktau_batch* plan);

/* Autotuner: for each n in ns_host, the (scheme, q) the batch planner would
 * use, tuning any class not yet in the process table or the cache file on a
 * synthetic matrix with a zero tie run in every row (timing launches on
 * `stream`, synchronous). */
int ktau_autotune(const int64_t* ns_host, int64_t count, const char* cache_path,
                  void* stream, int32_t* schemes_out_host, int32_t* q_out_host);

/* ---------------------------------------------------------------------------
 * Permutation test (Sec. 1: P-values of tau by permutation test, which needs
 * many tau of every pair).
 * ------------------------------------------------------------------------- */

/* Device workspace bytes of ktau_perm_test (0 for a bad shape or B < 1). */
size_t ktau_perm_workspace_size(int64_t m, int64_t n, int64_t B);

/* For each strict pair (y, x) with job id J in [J_begin, J_end) (J_begin < 0:
 * all jobs): |n_c - n_d| of row y against row x, and against row x with its
 * samples permuted by each of the B permutations (x'[t] = x[perms[b*n + t]]);
 * count_out[J - J_begin] (int64) = the number of permutations whose
 * |n_c - n_d| is at least the observed one, p_out[J - J_begin] (double,
 * may be NULL) = (1 + count) / (B + 1).  tau_B's denominator does not change
 * under the permutations, so this is the two-sided permutation test of tau_B,
 * decided in exact integers.
 * perms_dev: uint16 [B][n], each row a permutation of 0..n-1 (checked on the
 * device: a bad row latches KTAU_EINVAL in the workspace header and nothing
 * is written; read it with ktau_status).  X_dev as in ktau_allpairs; the
 * caller owns every buffer.  Errors returned at once: KTAU_EINVAL (null
 * pointer, B < 1 or B >= 2^31, misaligned workspace), KTAU_ERANGE (n >
 * KTAU_MAX_N or a bad job range), KTAU_ENOMEM (workspace too small). */
int ktau_perm_test(const float* X_dev, int64_t m, int64_t n, const uint16_t* perms_dev,
                   int64_t B, int64_t J_begin, int64_t J_end, int64_t* count_out_dev,
                   double* p_out_dev, void* workspace_dev, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Query-vs-database search (Sec. 1: select the subject rows of a database
 * that are co-expressed with a query row, ranking query-subject pairs by
 * their score).  The score is tau_B; results are the k database rows of
 * largest |tau_B| per query, ordered by |tau_B| descending then row index
 * ascending; rows whose tau_B is NaN (a constant row) are never returned;
 * missing results are idx -1, tau NaN, nd -1.
 * ------------------------------------------------------------------------- */

#define KTAU_MAX_K 1024

typedef struct ktau_db ktau_db;   /* opaque: ranked database resident in HBM */

/* Ranks the m x n database X_dev once into library-owned device memory
 * (about 10 m ceil128(n) bytes; Sec. 3: each vector ranked once
 * beforehand); X_dev may be freed afterwards.  Synchronises `stream`;
 * KTAU_ENAN if X_dev holds a NaN, KTAU_ERANGE if n > KTAU_MAX_N_NETWORK,
 * KTAU_EINVAL for a null pointer, m < 1 or n < 2, KTAU_ENOMEM if the device
 * allocation fails. */
int ktau_db_create(const float* X_dev, int64_t m, int64_t n, void* stream,
                   ktau_db** db_out);
/* The same with the scheme of the query pair kernel chosen by the caller:
 * scheme < 0 takes the default for n (KTAU_SCHEME_NAIVE up to 128 samples,
 * else ktau_default_scheme(n)); a network scheme must hold n and
 * KTAU_SCHEME_NAIVE needs n <= 256 (then the database also keeps its rows'
 * bit sets, 8 n ceil(n/32) bytes per row rounded up); anything else is
 * KTAU_EINVAL.  For tuning and tests. */
int ktau_db_create_ex(const float* X_dev, int64_t m, int64_t n, int scheme, void* stream,
                      ktau_db** db_out);
void ktau_db_destroy(ktau_db* db);
int64_t ktau_db_rows(const ktau_db* db);
int64_t ktau_db_samples(const ktau_db* db);

/* Device workspace bytes of a ktau_query call with nq query rows. */
size_t ktau_query_workspace_size(const ktau_db* db, int64_t nq, int64_t k);

/* nq query rows Q_dev (nq x n float32, n = the database's) against every
 * database row.  idx_out[nq*k] (int64), tau_out[nq*k] (double, signed
 * tau_B) and nd_out[nq*k] (int64 n_d) are device arrays; tau_out and nd_out
 * may be NULL.  Stream-ordered; a NaN query is latched in the workspace
 * header (ktau_status). */
int ktau_query(const ktau_db* db, const float* Q_dev, int64_t nq, int64_t k,
               int64_t* idx_out_dev, double* tau_out_dev, int64_t* nd_out_dev,
               void* workspace_dev, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Query server: continuous batching over a resident database, serving the
 * query-vs-database search of Sec. 1 (ktau_query per launch).
 *
 * Requests (1..many query rows each, a k each) are queued in arrival order by
 * ktau_server_submit and served by a worker thread inside the library.  When
 * a slot (a stream) is free, the worker forms a launch from the head of the
 * queue -- the head and the requests right behind it, up to
 * max_batch_queries rows; the launch computes the largest k among them and
 * each request keeps its own first k -- and admits it only if its device
 * memory fits in what is left of the mem_budget_bytes pool; otherwise it
 * waits until running launches complete.  A finished launch wakes the worker
 * from its stream (a host function), so admission follows completion without
 * polling.  Launches on different slots overlap on the
 * device.  Each request's results are identical whether it ran alone or
 * merged with others.  Latency = completion minus submission (queueing
 * included).  Intended for callers that cannot wait on the device: all calls
 * take and return host memory.
 * ------------------------------------------------------------------------- */

typedef struct ktau_server ktau_server;

typedef struct ktau_server_cfg {
  int32_t slots;             /* concurrent launches (streams); default 2        */
  int32_t max_batch_queries; /* rows merged into one launch; default 256        */
  int64_t mem_budget_bytes;  /* device pool for running launches; default 1 GiB */
  int32_t max_queue;         /* queued requests before submit blocks/refuses    */
  int32_t k_max;             /* largest k accepted; default 128 (<= KTAU_MAX_K) */
} ktau_server_cfg;

typedef struct ktau_latency {
  double queue_us;           /* submission -> launch                           */
  double device_us;          /* launch -> results on the host                  */
  double total_us;           /* submission -> results on the host              */
  int64_t batch_queries;     /* rows in the launch that served the request     */
  int64_t batch_requests;    /* requests merged into that launch               */
} ktau_latency;

typedef struct ktau_server_stats {
  int64_t launches, merged_requests, completed, failed;
  int64_t peak_pool_bytes, peak_running, queued;
} ktau_server_counters;

void ktau_server_default_cfg(ktau_server_cfg* cfg_host);

/* Starts a server over `db` (which must outlive it) on the current device;
 * allocates the pool and per-slot pinned staging. */
int ktau_server_create(const ktau_db* db, const ktau_server_cfg* cfg_host,
                       ktau_server** server_out);

/* Queues nq query rows (q_host: nq x n float32, copied before returning) for
 * top-k.  KTAU_ENAN for NaN rows, KTAU_ENOMEM if the request can never fit
 * the pool, KTAU_EBUSY if the queue is full and blocking == 0 (blocking != 0
 * waits for room).  *ticket_out identifies the request. */
int ktau_server_submit(ktau_server* server, const float* q_host, int64_t nq, int64_t k,
                       int blocking, int64_t* ticket_out);

/* Waits (timeout_ms < 0: forever) for a request; on success copies nq*k
 * results into idx_host / tau_host / nd_host (any may be NULL) and its
 * latency into lat_host, and forgets the ticket.  Returns the request's
 * status: KTAU_OK, KTAU_ECANCELED (cancelled or failed in its launch),
 * KTAU_ETIMEDOUT (still pending; the ticket stays valid). */
int ktau_server_wait(ktau_server* server, int64_t ticket, int64_t* idx_host,
                     double* tau_host, int64_t* nd_host, ktau_latency* lat_host,
                     int64_t timeout_ms);

/* Removes a request that has not been launched yet (KTAU_EBUSY otherwise). */
int ktau_server_cancel(ktau_server* server, int64_t ticket);

/* Failure drill: a queued request is launched alone and completes with
 * KTAU_ECANCELED without touching the device (KTAU_EBUSY if not queued). */
int ktau_server_inject_failure(ktau_server* server, int64_t ticket);

/* Stops (paused != 0) or resumes admitting queued requests to the device.
 * Submission goes on while paused and running launches complete; requests
 * queued meanwhile are batched by the policy above when admission resumes.
 * For operators (draining, maintenance) and for tests that need requests
 * queued together.  ktau_server_destroy resumes admission itself. */
int ktau_server_pause(ktau_server* server, int paused);

int ktau_server_stats(ktau_server* server, ktau_server_counters* stats_host);

/* Device pool bytes one launch of nq rows with this k takes (0 if invalid),
 * for sizing mem_budget_bytes. */
size_t ktau_server_launch_bytes(const ktau_server* server, int64_t nq, int64_t k);

/* Serves everything already queued, then stops the worker and frees the
 * server. */
void ktau_server_destroy(ktau_server* server);

/* ---------------------------------------------------------------------------
 * Diagnostics: kernels with a known amount of work per launch, for the
 * callers' own measurement of the peaks the rooflines are quoted against.
 * They are not part of the paper's method (no passage defines them); Sec. 5
 * is where the paper reports its own kernels' rates.
 * ------------------------------------------------------------------------- */

/* Threads per workgroup of the probes, int32 adds per thread per iteration of
 * the VALU probe, LDS bytes read per thread per iteration of the LDS probe. */
int ktau_probe_threads(void);
int ktau_probe_valu_ops_per_iter(void);
int ktau_probe_lds_bytes_per_iter(void);

/* Launch `blocks` workgroups of the VALU probe (int32 adds, 16 independent
 * chains per lane) or the LDS probe (conflict-free 16-byte reads of a 64 KB
 * workgroup buffer), `iters` iterations each, on `stream`; out_dev receives
 * one uint32 per thread (blocks * ktau_probe_threads()).  KTAU_EINVAL for a
 * null out_dev, blocks < 1 or iters < 1. */
int ktau_probe_valu(uint32_t* out_dev, int64_t blocks, int iters, void* stream);
int ktau_probe_lds(uint32_t* out_dev, int64_t blocks, int iters, void* stream);

/* Issue-rate probe: as the VALU probe, with the 16 chains per lane built from
 * one instruction kind: 0 int32 add (v_add_u32), 1 packed f16 minimum with a
 * negated operand (v_pk_minimum3_f16), 2 unsigned 16-bit dot product with
 * accumulate (v_dot2_u32_u16), 3 packed u16 minimum and add (v_pk_min_u16,
 * v_pk_add_u16).  ktau_probe_issue_instrs_per_iter gives the wave
 * instructions per wave and iteration of a kind (-1: no such kind);
 * KTAU_EINVAL as ktau_probe_valu, or for a kind outside 0..3. */
int ktau_probe_issue_instrs_per_iter(int kind);
int ktau_probe_issue(uint32_t* out_dev, int64_t blocks, int iters, int kind, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* KTAU_H */
