/*
 * mipq -- product quantisation and inverted-index hot path for MI355X (gfx950).
 *
 * C ABI.  Every entry point returns an int status (MIPQ_OK or a negative
 * MIPQ_E* code), never throws and never aborts; the text of the last error on
 * the calling thread is returned by mipq_last_error().
 *
 * Memory.  Unless stated otherwise every array argument is a DEVICE pointer
 * owned by the caller; the library allocates no device memory.  Calls that
 * need scratch space take a caller-owned device workspace `ws` of `ws_bytes`
 * bytes (at least what the matching *_workspace_size() query returns, aligned
 * to 256 bytes) and fail with MIPQ_ENOMEM when it is smaller.  The workspace
 * contents on entry are ignored.
 *
 * Streams.  `stream` is a hipStream_t (NULL = the default stream).  Calls only
 * enqueue work on it and return before it runs; outputs are valid once the
 * stream has reached the end of the call.  Calls that share a workspace must
 * be ordered on one stream.
 *
 * Layouts.
 *   rows       float32 [n][d], row-major, rows contiguous
 *   codebook   float32 [m][ks][ds], ds = d / m: centroid k of subspace j is the
 *              ds floats at codebook + (j*ks + k)*ds; subspace j covers the
 *              contiguous columns [j*ds, (j+1)*ds)
 *   codes      uint8 [n][m] (ks <= 256)
 *
 * Precision (the arithmetic used to rank candidate centroids):
 *   MIPQ_FP32  every candidate distance in float32 from the difference form
 *   MIPQ_BF16  distances ranked on matrix cores from bfloat16 operands split
 *              into high and low parts, with float32 accumulation; every
 *              (row, subspace) whose two best candidates are not separated
 *              by a proven error bound is re-decided in MIPQ_FP32 arithmetic.
 *   MIPQ_FP8   as MIPQ_BF16 with OCP E4M3 operands (high and low parts) under
 *              a power-of-two scale per subspace; its wider error bound sends
 *              more pairs to the exact re-decision.  Not offered for the
 *              coarse quantiser, the batched fit or the index build.
 * All give the same codes: the code of a (row, subspace) is the lowest index
 * k minimising the float32 difference-form distance
 *     sum over t ascending of (x_t - c_kt)^2,
 * with every subtraction, square and sum rounded to float32 (no fused
 * multiply-add).  Centroid sums, objectives and reconstruction errors are
 * accumulated in float64.
 */
#ifndef MIPQ_H
#define MIPQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MIPQ_ABI_VERSION 2

enum mipq_status {
  MIPQ_OK = 0,
  MIPQ_EINVAL = -1,       /* bad shape, null required pointer, bad enum */
  MIPQ_ENOMEM = -2,       /* workspace smaller than the *_workspace_size() query */
  MIPQ_EHIP = -3,         /* a HIP runtime call failed (text in mipq_last_error) */
  MIPQ_EUNSUPPORTED = -4, /* valid request this build does not implement */
  MIPQ_ENONFINITE = -5    /* MIPQ_CHECK_FINITE found a NaN or infinite input value */
};

/* Call flags (bit set) of mipq_pq_fit and mipq_pq_encode.
 *   MIPQ_CHECK_FINITE   before any other work, check that every input value
 *       the call reads (the training or encoded rows, an initial codebook, the
 *       codebook to encode with) is finite; if one is not, return
 *       MIPQ_ENONFINITE with nothing written.  The check waits for `stream`
 *       (the call is then synchronous up to the check).  Without the flag,
 *       non-finite inputs give unspecified codes: the matrix-core paths
 *       order NaN estimates differently from the float32 rule, in which a NaN
 *       distance never wins, so a row with a NaN in a subspace gets code 0
 *       there on the FP32 path and an arbitrary code on the others.
 *   MIPQ_DETERMINISTIC  (mipq_pq_fit) the float64 centroid sums of a round
 *       are formed in a fixed order (rows of each chunk by centroid, in row
 *       order, chunks in order) instead of by atomic additions, so two runs
 *       on the same inputs give bit-identical codebooks, labels and
 *       objectives.  Slower; the sums may differ from the default mode's in
 *       the last bits. */
enum mipq_flags { MIPQ_CHECK_FINITE = 1, MIPQ_DETERMINISTIC = 2 };

enum mipq_precision { MIPQ_FP32 = 0, MIPQ_BF16 = 1, MIPQ_FP8 = 2 };

/* Version of this header's ABI (MIPQ_ABI_VERSION). */
int mipq_abi_version(void);

/* Text of the last failure on the calling thread ("" if none). */
const char* mipq_last_error(void);

/* -------------------------------------------------------------------------
 * k-means codebook fit (paper Section 2.1: split the d dimensions into m
 * subspaces and fit ks centroids in each with k-means).
 *
 * Lloyd iteration, `iters` rounds, no tolerance test.  Each round assigns
 * every training row to its nearest centroid in each subspace (the code rule
 * above) and replaces every centroid that received rows by the float64 mean
 * of those rows; a centroid that received none keeps its value.
 *
 *   x            training rows [n][d] (or the rows indexed by train_rows)
 *   train_rows   optional int64 [n_train]: when non-NULL the training set is
 *                x[train_rows[i]] (gathered into the workspace), and the
 *                n argument is the number of rows of x
 *   n_train      number of training rows (used only with train_rows)
 *   init_rows    int64 [m][ks]: centroid k of subspace j starts as the
 *                subspace-j block of training row init_rows[j*ks + k];
 *                ignored when init_codebook is non-NULL
 *   init_codebook optional float32 [m][ks][ds] starting codebook (resume)
 *   codebook     OUT float32 [m][ks][ds]: float64 centroids rounded to nearest
 *   codebook64   OUT optional float64 [m][ks][ds]
 *   labels       OUT optional uint8 [n_train][m]: codes of the LAST
 *                assignment (against the codebook before the last update)
 *   objective    OUT optional float64 [iters]: objective[t] = sum over rows,
 *                subspaces and dimensions of (x - c)^2 in float64, c the
 *                float32 centroid chosen in round t
 *   rescored     OUT optional int64 [iters]: (row, subspace) pairs of round
 *                t's assignment whose matrix-core ranking was not separated
 *                by its error bound and were re-decided with the float32 rule
 *                (0 for MIPQ_FP32)
 *   flags        MIPQ_CHECK_FINITE, MIPQ_DETERMINISTIC (see mipq_flags)
 * Requirements: d % m == 0, d/m <= 16 (BF16, FP8) or <= 48 (FP32),
 * 1 <= ks <= 256, n_train >= 1, iters >= 0, init rows in range.
 * ------------------------------------------------------------------------- */
size_t mipq_pq_fit_workspace_size(int64_t n_train, int d, int m, int ks, int iters, int precision);
int mipq_pq_fit(const float* x, int64_t n, const int64_t* train_rows, int64_t n_train,
                int d, int m, int ks, int iters,
                const int64_t* init_rows, const float* init_codebook, int precision, int flags,
                float* codebook, double* codebook64, uint8_t* labels, double* objective,
                int64_t* rescored, void* ws, size_t ws_bytes, void* stream);

/* -------------------------------------------------------------------------
 * Encode (paper Section 2.1: each row of each subspace is represented by
 * its nearest subspace centroid, so a row becomes m codes; the paper's
 * library also gives the distance of each item to its centroid).
 *
 *   codes     OUT uint8 [n][m]
 *   min_dist  OUT optional float32 [n][m]: the float32-rule distance of the
 *             subspace block of each row to its chosen centroid (the value
 *             the code minimises)
 *   sse_rmse  OUT optional float64 [2]: SSE and RMSE of the codes, exactly as
 *             mipq_pq_decode_rmse defines them (float64 squares of the
 *             float64 differences); the sum order differs, so the two agree
 *             to float64 rounding, not bit for bit
 *   rescored  OUT optional int64 [1]: number of (row, subspace) pairs the
 *             BF16 path re-decided in FP32 arithmetic (0 for MIPQ_FP32)
 *   flags     MIPQ_CHECK_FINITE (see mipq_flags)
 * ------------------------------------------------------------------------- */
size_t mipq_pq_encode_workspace_size(int64_t n, int d, int m, int ks, int precision);
int mipq_pq_encode(const float* x, int64_t n, int d, int m, int ks, const float* codebook,
                   int precision, int flags, uint8_t* codes, float* min_dist, double* sse_rmse,
                   int64_t* rescored, void* ws, size_t ws_bytes, void* stream);

/* -------------------------------------------------------------------------
 * Encode that allocates nothing, for callers that cannot allocate device
 * memory or pass a workspace: code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation.
 *
 * Same arguments, rule and outputs as mipq_pq_encode, without the workspace.
 * Its scratch memory (packed centroid operands, squared-error partials) is a
 * fixed array of MIPQ_NOALLOC_SCRATCH_BYTES in device memory, one per GPU the
 * library runs on, held until the process ends; the call takes no allocation
 * of any kind.  Every call on a GPU uses that GPU's array: calls that overlap
 * on one GPU race (order them on one stream).
 * Limits: n <= MIPQ_NOALLOC_MAX_N and the scratch mipq_pq_encode_workspace_size
 * reports within MIPQ_NOALLOC_SCRATCH_BYTES (MIPQ_ENOMEM otherwise; m <= 64
 * with d/m <= 16 always fits); MIPQ_CHECK_FINITE is not accepted (it copies a
 * flag to the host), MIPQ_EINVAL.
 * ------------------------------------------------------------------------- */
#define MIPQ_NOALLOC_SCRATCH_BYTES ((size_t)8 << 20)
#define MIPQ_NOALLOC_MAX_N ((int64_t)1 << 24)
int mipq_pq_encode_noalloc(const float* x, int64_t n, int d, int m, int ks, const float* codebook,
                           int precision, int flags, uint8_t* codes, float* min_dist, double* sse_rmse,
                           int64_t* rescored, void* stream);

/* -------------------------------------------------------------------------
 * Decode and reconstruction error (paper Section 3: rows are encoded and
 * decoded to measure the reconstruction RMSE).
 *
 *   x_hat     OUT optional float32 [n][d]: concatenated coded centroids
 *   x         optional rows [n][d]; required for the error
 *   sse_rmse  OUT optional float64 [2]: SSE = sum of (x - x_hat)^2 in float64,
 *             RMSE = sqrt(SSE / (n*d)); requires x
 * ------------------------------------------------------------------------- */
size_t mipq_pq_decode_rmse_workspace_size(int64_t n, int d, int m, int ks);
int mipq_pq_decode_rmse(const uint8_t* codes, int64_t n, int d, int m, int ks,
                        const float* codebook, const float* x, float* x_hat, double* sse_rmse,
                        void* ws, size_t ws_bytes, void* stream);

/* -------------------------------------------------------------------------
 * Batched fit + encode of many independent problems (paper Section 3: the
 * rows are split into chunks that are quantised in parallel, each chunk with
 * its own codebook).
 *
 * Problem p fits its own codebook on all of its own rows (the Lloyd rounds
 * of mipq_pq_fit with train_rows NULL, `iters` rounds, from its init_rows),
 * encodes all of its rows with the final codebook and, when sse_rmse is
 * non-NULL, reports the reconstruction error of those codes.  All problems
 * share d, m, ks and precision (MIPQ_BF16 only).  Per problem the outputs are
 * those of mipq_pq_fit + mipq_pq_encode + mipq_pq_decode_rmse on that
 * problem: same code rule, same reduction order for the error and, when any
 * problem returns its objective (or the plan is deterministic), the same row
 * chunks for the float64 centroid sums and the same reduction order for the
 * objective.  (Within a chunk the float64 sums are formed by atomic
 * additions, so their last bits, and hence rarely a float32 centroid, can
 * differ between any two runs; integer-valued rows make every sum exact.)
 *
 * Each phase is one launch over all problems.  Without objectives (and not
 * deterministic) a Lloyd round is one fused launch over all (problem, row
 * chunk of at most 32,768 rows, subspace) items: the matrix-core assignment
 * and the float64 sums of the chunk's rows.  Otherwise a round is a
 * persistent matrix-core assignment over the flat list of (problem,
 * 4-subspace group, 32-row tile) units and one accumulation launch over all
 * (problem, row chunk, subspace) items.  Then one finalisation launch over
 * all (problem, subspace, centroid tile) blocks.  The final encode is the
 * persistent assignment.
 */
typedef struct mipq_problem {
  const float* x;            /* rows [n][d] */
  int64_t n;                 /* number of rows, >= 1, n*m < 2^32 */
  const int64_t* init_rows;  /* int64 [m][ks]: centroid k of subspace j starts as
                                row init_rows[j*ks + k] of x */
  float* codebook;           /* OUT float32 [m][ks][ds] */
  uint8_t* codes;            /* OUT uint8 [n][m]: codes against the final codebook */
  double* sse_rmse;          /* OUT optional float64 [2]: SSE and RMSE of the codes */
  double* objective;         /* OUT optional float64 [iters] (as mipq_pq_fit) */
} mipq_problem;

/* Launch plan for one problem table: the grid and register/occupancy variant
 * of the persistent assignment and, with MIPQ_PLAN_GRAPH, the launch sequence
 * recorded as HIP graphs (set-up, one Lloyd round replayed `iters` times,
 * encode + error).  Neither choice changes any output: every grid and variant
 * computes the same codes and codebooks.
 *
 * MIPQ_PLAN_AUTOTUNE: the choice is looked up in a tuning cache, keyed by the
 * device architecture, subspace width, ks, m and the power-of-two buckets of
 * the total rows and the problem count.  On a miss (or with MIPQ_PLAN_RETUNE,
 * which ignores the cache) every variant is timed at 1, 2, 4, 8 and 16 times its
 * resident blocks on the problems' own round-0 assignment (which writes their
 * codes; the fit overwrites them), and the fastest is stored.  The cache is
 * a JSON object, one entry per line, at $MIPQ_TUNE_CACHE, else
 * $HOME/.cache/mipq/autotune.json; it is rewritten through a temporary file
 * and rename.  A cache that cannot be read or written is treated as empty and
 * never fails the call.  Without MIPQ_PLAN_AUTOTUNE: variant 0 at twice its
 * resident blocks.
 *
 * A plan is bound to the problem table (pointers and sizes), the shapes and
 * the workspace it was made with; the plan object is host memory owned by the
 * library.  mipq_plan_create waits for `stream`.  Graphs are replayed on
 * whatever stream mipq_pq_fit_batched is given. */
typedef struct mipq_plan mipq_plan;
/* MIPQ_PLAN_DETERMINISTIC: the float64 centroid sums in a fixed order, as
 * MIPQ_DETERMINISTIC does for mipq_pq_fit (runs of the plan are then
 * bit-identical). */
enum mipq_plan_flags {
  MIPQ_PLAN_AUTOTUNE = 1,
  MIPQ_PLAN_GRAPH = 2,
  MIPQ_PLAN_DETERMINISTIC = 4,
  MIPQ_PLAN_RETUNE = 8
};

/* n: host int64 [nprob], the rows of every problem. */
size_t mipq_pq_fit_batched_workspace_size(const int64_t* n, int nprob, int d, int m, int ks, int iters,
                                          int precision);
/* probs: host array [nprob].  plan: optional (NULL: default grid, no graphs;
 * the problem table is then copied into the workspace and the call waits
 * for that copy).  rescored: optional int64 [1], pairs the final encode
 * re-decided with the exact rule, summed over problems. */
int mipq_pq_fit_batched(const mipq_problem* probs, int nprob, int d, int m, int ks, int iters, int precision,
                        const mipq_plan* plan, int64_t* rescored, void* ws, size_t ws_bytes, void* stream);
int mipq_plan_create(mipq_plan** plan, const mipq_problem* probs, int nprob, int d, int m, int ks, int iters,
                     int precision, int flags, void* ws, size_t ws_bytes, void* stream);
/* info (host int64 [count], count >= 6): [0] assignment grid, [1] resident
 * blocks of the chosen variant (rounded up to a multiple of 8), [2] graphs
 * recorded (0/1), [3] variant, [4] choice taken from the tuning cache (0/1),
 * [5] candidates timed by this call, then (grid, variant, nanoseconds per
 * launch) for each candidate.  Entries beyond what exists are set to 0. */
int mipq_plan_info(const mipq_plan* plan, int64_t* info, int count);
int mipq_plan_destroy(mipq_plan* plan);

/* -------------------------------------------------------------------------
 * Decoded centroids (paper Section 3: every chunk returns its centroids as
 * rows, which are pooled into a centroid dataset for the global fit).
 *
 *   codebooks  float32 [nbooks][m][ks][ds]
 *   out        OUT float32 [nbooks*ks][d]: row b*ks + k is the decode of the
 *              code row (k, k, ..., k) with codebook b
 * ------------------------------------------------------------------------- */
int mipq_pq_decode_centroids(const float* codebooks, int64_t nbooks, int d, int m, int ks, float* out,
                              void* stream);

/* -------------------------------------------------------------------------
 * Inverted file (paper Section 2.2: the ids of rows are stored per bucket and
 * a query returns its first to k-th nearest neighbours).  Buckets are coarse
 * k-means lists; each row stores the PQ codes of its residual x - c_list.
 *
 * Coarse rule: label = lowest l minimising the sum over dimensions t
 * ascending of (x_t - c_lt)^2 with the difference rounded to float32 and the
 * squares and sums in float64.  MIPQ_BF16 ranks on matrix cores and
 * re-decides unseparated rows with that rule; MIPQ_FP32 applies it directly.
 *
 * mipq_coarse_assign: labels int32 [n] of rows x [n][d] against coarse
 *   float32 [kc][d]; rescored: optional int64 [1] counter (rows re-decided).
 *
 * mipq_ii_build:
 *   x             rows [n][d]
 *   train_rows    int64 [n_train]: the training sample (rows of x) for the
 *                 coarse quantiser and the residual PQ
 *   coarse_init   int64 [kc]: coarse centroid l starts as training row
 *                 coarse_init[l] (an index into the sample)
 *   pq_init       int64 [m][ks]: residual PQ initial rows (indices into the
 *                 sample), as mipq_pq_fit's init_rows
 *   coarse        OUT float32 [kc][d]   pq_codebook OUT float32 [m][ks][d/m]
 *   offsets       OUT int64 [kc+1]: list l holds sorted positions
 *                 offsets[l] .. offsets[l+1]-1
 *   ids           OUT int32 [n]: row ids by list, ascending inside a list
 *   codes_sorted  OUT uint8 [n][m]: residual codes of ids[i] at row i
 *   labels        OUT optional int32 [n]: coarse label of every row
 *   coarse_objective OUT optional float64 [coarse_iters]
 * Steps: coarse Lloyd (coarse_iters rounds, centroid = float64 mean of its
 * rows in id order, empty keeps its value) on the sample; final labels of the
 * sample; residual PQ fit (pq_iters rounds) on the sample's residuals; labels
 * and residual codes of all rows; stable bucketing by label.
 * Requirements: kc <= 65536, n < 2^31, d % m == 0, d % 16 == 0 and d <= 256
 * for MIPQ_BF16 coarse ranking.
 * ------------------------------------------------------------------------- */
/* mipq_kmeans_fit: the coarse quantiser on its own (k-means over whole rows,
 *   k <= 65536 centroids): Lloyd, `iters` rounds, assignments by the coarse
 *   rule above, centroid = float64 mean of its rows summed in id order (an
 *   empty centroid keeps its value).  Steps 1-2 of mipq_ii_build.
 *   x, train_rows, n_train  as in mipq_pq_fit (train_rows optional)
 *   init_rows     int64 [k]: centroid l starts as training row init_rows[l]
 *   centroids     OUT float32 [k][d]
 *   labels        OUT optional int32 [n_train]: the last assignment (against
 *                 the centroids before the last update); unwritten if iters == 0
 *   objective     OUT optional float64 [iters]: sum over rows of the squared
 *                 distance (float64) to the float32 centroid chosen in round t
 *   precision     MIPQ_FP32 or MIPQ_BF16 (ranking on matrix cores, exact decisions)
 */
size_t mipq_kmeans_fit_workspace_size(int64_t n_train, int d, int k, int iters, int precision);
int mipq_kmeans_fit(const float* x, int64_t n, const int64_t* train_rows, int64_t n_train, int d, int k,
                    int iters, const int64_t* init_rows, int precision, float* centroids, int32_t* labels,
                    double* objective, void* ws, size_t ws_bytes, void* stream);
size_t mipq_coarse_assign_workspace_size(int d, int kc, int precision);
int mipq_coarse_assign(const float* x, int64_t n, int d, const float* coarse, int kc, int precision,
                       int32_t* labels, int64_t* rescored, void* ws, size_t ws_bytes, void* stream);
size_t mipq_ii_build_workspace_size(int64_t n, int d, int kc, int64_t n_train, int m, int ks, int pq_iters,
                                    int coarse_iters, int precision);
int mipq_ii_build(const float* x, int64_t n, int d, int kc, int coarse_iters, const int64_t* train_rows,
                  int64_t n_train, const int64_t* coarse_init, int m, int ks, int pq_iters,
                  const int64_t* pq_init, int precision, float* coarse, float* pq_codebook,
                  int64_t* offsets, int32_t* ids, uint8_t* codes_sorted, int32_t* labels,
                  double* coarse_objective, void* ws, size_t ws_bytes, void* stream);

/* -------------------------------------------------------------------------
 * Index built piecewise (paper Section 3.1.2, the index library: codes are
 * added to an index and indexes are merged, which is how the index is built
 * in parallel over the data chunks of Section 3).
 *
 * mipq_ii_add: the posting lists of rows x [n][d] under fixed quantisers
 *   (coarse float32 [kc][d], pq_codebook float32 [m][ks][d/m], e.g. those of
 *   an mipq_ii_build): coarse labels, residual codes and stable bucketing,
 *   exactly as the last two steps of mipq_ii_build.  Outputs as there:
 *   offsets int64 [kc+1], ids int32 [n] (row ids 0..n-1 of this x, ascending
 *   inside a list), codes_sorted uint8 [n][m], optional labels int32 [n].
 *   n == 0 is valid (all offsets 0).  precision: MIPQ_FP32 or MIPQ_BF16 as
 *   in mipq_ii_build; the code rule and the coarse rule make every row's
 *   label and code independent of the other rows, so adding the rows of
 *   consecutive chunks and merging gives the lists of one call on all rows.
 *
 * mipq_ii_merge: concatenates nparts indexes over consecutive row ranges
 *   (part p covers rows base_p .. base_p + part_n[p] - 1, base_p = sum of
 *   part_n of the parts before it).  List l of the result is list l of part
 *   0, then of part 1, ..., with every id shifted by its part's base.
 *   part_offsets[p] (int64 [kc+1]), part_ids[p] (int32 [part_n[p]]) and
 *   part_codes[p] (uint8 [part_n[p]][m]) are DEVICE pointers held in HOST
 *   arrays of length nparts; the parts must be valid indexes of this kc and
 *   m (offsets non-decreasing from 0 to part_n[p], ids in [0, part_n[p])),
 *   which the call does not check on the device.  Outputs: offsets int64
 *   [kc+1], ids int32 [sum part_n], codes_sorted uint8 [sum part_n][m].
 *   The call copies the part table into the workspace and waits for that
 *   copy on the stream before it returns (the kernels stay queued).
 *   Requirements: 1 <= nparts, kc <= 65536, m <= 256, sum part_n < 2^31.
 * ------------------------------------------------------------------------- */
size_t mipq_ii_add_workspace_size(int64_t n, int d, int kc, int m, int ks, int precision);
int mipq_ii_add(const float* x, int64_t n, int d, const float* coarse, int kc, const float* pq_codebook, int m,
                int ks, int precision, int64_t* offsets, int32_t* ids, uint8_t* codes_sorted, int32_t* labels,
                void* ws, size_t ws_bytes, void* stream);
size_t mipq_ii_merge_workspace_size(int nparts, int kc);
int mipq_ii_merge(const int64_t* const* part_offsets, const int32_t* const* part_ids,
                  const uint8_t* const* part_codes, const int64_t* part_n, int nparts, int kc, int m,
                  int64_t* offsets, int32_t* ids, uint8_t* codes_sorted, void* ws, size_t ws_bytes, void* stream);

/* -------------------------------------------------------------------------
 * ADC search over an index built by mipq_ii_build (paper Section 2.2: the
 * first to k-th nearest neighbours of a query).
 *
 * For query q: the nprobe lists with the smallest coarse distance (coarse
 * rule above, ties to the lower list); for each probed list l a table
 * LUT[j][k] = float32 subspace-j distance (the code rule) of (q - c_l) to the
 * residual centroid C_j[k]; every row of the list scores
 * s = sum over j ascending of LUT[j][code_j] in float32; the topk smallest
 * (s, id) pairs, ascending, are returned (ids -1 and +inf when fewer rows).
 *
 *   q         float32 [nq][d]      out_ids  OUT int32 [nq][topk]
 *   out_dist  OUT float32 [nq][topk]
 *   wide      OUT optional int64 [1]: queries whose probe selection needed the
 *             exact rule on every list
 *   work      OUT optional int64 [4]: work the list scans executed (the exact
 *             skips below avoid the rest): [0] table entries built, [1] rows
 *             given the partial sum over their first 4 subspaces, [2] rows
 *             summed over all subspaces (from the first; a row that passed
 *             the partial sum is counted in both), [3] (query, list) pairs
 *             whose list was scanned (not left at once by the list bound)
 * Requirements: 1 <= nprobe <= min(kc, 256), 1 <= topk <= 1024, d/m in
 * {1, 2, 4, 8, 16}, d <= 16 or d in {32, 64, 96, 128, 192, 256}, and the
 * table with its key buffer within 64 KiB of LDS (m * ks <= 11264 always
 * fits; larger tables return MIPQ_EUNSUPPORTED).
 * ------------------------------------------------------------------------- */
size_t mipq_adc_search_workspace_size(int nq, int d, int kc, int nprobe, int topk);
int mipq_adc_search(const float* q, int nq, int d, const float* coarse, int kc, const float* pq_codebook,
                    int m, int ks, const int64_t* offsets, const int32_t* ids, const uint8_t* codes_sorted,
                    int nprobe, int topk, int32_t* out_ids, float* out_dist, int64_t* wide, int64_t* work,
                    void* ws, size_t ws_bytes, void* stream);

/* -------------------------------------------------------------------------
 * Reconstruction-loss backward with the codes held fixed.
 *
 * For x_hat_n = concatenation over subspaces j of C_j[codes[n][j]] (the
 * decode of Section 3) and L = sum over n of ||x_n - x_hat_n||^2:
 *   dL/dx_n    = 2 g (x_n - x_hat_n)
 *   dL/dC_j[k] = 2 g (cnt_jk C_j[k] - S_jk),  S_jk / cnt_jk the float64 sum /
 *                number of the subspace-j blocks of the rows coded k
 * (setting dL/dC = 0 gives the k-means mean of Section 2.1's fit).
 *
 *   grad_out      optional float64 [1]: upstream g (NULL: g = 1)
 *   grad_x        OUT optional float32 [n][d]
 *   grad_codebook OUT optional float32 [m][ks][ds]
 *   loss          OUT optional float64 [1]: L, summed in float64
 * Codes >= ks make the loss and the affected grad_x entries NaN.
 * ------------------------------------------------------------------------- */
size_t mipq_recon_backward_workspace_size(int64_t n, int d, int m, int ks);
int mipq_recon_backward(const float* x, const uint8_t* codes, const float* codebook, int64_t n, int d,
                        int m, int ks, const double* grad_out, float* grad_x, float* grad_codebook,
                        double* loss, void* ws, size_t ws_bytes, void* stream);

/* -------------------------------------------------------------------------
 * Optimized PQ (paper Section 3.1.1: the PQ library implements PQ and
 * optimized PQ).  Rows are quantised after an orthogonal rotation y = x R;
 * R is fitted by alternating Lloyd rounds on the rotated rows with the
 * orthogonal Procrustes step below (the composition is in the Python layer).
 *
 * mipq_rotate: y [n][d] = x [n][d] R, R float64 [d][d] row-major (y_j =
 *   sum over t of x_t R[t][j]).  Each output is the float64 sum over t
 *   ascending of the float64 products x_t * R[t][j] (product and sum rounded
 *   separately), rounded once to float32.  y must not overlap x.  n == 0 is
 *   valid.  d in [1, 4096].
 *
 * mipq_opq_procrustes: the orthogonal R minimising ||X R - Y_hat||_F for
 *   x, y_hat float32 [n][d]: R = U V^T for U S V^T = M = X^T Y_hat.
 *   M is summed in float64 (float32 products are exact; the order of the
 *   sums is fixed by n and d, so results repeat bit for bit).  The singular
 *   value decomposition is one-sided Jacobi in float64 on one work-group;
 *   columns of U whose singular value is at most d * 2^-52 * the largest are
 *   completed to an orthonormal basis (R is then one of the minimisers).
 *   v_init: optional float64 [d][d] row-major orthogonal start V0 (the
 *   v_out of a previous call on a similar M): the sweeps then run on M V0,
 *   which converges in fewer sweeps; R is the same minimiser up to rounding.
 *   rotation: OUT float64 [d][d] row-major; v_out: OUT optional float64
 *   [d][d] row-major (V); cross: OUT optional float64 [d][d] (M); sweeps:
 *   OUT optional device int (Jacobi sweeps run, 65 if 64 sweeps did not
 *   converge).  d in [1, 256]; n >= 0 (n == 0 gives M = 0 and R = I when
 *   v_init is not given).
 * ------------------------------------------------------------------------- */
int mipq_rotate(const float* x, int64_t n, int d, const double* rotation, float* y, void* stream);
size_t mipq_opq_procrustes_workspace_size(int64_t n, int d);
int mipq_opq_procrustes(const float* x, const float* y_hat, int64_t n, int d, const double* v_init,
                        double* rotation, double* v_out, double* cross, int* sweeps, void* ws, size_t ws_bytes,
                        void* stream);

/* -------------------------------------------------------------------------
 * Per-kernel timing (tracing aid, off by default).
 *
 * mipq_profile_enable(1) makes every subsequent launch of the kernels below
 * record a pair of HIP events on its own stream; mipq_profile_collect()
 * waits for the recorded events of one kernel, returns the number of
 * launches and their summed duration in milliseconds, and forgets them.
 * ------------------------------------------------------------------------- */
enum mipq_kernel {
  MIPQ_K_ASSIGN_FP32 = 0,   /* plain float32 assignment */
  MIPQ_K_ASSIGN_BF16 = 1,   /* matrix-core assignment (with exact re-decision) */
  MIPQ_K_UPDATE = 2,        /* float64 centroid sums per row chunk */
  MIPQ_K_FINALIZE = 3,      /* centroid means, objective (+ operand packing) */
  MIPQ_K_PACK_BF16 = 4,     /* stand-alone centroid operand packing */
  MIPQ_K_DECODE = 5,        /* decode + squared error */
  MIPQ_K_BACKWARD = 6,      /* reconstruction-loss gradient pass */
  MIPQ_K_COARSE_PACK = 7,   /* coarse centre + operand packing */
  MIPQ_K_COARSE_ASSIGN = 8, /* coarse assignment */
  MIPQ_K_SORT = 9,          /* stable bucketing by label */
  MIPQ_K_COARSE_UPDATE = 10,/* coarse centroid update */
  MIPQ_K_ADC = 11,          /* ADC search */
  MIPQ_K_ASSIGN_BF16_BATCHED = 12, /* persistent matrix-core assignment, many problems */
  MIPQ_K_ASSIGN_FP8 = 13,   /* FP8 matrix-core assignment (with exact re-decision) */
  MIPQ_K_PACK_FP8 = 14,     /* FP8 centroid operand packing */
  MIPQ_K_ROTATE = 15,       /* optimized PQ: rotation y = x R */
  MIPQ_K_CROSS = 16,        /* optimized PQ: cross matrix X^T Y_hat */
  MIPQ_K_POLAR = 17,        /* optimized PQ: orthogonal factor by Jacobi */
  MIPQ_K_ADC_SCAN = 18,     /* ADC search: the list scans alone (also inside MIPQ_K_ADC) */
  MIPQ_K_FIT_ROUND_BF16 = 19, /* fit round: matrix-core assignment fused with the float64 sums */
  MIPQ_KERNEL_COUNT = 20
};
int mipq_profile_enable(int on);
int mipq_profile_collect(int kernel, int64_t* launches, double* total_ms);

/* -------------------------------------------------------------------------
 * Peak probes (measurement aid for the roofline fractions, not part of the
 * method).
 *
 * mipq_peak_probe enqueues one launch of `blocks` work-groups of 256 threads
 * that does nothing but one kind of work, so that its sustained rate can be
 * timed by the caller (events on `stream`):
 *   MIPQ_PROBE_ADD_F32 / FMA_F32 / MIN3_F32 / FMA_F64: 8 independent chains
 *     of 2048 instructions per lane (v_add_f32 with a scalar operand,
 *     v_fma_f32, v_min3_f32, v_fma_f64); work = lane instructions of the
 *     launch;
 *   MIPQ_PROBE_ADD_VV / MIN_VV / MIN3_ADD: the same with vector-register
 *     operands only (v_add_f32, v_min_f32; 3-input minima and adds in
 *     alternate chains): which kinds issue two per quad-cycle;
 *   MIPQ_PROBE_MFMA_BF16 / MFMA_F8: four independent accumulators of 512
 *     32x32x16 BF16 (32x32x64 E4M3) MFMAs per wave; work = flops;
 *   MIPQ_PROBE_COPY: copies the first half of `out` onto its second half in
 *     16-byte words; work = bytes read + written.
 *   out        device buffer: >= blocks*256*8 bytes (its contents become
 *              meaningless), or for MIPQ_PROBE_COPY the buffer to copy
 *              within (16-byte aligned)
 *   work       OUT optional host double: the work of one launch (above)
 * ------------------------------------------------------------------------- */
enum mipq_probe {
  MIPQ_PROBE_ADD_F32 = 0,
  MIPQ_PROBE_FMA_F32 = 1,
  MIPQ_PROBE_MIN3_F32 = 2,
  MIPQ_PROBE_FMA_F64 = 3,
  MIPQ_PROBE_MFMA_BF16 = 4,
  MIPQ_PROBE_MFMA_F8 = 5,
  MIPQ_PROBE_COPY = 6,
  MIPQ_PROBE_ADD_VV = 7,
  MIPQ_PROBE_MIN_VV = 8,
  MIPQ_PROBE_MIN3_ADD = 9
};
int mipq_peak_probe(int kind, int blocks, void* out, size_t out_bytes, double* work, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MIPQ_H */
