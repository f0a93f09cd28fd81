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
 * Both give the same codes: the code of a (row, subspace) is the lowest index
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

#define MIPQ_ABI_VERSION 1

enum mipq_status {
  MIPQ_OK = 0,
  MIPQ_EINVAL = -1,       /* bad shape, null required pointer, bad enum */
  MIPQ_ENOMEM = -2,       /* workspace smaller than the *_workspace_size() query */
  MIPQ_EHIP = -3,         /* a HIP runtime call failed (text in mipq_last_error) */
  MIPQ_EUNSUPPORTED = -4  /* valid request this build does not implement */
};

enum mipq_precision { MIPQ_FP32 = 0, MIPQ_BF16 = 1 };

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
 * Requirements: d % m == 0, d/m <= 16 (BF16) or <= 32 (FP32), 1 <= ks <= 256,
 * n_train >= 1, iters >= 0, init rows in range.
 * ------------------------------------------------------------------------- */
size_t mipq_pq_fit_workspace_size(int64_t n_train, int d, int m, int ks, int iters, int precision);
int mipq_pq_fit(const float* x, int64_t n, const int64_t* train_rows, int64_t n_train,
                int d, int m, int ks, int iters,
                const int64_t* init_rows, const float* init_codebook, int precision,
                float* codebook, double* codebook64, uint8_t* labels, double* objective,
                void* ws, size_t ws_bytes, void* stream);

/* -------------------------------------------------------------------------
 * Encode (paper Section 2.1: each row of each subspace is represented by
 * its nearest subspace centroid, so a row becomes m codes).
 *
 *   codes     OUT uint8 [n][m]
 *   rescored  OUT optional int64 [1]: number of (row, subspace) pairs the
 *             BF16 path re-decided in FP32 arithmetic (0 for MIPQ_FP32)
 * ------------------------------------------------------------------------- */
size_t mipq_pq_encode_workspace_size(int64_t n, int d, int m, int ks, int precision);
int mipq_pq_encode(const float* x, int64_t n, int d, int m, int ks, const float* codebook,
                   int precision, uint8_t* codes, int64_t* rescored,
                   void* ws, size_t ws_bytes, void* stream);

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
  MIPQ_KERNEL_COUNT = 7
};
int mipq_profile_enable(int on);
int mipq_profile_collect(int kernel, int64_t* launches, double* total_ms);

#ifdef __cplusplus
}
#endif

#endif /* MIPQ_H */
