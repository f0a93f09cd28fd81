// Internal declarations shared by the HIP sources of libmipq.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "mipq.h"

namespace mipq {

// ---- error reporting -------------------------------------------------------
int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);

#define MIPQ_HIP(call)                                   \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return ::mipq::hip_fail(e_, #call); \
  } while (0)

#define MIPQ_LAUNCHED(what)                              \
  do {                                                   \
    hipError_t e_ = hipGetLastError();                   \
    if (e_ != hipSuccess) return ::mipq::hip_fail(e_, what); \
  } while (0)

// ---- per-kernel event timing (see mipq_profile_enable) -----------------------
class ProfScope {
 public:
  ProfScope(int kernel, hipStream_t s);
  ~ProfScope();
  ProfScope(const ProfScope&) = delete;
  ProfScope& operator=(const ProfScope&) = delete;

 private:
  int kernel_;
  hipStream_t s_;
  hipEvent_t a_ = nullptr, b_ = nullptr;
};

// ---- workspace carving -----------------------------------------------------
// Sub-buffers are 256-byte aligned; the same carving code sizes and fills.
struct Carver {
  char* base;
  size_t used = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  template <class T>
  T* take(size_t count) {
    used = (used + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + used) : nullptr;
    used += count * sizeof(T);
    return p;
  }
  size_t bytes() const { return (used + 255) & ~size_t(255); }
};

// ---- constants ---------------------------------------------------------------
constexpr int kMaxKs = 256;        // codes are uint8
constexpr int kMaxDsBf16 = 16;     // two 8-dimension blocks per subspace
constexpr int kMaxDsFp32 = 64;
constexpr int kMaxDsFit = 48;      // float64 centroid sums held in LDS
// LDS of one update block at ks = 256, d/m = 48: sums 256 x 49 float64, counts,
// the float32 codebook of the subspace; within the 160 KiB of a CU
static_assert(256 * (kMaxDsFit + 1) * 8 + 128 * 8 + 256 * kMaxDsFit * 4 + 16 * 8 <= 160 * 1024,
              "update block LDS");

// One problem of a batched fit (device copy, built by the host from the
// caller's problem table).  Work-list offsets: unit0 = first (32-row tile x
// subspace group) assignment unit, item0 = first (chunk x subspace)
// accumulation item, dblk0 = first decode block of this problem.
struct BatchProb {
  const float* x;
  int64_t n;
  const int64_t* init_rows;
  float* c32;
  uint8_t* codes;
  double* sse_rmse;
  double* objective;
  int64_t unit0;
  int64_t item0;
  int64_t rpc;      // rows per accumulation chunk
  int64_t dblk0;
  int nch;          // accumulation chunks
  int nblk;         // decode blocks
};
constexpr int kBatchPend = 512;   // pending exact re-decisions per wave (LDS)

// number of 32x32x16 MFMAs per 32-centroid tile for NB 8-dim blocks
__host__ __device__ constexpr int bf16_nmfma(int nb) { return nb + (nb + 1) / 2 + ((nb % 2 == 0) ? 1 : 0); }
inline int ceil_div(int64_t a, int64_t b) { return int((a + b - 1) / b); }
inline int tiles_for(int ks) { return ks <= 32 ? 1 : ks <= 64 ? 2 : ks <= 128 ? 4 : 8; }
constexpr int kMaxTiles = 8;   // tiles_for(kMaxKs)

// ---- launchers (each returns MIPQ_OK or an error code) ---------------------
int launch_zero_u32(uint32_t* p, size_t count, hipStream_t s);
int launch_gather_rows(const float* x, int64_t n, int d, const int64_t* rows, int64_t n_rows,
                       float* out, uint32_t* bad, hipStream_t s);
int launch_init_codebook(const float* train, int64_t n_train, int d, int m, int ks,
                         const int64_t* init_rows, const float* init_cb, double* c64, float* c32,
                         uint32_t* bad, uint32_t* done, hipStream_t s);
int launch_assign_fp32(const float* x, int64_t n, int d, int m, int ks, const float* c32,
                       uint8_t* codes, hipStream_t s);
// Lloyd update of one round; aop == NULL: plain path (no operand packing)
int update_chunks(int64_t n, int m);
// chunks of a problem in the fused batched round: at most kFusedChunkRows rows
// each, so that a chunk's pending list fits its block's LDS
constexpr int64_t kFusedChunkRows = 32768;
inline int fused_chunks(int64_t n) { return n < 1 ? 1 : (int)((n + kFusedChunkRows - 1) / kFusedChunkRows); }
// objective: also the float64 objective terms of the round (else part_j holds zeros)
// det: float64 sums in a fixed order (no atomic additions; MIPQ_DETERMINISTIC)
int launch_update(const float* x, int64_t n, int d, int m, int ks, const uint8_t* codes, float* c32,
                  double* c64, int nch, double* part_s, uint32_t* part_cnt, double* part_j,
                  double* j_sub, void* aop, float* cmax, float* mu, bool objective, bool det, hipStream_t s);
// the finalize of launch_update alone (centroid means, objective when j_sub,
// next operands when aop) over nch chunk partials
int launch_finalize(int m, int ks, int ds, int nch, const double* part_s, const uint32_t* part_cnt,
                    const double* part_j, float* c32, double* c64, double* j_sub, void* aop, float* cmax,
                    const float* mu, hipStream_t s);
int launch_objective(const double* j_sub, int iters, int m, double* objective, hipStream_t s);
int launch_copy_f64(const double* src, double* dst, size_t count, hipStream_t s);
int launch_decode_sse(const uint8_t* codes, int64_t n, int d, int m, int ks, const float* c32,
                      const float* x, float* x_hat, double* partials, int nblk, hipStream_t s);
int decode_blocks(int64_t n, int m);
int launch_decode_centroids(const float* cb, int64_t nbooks, int m, int ks, int ds, float* out, hipStream_t s);
int launch_sse_final(const double* partials, int nblk, int64_t n, int d, double* out, hipStream_t s);
// float32-rule distance of each (row, subspace) to its coded centroid
// (min_dist optional) and per-block float64 squared-error partials
int launch_code_dist(const float* x, int64_t n, int d, int m, int ks, const float* c32, const uint8_t* codes,
                     float* min_dist, double* partials, int nblk, hipStream_t s);
// flag[0] |= 1 if any of the count floats is NaN or infinite
int launch_nonfinite(const float* p, size_t count, uint32_t* flag, hipStream_t s);

// BF16 matrix-core path
struct Bf16Geom {
  int groups = 1;    // blocks of 4 subspaces
  int rpb = 32;      // rows per block (multiple of 32)
  int rowblks = 0;   // row blocks covering n
  int blocks = 0;    // launched blocks (XCD-padded)
};
Bf16Geom bf16_geometry(int64_t n, int m, int max_tiles);   // max_tiles: 32-row tiles per block at most
size_t bf16_operand_count(int m, int ks, int ds);   // number of 16-byte operand slots
// reconstruction-loss backward with fixed codes: grad_x (optional), grad_c
// (optional), per-subspace loss; g = *gscale (NULL: 1)
int backward_chunks(int64_t n, int m);
int launch_backward(const float* x, int64_t n, int d, int m, int ks, const uint8_t* codes,
                    const float* c32, const double* gscale, float* grad_x, float* grad_c, int nch,
                    double* part_s, uint32_t* part_cnt, double* part_j, double* loss_sub, hipStream_t s);
// inverted file (ivf.hip)
int coarse_ksteps(int d);
size_t coarse_operand_count(int kc, int d);
int launch_coarse_prepare(const float* cc, int kc, int d, float* mu, unsigned int* cmax_bits, void* aop,
                          hipStream_t s);
int launch_coarse_assign(const float* x, int64_t n, int d, const float* cc, int kc, const void* aop,
                         const float* mu, const unsigned int* cmax_bits, int32_t* labels, int64_t* rescored,
                         bool exact_only, hipStream_t s);
int sort_blocks(int64_t n);
// uint32 entries of the sort's histogram workspace (block counts and digit totals)
size_t sort_hist_entries(int64_t n);
int launch_sort_by_label(const int32_t* labels, int64_t n, int kc, uint32_t* keys_a, uint32_t* keys_b,
                         int32_t* vals_a, int32_t* vals_b, uint32_t* hist, int32_t* ids_out,
                         uint32_t* keys_out_sorted, int64_t* offsets, hipStream_t s);
int launch_coarse_update(const float* x, int d, const int32_t* ids, const int64_t* offsets, int kc, float* cc,
                         double* cc64, double* obj_list, double* obj_out, hipStream_t s);
int launch_gather_coarse(const float* x, int64_t n, int d, const int64_t* rows, int kc, float* cc, double* cc64,
                         hipStream_t s);
int launch_residuals(const float* x, int64_t n, int d, const int32_t* labels, const float* cc, int kc, float* r,
                     hipStream_t s);
int launch_gather_codes(const uint8_t* codes, int64_t n, int m, const int32_t* ids, uint8_t* out, hipStream_t s);
// optimized PQ: rotation y = x R, cross matrix X^T Y_hat (chunk partials in
// part, nch from cross_chunks), orthogonal polar factor of M (one work-group)
int launch_rotate(const float* x, int64_t n, int d, const double* r, float* y, hipStream_t s);
int cross_chunks(int64_t n, int d);
int launch_cross(const float* x, const float* yh, int64_t n, int d, int nch, double* part, double* m,
                 hipStream_t s);
size_t polar_log_bytes(int d, int max_sweeps);   // rotation log of launch_polar (0: none needed)
int launch_polar(const double* m, int d, int max_sweeps, const double* v0, double* m0, double* a, double* v,
                 double* rj, double* vj, void* rlog, double* r, double* v_out, int* sweeps, hipStream_t s);
// merge of inverted lists of consecutive row ranges; parts: device array of
// {const int64_t* off; const int32_t* ids; const uint8_t* codes; int64_t n; int64_t base}
size_t merge_part_bytes();
int launch_merge_lists(const void* parts, int nparts, int64_t total_rows, int kc, int m, int64_t* pre,
                       int64_t* total, int64_t* offsets, int32_t* ids, uint8_t* codes, bool vec16, hipStream_t s);

// ADC search (adc.hip)
// LDS of one scan block (the table m x ks floats, the query, the key buffer)
constexpr size_t kAdcMaxLds = 64 * 1024;
bool adc_fits_lds(int d, int m, int ks, int topk);
// order_ws: adc_order_bytes(nq * nprobe, nprobe, kc) bytes (the scan blocks' order)
size_t adc_order_bytes(int64_t pairs, int nprobe, int kc);
int launch_adc(const float* q, int nq, int d, const float* cc, int kc, const void* aop, const float* mu,
               const unsigned int* cmax_bits, const float* pq, int m, int ks, const int64_t* offsets,
               const int32_t* ids, const uint8_t* codes, int nprobe, int topk, float* est, int32_t* probes,
               unsigned long long* qthr, uint64_t* pair_out, void* order_ws, int64_t* wide, int32_t* out_ids,
               float* out_dist, int64_t* work, hipStream_t s);

// operands of the centred codebook; mu: m * kMaxDsBf16 floats (subspace centres)
int launch_pack_bf16(const float* c32, int m, int ks, int ds, void* aop, float* cmax, float* mu,
                     hipStream_t s);
// batched problems (device table probs[nprob], see BatchProb)
int launch_init_batched(const BatchProb* probs, int nprob, int d, int m, int ks, double* c64_all, uint32_t* bad,
                        hipStream_t s);
int launch_pack_bf16_batched(const BatchProb* probs, int nprob, int m, int ks, int ds, void* aop,
                             size_t aop_stride, float* cmax, float* mu, hipStream_t s);
// the batched assignment in two variants: 0 re-decides pending rows one at a
// time, 1 with the centroids held in registers (more registers per wave)
constexpr int kBatchedVariants = 2;
int assign_bf16_batched_resident(int ds, int ks, bool full, int variant, int* resident);
int launch_assign_bf16_batched(const BatchProb* probs, int nprob, int64_t units, int d, int m, int ks,
                               const void* aop, size_t aop_stride, const float* cmax, const float* mu, bool full,
                               int variant, int grid, int64_t* rescored, hipStream_t s);
// one Lloyd update of every problem (accumulate: form the partials, which a
// fused round has already formed otherwise), then the next round's norm
// bounds cmax from the tiles' bounds tmax (nprob m kMaxTiles floats) and
// *round advanced
int launch_update_batched(const BatchProb* probs, int nprob, int64_t items, int d, int m, int ks, double* c64,
                          double* part_s, uint32_t* part_cnt, double* part_j, double* j_all,
                          const uint32_t* round, int iters, void* aop, size_t aop_stride, float* cmax, float* mu,
                          bool det, bool accumulate, float* tmax, hipStream_t s);
// rows per wave of the fused batched round's pending lists for chunks of at
// most max_rpc rows, 0 when they do not fit a block's LDS (or 16-bit offsets)
// or d/m is out of the matrix-core path's range
int fit_round_batched_rpw(int ks, int ds, int64_t max_rpc);
// one Lloyd round's assignment and partial sums of every problem (the items
// and partial layout of launch_update_batched, chunks of fused_chunks rows),
// for plans without objectives
int launch_fit_round_bf16_batched(const BatchProb* probs, int nprob, int64_t items, int d, int m, int ks,
                                  const void* aop, size_t aop_stride, const float* cmax, const float* mu, bool full,
                                  int rpw, double* part_s, uint32_t* part_cnt, double* part_j, hipStream_t s);
int launch_decode_sse_batched(const BatchProb* probs, int nprob, int64_t blocks, int d, int m, int ks, bool vec,
                              double* partials, hipStream_t s);
int launch_objective_batched(const BatchProb* probs, int nprob, int iters, int m, const double* j_all,
                             hipStream_t s);

// FP8 matrix-core path: operands (32-byte slots) and per-subspace statistics
size_t fp8_operand_count(int m, int ks);
size_t fp8_stats_count(int m);
int launch_pack_fp8(const float* c32, int m, int ks, int ds, void* aop, float* stats, hipStream_t s);
int launch_assign_fp8(const float* x, int64_t n, int d, int m, int ks, const void* aop, const float* stats,
                      const float* c32, uint8_t* codes, int64_t* rescored, hipStream_t s);

// rescored: optional int64 counter, incremented by the pairs re-decided exactly
// min_dist / sse_part (either optional; both NULL: codes only): the chosen
// centroid's float32-rule distance and per-wave float64 squared-error partials
// (assign_bf16_sse_parts(n, m) of them, reduced by launch_sse_final)
int launch_assign_bf16(const float* x, int64_t n, int d, int m, int ks, const void* aop,
                       const float* cmax, const float* mu, const float* c32, uint8_t* codes,
                       int64_t* rescored, float* min_dist, double* sse_part, hipStream_t s);
int assign_bf16_sse_parts(int64_t n, int m);

// Fused Lloyd round (BF16 assignment + float64 sums by code, one launch):
// nch row chunks of (12 or 4 waves) * rpw rows (rpw = 0: the shape does not
// fit the LDS).
// Writes the chunks' partials in launch_update's layout (finalize with
// launch_finalize); cmax is read, cmax_zero (another m floats) zeroed for the
// finalize to raise.
struct FitGeom {
  int nch = 0, rpw = 0;
};
FitGeom fit_round_geometry(int64_t n, int m, int ks, int ds);
int launch_fit_round_bf16(const float* x, int64_t n, int d, int m, int ks, const void* aop, const float* cmax,
                          const float* mu, const float* c32, uint8_t* codes, int64_t* rescored, double* part_s,
                          uint32_t* part_cnt, float* cmax_zero, hipStream_t s);

}  // namespace mipq
