// C-ABI entry points of libmipq: argument checks, workspace carving and the
// launch sequence of each call.  See include/mipq.h for the contract.
#include <stdarg.h>
#include <stdio.h>

#include <initializer_list>
#include <vector>

#include "mipq_internal.h"

namespace mipq {

namespace {
thread_local char g_err[512] = "";
}

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(MIPQ_EHIP, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

namespace {

int check_shape(int64_t n, int d, int m, int ks, int precision, bool fit) {
  if (n < 0) return fail(MIPQ_EINVAL, "n must be >= 0 (got %lld)", (long long)n);
  if (d <= 0 || m <= 0) return fail(MIPQ_EINVAL, "d and m must be positive (d=%d, m=%d)", d, m);
  if (d % m != 0) return fail(MIPQ_EINVAL, "d=%d is not divisible by m=%d", d, m);
  if (ks < 1 || ks > kMaxKs) return fail(MIPQ_EINVAL, "ks must be in [1, %d] (got %d)", kMaxKs, ks);
  const int ds = d / m;
  if (precision == MIPQ_FP32) {
    if (ds > (fit ? kMaxDsFit : kMaxDsFp32))
      return fail(MIPQ_EUNSUPPORTED, "FP32 path supports d/m <= %d here (got %d)",
                  fit ? kMaxDsFit : kMaxDsFp32, ds);
  } else if (precision == MIPQ_BF16 || precision == MIPQ_FP8) {
    if (ds > kMaxDsBf16)
      return fail(MIPQ_EUNSUPPORTED, "matrix-core paths support d/m <= %d (got %d)", kMaxDsBf16, ds);
    if ((uint64_t)n * (uint64_t)m >= (1ull << 32))
      return fail(MIPQ_EUNSUPPORTED, "matrix-core paths need n*m < 2^32");
  } else {
    return fail(MIPQ_EINVAL, "unknown precision %d", precision);
  }
  return MIPQ_OK;
}

struct EncodeWs {
  void* aop = nullptr;
  float* cmax = nullptr;
  float* mu = nullptr;
  size_t bytes = 0;
};

// flag word of the finite check and the squared-error partials of an encode
struct EncodeExtraWs {
  uint32_t* flag = nullptr;
  double* partials = nullptr;
  int nblk = 0;
  size_t bytes = 0;
};

// partials: decode_blocks of the separate distance pass, or the per-wave
// partials of the BF16 assignment, which forms them itself
EncodeExtraWs carve_encode_extra(void* ws, int64_t n, int m, int precision) {
  Carver c(ws);
  EncodeExtraWs e;
  e.flag = c.take<uint32_t>(4);
  e.nblk = precision == MIPQ_BF16 ? assign_bf16_sse_parts(n, m) : decode_blocks(n, m);
  e.partials = c.take<double>(e.nblk);
  e.bytes = c.bytes();
  return e;
}

EncodeWs carve_encode(void* ws, int m, int ks, int ds, int precision) {
  Carver c(ws);
  EncodeWs e;
  if (precision == MIPQ_BF16) {
    e.aop = c.take<uint4>(bf16_operand_count(m, ks, ds));
    e.cmax = c.take<float>(m);
    e.mu = c.take<float>((size_t)m * kMaxDsBf16);
  } else if (precision == MIPQ_FP8) {
    e.aop = c.take<uint4>(2 * fp8_operand_count(m, ks));   // 32-byte slots
    e.mu = c.take<float>(fp8_stats_count(m));               // per-subspace statistics
  }
  e.bytes = c.bytes();
  return e;
}

struct FitWs {
  float* xs = nullptr;
  uint8_t* codes = nullptr;
  double* c64 = nullptr;
  double* part_s = nullptr;
  uint32_t* part_cnt = nullptr;
  double* part_j = nullptr;
  double* j_sub = nullptr;
  uint32_t* bad = nullptr;
  uint32_t* flag = nullptr;
  float* cmax2 = nullptr;   // the second norm-bound buffer of the fused rounds
  int nch = 1;   // chunk partials the workspace holds (two-pass or fused rounds)
  EncodeWs enc;
  size_t bytes = 0;
};

// BF16 fits without the objective and without MIPQ_DETERMINISTIC run each
// Lloyd round as one fused launch (assignment + sums) and the finalize
bool fused_rounds(int64_t n_train, int m, int ks, int ds, int precision, bool objective, bool det) {
  return precision == MIPQ_BF16 && !objective && !det && fit_round_geometry(n_train, m, ks, ds).rpw > 0;
}

FitWs carve_fit(void* ws, int64_t n_train, bool gather, int d, int m, int ks, int iters,
                int precision, bool need_codes, bool need_c64) {
  Carver c(ws);
  FitWs f;
  const int ds = d / m;
  f.nch = update_chunks(n_train, m);
  if (precision == MIPQ_BF16) {   // room for the fused rounds' partials too
    const int fch = fit_round_geometry(n_train, m, ks, ds).nch;
    if (fch > f.nch) f.nch = fch;
  }
  if (gather) f.xs = c.take<float>((size_t)n_train * d);
  if (need_codes) f.codes = c.take<uint8_t>((size_t)n_train * m);
  if (need_c64) f.c64 = c.take<double>((size_t)m * ks * ds);
  f.part_s = c.take<double>((size_t)f.nch * m * ks * ds);
  f.part_cnt = c.take<uint32_t>((size_t)f.nch * m * ks);
  f.part_j = c.take<double>((size_t)f.nch * m);
  f.j_sub = c.take<double>((size_t)(iters > 0 ? iters : 1) * m);
  f.bad = c.take<uint32_t>(4);
  f.flag = c.take<uint32_t>(4);
  if (precision == MIPQ_BF16) f.cmax2 = c.take<float>((size_t)m);
  const size_t off = c.bytes();
  EncodeWs e = carve_encode(ws ? static_cast<char*>(ws) + off : nullptr, m, ks, ds, precision);
  f.enc = e;
  f.bytes = off + e.bytes;
  return f;
}

// MIPQ_CHECK_FINITE: flag |= 1 for any non-finite value of the arrays, then
// wait for the stream and report
struct FloatSpan {
  const float* p;
  size_t count;
};
int check_finite(std::initializer_list<FloatSpan> arrays, uint32_t* flag, hipStream_t s) {
  int rc;
  if ((rc = launch_zero_u32(flag, 1, s))) return rc;
  for (const FloatSpan& a : arrays)
    if (a.p && (rc = launch_nonfinite(a.p, a.count, flag, s))) return rc;
  uint32_t h = 0;
  MIPQ_HIP(hipMemcpyAsync(&h, flag, sizeof(h), hipMemcpyDeviceToHost, s));
  MIPQ_HIP(hipStreamSynchronize(s));
  if (h) return fail(MIPQ_ENONFINITE, "an input value is NaN or infinite");
  return MIPQ_OK;
}

int check_flags(int flags, int allowed) {
  if (flags & ~allowed) return fail(MIPQ_EINVAL, "unknown flags 0x%x", flags & ~allowed);
  return MIPQ_OK;
}

int check_ws(void* ws, size_t have, size_t need) {
  if (need == 0) return MIPQ_OK;
  if (!ws) return fail(MIPQ_EINVAL, "workspace pointer is NULL (%zu bytes needed)", need);
  if (have < need) return fail(MIPQ_ENOMEM, "workspace too small: %zu < %zu bytes", have, need);
  if (reinterpret_cast<uintptr_t>(ws) & 255u) return fail(MIPQ_EINVAL, "workspace must be 256-byte aligned");
  return MIPQ_OK;
}

// codes of `x` against `c32` by the exact rule (operands already packed for BF16)
int assign_any(const float* x, int64_t n, int d, int m, int ks, const float* c32, int precision,
               uint8_t* codes, const EncodeWs& e, int64_t* rescored, hipStream_t s) {
  if (precision == MIPQ_FP32) return launch_assign_fp32(x, n, d, m, ks, c32, codes, s);
  if (precision == MIPQ_FP8) return launch_assign_fp8(x, n, d, m, ks, e.aop, e.mu, c32, codes, rescored, s);
  return launch_assign_bf16(x, n, d, m, ks, e.aop, e.cmax, e.mu, c32, codes, rescored, nullptr, nullptr, s);
}

// operands of the matrix-core paths for the codebook c32
int pack_any(const float* c32, int m, int ks, int ds, int precision, const EncodeWs& e, hipStream_t s) {
  if (precision == MIPQ_BF16) return launch_pack_bf16(c32, m, ks, ds, e.aop, e.cmax, e.mu, s);
  if (precision == MIPQ_FP8) return launch_pack_fp8(c32, m, ks, ds, e.aop, e.mu, s);
  return MIPQ_OK;
}

}  // namespace
}  // namespace mipq

using namespace mipq;

extern "C" {

int mipq_abi_version(void) { return MIPQ_ABI_VERSION; }

const char* mipq_last_error(void) { return g_err; }

size_t mipq_pq_fit_workspace_size(int64_t n_train, int d, int m, int ks, int iters, int precision) {
  if (check_shape(n_train, d, m, ks, precision, true) != MIPQ_OK || iters < 0) return 0;
  // worst case: gathered sample, internal codes and float64 codebook
  return carve_fit(nullptr, n_train, true, d, m, ks, iters, precision, true, true).bytes;
}

int mipq_pq_fit(const float* x, int64_t n, const int64_t* train_rows, int64_t n_train, int d, int m,
                int ks, int iters, const int64_t* init_rows, const float* init_codebook,
                int precision, int flags, float* codebook, double* codebook64, uint8_t* labels,
                double* objective, int64_t* rescored, void* ws, size_t ws_bytes, void* stream) {
  int rc;
  const int64_t nt = train_rows ? n_train : n;
  if ((rc = check_shape(nt, d, m, ks, precision, true))) return rc;
  if ((rc = check_flags(flags, MIPQ_CHECK_FINITE | MIPQ_DETERMINISTIC))) return rc;
  if (train_rows && (n < 1 || n_train < 1)) return fail(MIPQ_EINVAL, "empty row set");
  if (nt < 1) return fail(MIPQ_EINVAL, "fit needs at least one training row");
  if (iters < 0 || iters > (1 << 16)) return fail(MIPQ_EINVAL, "iters out of range (%d)", iters);
  if (!x || !codebook) return fail(MIPQ_EINVAL, "x and codebook are required");
  if (!init_rows && !init_codebook) return fail(MIPQ_EINVAL, "init_rows or init_codebook is required");
  hipStream_t s = static_cast<hipStream_t>(stream);
  FitWs f = carve_fit(ws, nt, train_rows != nullptr, d, m, ks, iters, precision, labels == nullptr,
                      codebook64 == nullptr);
  if ((rc = check_ws(ws, ws_bytes, f.bytes))) return rc;
  const int ds = d / m;
  const float* train = x;
  if (train_rows) {
    if ((rc = launch_gather_rows(x, n, d, train_rows, n_train, f.xs, f.bad, s))) return rc;
    train = f.xs;
  }
  if ((flags & MIPQ_CHECK_FINITE) &&
      (rc = check_finite({{train, (size_t)nt * d}, {init_codebook, init_codebook ? (size_t)m * ks * ds : 0}},
                         f.flag, s)))
    return rc;
  uint8_t* codes = labels ? labels : f.codes;
  double* c64 = codebook64 ? codebook64 : f.c64;
  float* c32 = codebook;   // working float32 codebook, final value on return
  if (rescored && (rc = launch_zero_u32(reinterpret_cast<uint32_t*>(rescored), 2 * (size_t)iters, s))) return rc;
  if ((rc = launch_init_codebook(train, nt, d, m, ks, init_codebook ? nullptr : init_rows, init_codebook,
                                 c64, c32, f.bad, nullptr, s)))
    return rc;
  const bool bf = precision == MIPQ_BF16;
  const bool det = (flags & MIPQ_DETERMINISTIC) != 0;
  if (iters > 0 && (rc = pack_any(c32, m, ks, ds, precision, f.enc, s))) return rc;
  if (fused_rounds(nt, m, ks, ds, precision, objective != nullptr, det)) {
    const int nch = fit_round_geometry(nt, m, ks, ds).nch;
    for (int it = 0; it < iters; ++it) {
      // the round reads one norm-bound buffer and clears the other, which its
      // finalize raises for the next round
      float* cm_read = (it & 1) ? f.cmax2 : f.enc.cmax;
      float* cm_next = (it & 1) ? f.enc.cmax : f.cmax2;
      // the sums need no stored codes: only the last round stores them, and
      // only for a caller that takes the labels
      uint8_t* round_codes = (labels && it + 1 == iters) ? codes : nullptr;
      if ((rc = launch_fit_round_bf16(train, nt, d, m, ks, f.enc.aop, cm_read, f.enc.mu, c32, round_codes,
                                      rescored ? rescored + it : nullptr, f.part_s, f.part_cnt, cm_next, s)))
        return rc;
      if ((rc = launch_finalize(m, ks, ds, nch, f.part_s, f.part_cnt, nullptr, c32, c64, nullptr, f.enc.aop, cm_next,
                                f.enc.mu, s)))
        return rc;
    }
    return MIPQ_OK;
  }
  for (int it = 0; it < iters; ++it) {
    if ((rc = assign_any(train, nt, d, m, ks, c32, precision, codes, f.enc, rescored ? rescored + it : nullptr,
                         s)))
      return rc;
    // the update also packs the next round's operands (BF16)
    if ((rc = launch_update(train, nt, d, m, ks, codes, c32, c64, update_chunks(nt, m), f.part_s, f.part_cnt, f.part_j,
                            f.j_sub + (size_t)it * m, bf ? f.enc.aop : nullptr, f.enc.cmax, f.enc.mu,
                            objective != nullptr, det, s)))
      return rc;
    if (precision == MIPQ_FP8 && it + 1 < iters && (rc = launch_pack_fp8(c32, m, ks, ds, f.enc.aop, f.enc.mu, s)))
      return rc;
  }
  if (objective && (rc = launch_objective(f.j_sub, iters, m, objective, s))) return rc;
  return MIPQ_OK;
}

size_t mipq_pq_encode_workspace_size(int64_t n, int d, int m, int ks, int precision) {
  if (check_shape(n, d, m, ks, precision, false) != MIPQ_OK) return 0;
  const size_t main = carve_encode(nullptr, m, ks, d / m, precision).bytes;
  return main + carve_encode_extra(nullptr, n, m, precision).bytes;
}

int mipq_pq_encode(const float* x, int64_t n, int d, int m, int ks, const float* codebook,
                   int precision, int flags, uint8_t* codes, float* min_dist, double* sse_rmse,
                   int64_t* rescored, void* ws, size_t ws_bytes, void* stream) {
  int rc;
  if ((rc = check_shape(n, d, m, ks, precision, false))) return rc;
  if ((rc = check_flags(flags, MIPQ_CHECK_FINITE))) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (n > 0 && (!x || !codebook || !codes)) return fail(MIPQ_EINVAL, "x, codebook and codes are required");
  EncodeWs e = carve_encode(ws, m, ks, d / m, precision);
  EncodeExtraWs ex = carve_encode_extra(ws ? static_cast<char*>(ws) + e.bytes : nullptr, n, m, precision);
  if ((n > 0 || (flags & MIPQ_CHECK_FINITE)) && (rc = check_ws(ws, ws_bytes, e.bytes + ex.bytes))) return rc;
  if ((flags & MIPQ_CHECK_FINITE) &&
      (rc = check_finite({{x, (size_t)n * d}, {codebook, (size_t)m * ks * (d / m)}}, ex.flag, s)))
    return rc;
  if (rescored && (rc = launch_zero_u32(reinterpret_cast<uint32_t*>(rescored), 2, s))) return rc;
  if (n > 0) {
    if ((rc = pack_any(codebook, m, ks, d / m, precision, e, s))) return rc;
    if (precision == MIPQ_BF16) {   // distances and squared errors formed by the assignment itself
      if ((rc = launch_assign_bf16(x, n, d, m, ks, e.aop, e.cmax, e.mu, codebook, codes, rescored, min_dist,
                                   sse_rmse ? ex.partials : nullptr, s)))
        return rc;
    } else {
      if ((rc = assign_any(x, n, d, m, ks, codebook, precision, codes, e, rescored, s))) return rc;
      if ((min_dist || sse_rmse) &&
          (rc = launch_code_dist(x, n, d, m, ks, codebook, codes, min_dist, ex.partials, ex.nblk, s)))
        return rc;
    }
  }
  if (sse_rmse && (rc = launch_sse_final(ex.partials, n > 0 ? ex.nblk : 0, n, d, sse_rmse, s))) return rc;
  return MIPQ_OK;
}

size_t mipq_pq_decode_rmse_workspace_size(int64_t n, int d, int m, int ks) {
  if (check_shape(n, d, m, ks, MIPQ_FP32, false) != MIPQ_OK) return 0;
  Carver c(nullptr);
  c.take<double>(decode_blocks(n, m));
  return c.bytes();
}

int mipq_pq_decode_rmse(const uint8_t* codes, int64_t n, int d, int m, int ks, const float* codebook,
                        const float* x, float* x_hat, double* sse_rmse, void* ws, size_t ws_bytes,
                        void* stream) {
  int rc;
  if ((rc = check_shape(n, d, m, ks, MIPQ_FP32, false))) return rc;
  if (!codebook || (n > 0 && !codes)) return fail(MIPQ_EINVAL, "codes and codebook are required");
  if (sse_rmse && !x) return fail(MIPQ_EINVAL, "the reconstruction error needs x");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Carver c(ws);
  const int nblk = decode_blocks(n, m);
  double* partials = c.take<double>(nblk);
  if ((rc = check_ws(ws, ws_bytes, c.bytes()))) return rc;
  if (n > 0 && (rc = launch_decode_sse(codes, n, d, m, ks, codebook, x, x_hat, partials, nblk, s))) return rc;
  if (sse_rmse) {
    if (n == 0 && (rc = launch_copy_f64(nullptr, nullptr, 0, s))) return rc;
    if ((rc = launch_sse_final(partials, n > 0 ? nblk : 0, n, d, sse_rmse, s))) return rc;
  }
  return MIPQ_OK;
}

int mipq_pq_decode_centroids(const float* codebooks, int64_t nbooks, int d, int m, int ks, float* out,
                              void* stream) {
  int rc;
  if (nbooks < 0) return fail(MIPQ_EINVAL, "nbooks must be >= 0");
  if ((rc = check_shape(0, d, m, ks, MIPQ_FP32, false))) return rc;
  if (nbooks > 0 && (!codebooks || !out)) return fail(MIPQ_EINVAL, "codebooks and out are required");
  return launch_decode_centroids(codebooks, nbooks, m, ks, d / m, out, static_cast<hipStream_t>(stream));
}

size_t mipq_recon_backward_workspace_size(int64_t n, int d, int m, int ks) {
  if (check_shape(n, d, m, ks, MIPQ_FP32, true) != MIPQ_OK) return 0;
  const int nch = backward_chunks(n, m);
  Carver c(nullptr);
  c.take<double>((size_t)nch * d * ks);
  c.take<uint32_t>((size_t)nch * m * ks);
  c.take<double>((size_t)nch * m);
  c.take<double>(m);
  return c.bytes();
}

int mipq_recon_backward(const float* x, const uint8_t* codes, const float* codebook, int64_t n, int d,
                        int m, int ks, const double* grad_out, float* grad_x, float* grad_codebook,
                        double* loss, void* ws, size_t ws_bytes, void* stream) {
  int rc;
  if ((rc = check_shape(n, d, m, ks, MIPQ_FP32, true))) return rc;
  if (!codebook || (n > 0 && (!x || !codes))) return fail(MIPQ_EINVAL, "x, codes and codebook are required");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nch = backward_chunks(n, m);
  Carver c(ws);
  double* part_s = c.take<double>((size_t)nch * d * ks);
  uint32_t* part_cnt = c.take<uint32_t>((size_t)nch * m * ks);
  double* part_j = c.take<double>((size_t)nch * m);
  double* loss_sub = c.take<double>(m);
  if ((rc = check_ws(ws, ws_bytes, c.bytes()))) return rc;
  if ((rc = launch_backward(x, n, d, m, ks, codes, codebook, grad_out, grad_x, grad_codebook, nch, part_s,
                            part_cnt, part_j, loss_sub, s)))
    return rc;
  if (loss && (rc = launch_objective(loss_sub, 1, m, loss, s))) return rc;
  return MIPQ_OK;
}

// ---------------------------------------------------------------- inverted file
namespace {

struct CoarseWs {
  void* aop = nullptr;
  float* mu = nullptr;
  unsigned int* cmax = nullptr;
};

CoarseWs carve_coarse(Carver& c, int d, int kc, int precision) {
  CoarseWs w;
  if (precision == MIPQ_BF16) {
    w.aop = c.take<uint4>(coarse_operand_count(kc, d));
    w.mu = c.take<float>(d);
    w.cmax = c.take<unsigned int>(4);
  }
  return w;
}

int check_coarse(int64_t n, int d, int kc, int precision) {
  if (n < 0 || n >= (int64_t(1) << 31)) return fail(MIPQ_EINVAL, "n out of range (%lld)", (long long)n);
  if (d <= 0) return fail(MIPQ_EINVAL, "d must be positive");
  if (kc < 1 || kc > 65536) return fail(MIPQ_EINVAL, "kc must be in [1, 65536] (got %d)", kc);
  if (precision == MIPQ_BF16) {
    const int S = coarse_ksteps(d);
    if (d > 256 || !(S == 1 || S == 2 || S == 4 || S == 6 || S == 8 || S == 12 || S == 16))
      return fail(MIPQ_EUNSUPPORTED, "coarse matrix-core path needs d <= 16 or d in {32, 64, 96, 128, 192, 256}");
  } else if (precision == MIPQ_FP8) {
    return fail(MIPQ_EUNSUPPORTED, "the coarse quantiser runs in MIPQ_FP32 or MIPQ_BF16");
  } else if (precision != MIPQ_FP32) {
    return fail(MIPQ_EINVAL, "unknown precision %d", precision);
  }
  return MIPQ_OK;
}

int coarse_assign_any(const float* x, int64_t n, int d, const float* cc, int kc, int precision,
                      const CoarseWs& w, int32_t* labels, int64_t* rescored, hipStream_t s) {
  int rc;
  if (precision == MIPQ_BF16 && (rc = launch_coarse_prepare(cc, kc, d, w.mu, w.cmax, w.aop, s))) return rc;
  return launch_coarse_assign(x, n, d, cc, kc, w.aop, w.mu, w.cmax, labels, rescored,
                              precision != MIPQ_BF16, s);
}

struct BuildWs {
  float* xs;
  double* cc64;
  int32_t* tlabels;
  uint32_t *keys_a, *keys_b, *keys_sorted, *hist;
  int32_t *vals_a, *vals_b, *tids;
  int64_t* toffsets;
  double* obj_list;
  CoarseWs cw;
  float* rtrain;
  int32_t* lab;
  uint8_t* codes;
  float* rbuf;
  int64_t chunk;
  void* sub;
  size_t sub_bytes;
  size_t bytes;
};

BuildWs carve_build(void* ws, int64_t n, int d, int kc, int64_t n_train, int m, int ks, int pq_iters,
                    int precision, bool need_labels) {
  Carver c(ws);
  BuildWs b;
  const int64_t nmax = n > n_train ? n : n_train;
  b.xs = c.take<float>((size_t)n_train * d);
  b.cc64 = c.take<double>((size_t)kc * d);
  b.tlabels = c.take<int32_t>(n_train);
  b.keys_a = c.take<uint32_t>(nmax);
  b.keys_b = c.take<uint32_t>(nmax);
  b.keys_sorted = c.take<uint32_t>(nmax);
  b.hist = c.take<uint32_t>(sort_hist_entries(nmax));
  b.vals_a = c.take<int32_t>(nmax);
  b.vals_b = c.take<int32_t>(nmax);
  b.tids = c.take<int32_t>(n_train);
  b.toffsets = c.take<int64_t>(kc + 1);
  b.obj_list = c.take<double>(kc);
  b.cw = carve_coarse(c, d, kc, precision);
  b.rtrain = c.take<float>((size_t)n_train * d);
  b.lab = need_labels ? c.take<int32_t>(n) : nullptr;
  b.codes = c.take<uint8_t>((size_t)n * m);
  b.chunk = n < (int64_t(1) << 20) ? n : (int64_t(1) << 20);
  b.rbuf = c.take<float>((size_t)b.chunk * d);
  const size_t fitb = mipq_pq_fit_workspace_size(n_train, d, m, ks, pq_iters, precision);
  const size_t encb = mipq_pq_encode_workspace_size(b.chunk, d, m, ks, precision);
  b.sub_bytes = fitb > encb ? fitb : encb;
  b.sub = c.take<char>(b.sub_bytes);
  b.bytes = c.bytes();
  return b;
}

}  // namespace

size_t mipq_coarse_assign_workspace_size(int d, int kc, int precision) {
  if (check_coarse(0, d, kc, precision) != MIPQ_OK) return 0;
  Carver c(nullptr);
  carve_coarse(c, d, kc, precision);
  return c.bytes();
}

int mipq_coarse_assign(const float* x, int64_t n, int d, const float* coarse, int kc, int precision,
                       int32_t* labels, int64_t* rescored, void* ws, size_t ws_bytes, void* stream) {
  int rc;
  if ((rc = check_coarse(n, d, kc, precision))) return rc;
  if (!coarse || (n > 0 && (!x || !labels))) return fail(MIPQ_EINVAL, "x, coarse and labels are required");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Carver c(ws);
  CoarseWs w = carve_coarse(c, d, kc, precision);
  if ((rc = check_ws(ws, ws_bytes, c.bytes()))) return rc;
  if (rescored && (rc = launch_zero_u32(reinterpret_cast<uint32_t*>(rescored), 2, s))) return rc;
  if (n == 0) return MIPQ_OK;
  return coarse_assign_any(x, n, d, coarse, kc, precision, w, labels, rescored, s);
}

namespace {
struct KmWs {
  float* xs;
  double* cc64;
  int32_t* lab;
  uint32_t *keys_a, *keys_b, *keys_sorted, *hist;
  int32_t *vals_a, *vals_b, *tids;
  int64_t* toffsets;
  double* obj_list;
  CoarseWs cw;
  size_t bytes;
};

KmWs carve_kmeans(void* ws, int64_t n_train, bool gather, int d, int k, int precision, bool need_labels) {
  Carver c(ws);
  KmWs w;
  w.xs = gather ? c.take<float>((size_t)n_train * d) : nullptr;
  w.cc64 = c.take<double>((size_t)k * d);
  w.lab = need_labels ? c.take<int32_t>(n_train) : nullptr;
  w.keys_a = c.take<uint32_t>(n_train);
  w.keys_b = c.take<uint32_t>(n_train);
  w.keys_sorted = c.take<uint32_t>(n_train);
  w.hist = c.take<uint32_t>(sort_hist_entries(n_train));
  w.vals_a = c.take<int32_t>(n_train);
  w.vals_b = c.take<int32_t>(n_train);
  w.tids = c.take<int32_t>(n_train);
  w.toffsets = c.take<int64_t>(k + 1);
  w.obj_list = c.take<double>(k);
  w.cw = carve_coarse(c, d, k, precision);
  w.bytes = c.bytes();
  return w;
}
}  // namespace

size_t mipq_kmeans_fit_workspace_size(int64_t n_train, int d, int k, int iters, int precision) {
  if (n_train < 1 || iters < 0 || check_coarse(n_train, d, k, precision) != MIPQ_OK) return 0;
  return carve_kmeans(nullptr, n_train, true, d, k, precision, true).bytes;
}

int mipq_kmeans_fit(const float* x, int64_t n, const int64_t* train_rows, int64_t n_train, int d, int k, int iters,
                    const int64_t* init_rows, int precision, float* centroids, int32_t* labels, double* objective,
                    void* ws, size_t ws_bytes, void* stream) {
  int rc;
  const int64_t nt = train_rows ? n_train : n;
  if ((rc = check_coarse(nt, d, k, precision))) return rc;
  if (nt < 1 || (train_rows && n < 1)) return fail(MIPQ_EINVAL, "fit needs at least one training row");
  if (iters < 0 || iters > (1 << 16)) return fail(MIPQ_EINVAL, "iters out of range (%d)", iters);
  if (!x || !init_rows || !centroids) return fail(MIPQ_EINVAL, "x, init_rows and centroids are required");
  hipStream_t s = static_cast<hipStream_t>(stream);
  KmWs w = carve_kmeans(ws, nt, train_rows != nullptr, d, k, precision, labels == nullptr);
  if ((rc = check_ws(ws, ws_bytes, w.bytes))) return rc;
  const float* train = x;
  if (train_rows) {
    uint32_t* bad = w.hist;   // scratch flag before the first sort
    if ((rc = launch_gather_rows(x, n, d, train_rows, nt, w.xs, bad, s))) return rc;
    train = w.xs;
  }
  int32_t* lab = labels ? labels : w.lab;
  if ((rc = launch_gather_coarse(train, nt, d, init_rows, k, centroids, w.cc64, s))) return rc;
  for (int it = 0; it < iters; ++it) {
    if ((rc = coarse_assign_any(train, nt, d, centroids, k, precision, w.cw, lab, nullptr, s))) return rc;
    if ((rc = launch_sort_by_label(lab, nt, k, w.keys_a, w.keys_b, w.vals_a, w.vals_b, w.hist, w.tids,
                                   w.keys_sorted, w.toffsets, s)))
      return rc;
    if ((rc = launch_coarse_update(train, d, w.tids, w.toffsets, k, centroids, w.cc64, w.obj_list,
                                   objective ? objective + it : nullptr, s)))
      return rc;
  }
  return MIPQ_OK;
}

size_t mipq_ii_build_workspace_size(int64_t n, int d, int kc, int64_t n_train, int m, int ks, int pq_iters,
                                    int coarse_iters, int precision) {
  if (check_coarse(n, d, kc, precision) != MIPQ_OK || check_shape(n_train, d, m, ks, precision, true) != MIPQ_OK)
    return 0;
  (void)coarse_iters;
  return carve_build(nullptr, n, d, kc, n_train, m, ks, pq_iters, precision, true).bytes;
}

int mipq_ii_build(const float* x, int64_t n, int d, int kc, int coarse_iters, const int64_t* train_rows,
                  int64_t n_train, const int64_t* coarse_init, int m, int ks, int pq_iters,
                  const int64_t* pq_init, int precision, float* coarse, float* pq_codebook,
                  int64_t* offsets, int32_t* ids, uint8_t* codes_sorted, int32_t* labels,
                  double* coarse_objective, void* ws, size_t ws_bytes, void* stream) {
  int rc;
  if ((rc = check_coarse(n, d, kc, precision))) return rc;
  if ((rc = check_shape(n_train, d, m, ks, precision, true))) return rc;
  if (n < 1 || n_train < 1) return fail(MIPQ_EINVAL, "n and n_train must be positive");
  if (coarse_iters < 0 || pq_iters < 0) return fail(MIPQ_EINVAL, "iteration counts must be >= 0");
  if (!x || !train_rows || !coarse_init || !pq_init || !coarse || !pq_codebook || !offsets || !ids || !codes_sorted)
    return fail(MIPQ_EINVAL, "a required pointer is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  BuildWs b = carve_build(ws, n, d, kc, n_train, m, ks, pq_iters, precision, labels == nullptr);
  if ((rc = check_ws(ws, ws_bytes, b.bytes))) return rc;
  int32_t* lab = labels ? labels : b.lab;
  uint32_t* bad = reinterpret_cast<uint32_t*>(b.hist);   // scratch flag before the first sort
  // 1. training sample and coarse init
  if ((rc = launch_gather_rows(x, n, d, train_rows, n_train, b.xs, bad, s))) return rc;
  if ((rc = launch_gather_coarse(b.xs, n_train, d, coarse_init, kc, coarse, b.cc64, s))) return rc;
  // 2. coarse Lloyd rounds on the sample
  for (int it = 0; it < coarse_iters; ++it) {
    if ((rc = coarse_assign_any(b.xs, n_train, d, coarse, kc, precision, b.cw, b.tlabels, nullptr, s))) return rc;
    if ((rc = launch_sort_by_label(b.tlabels, n_train, kc, b.keys_a, b.keys_b, b.vals_a, b.vals_b, b.hist, b.tids,
                                   b.keys_sorted, b.toffsets, s)))
      return rc;
    if ((rc = launch_coarse_update(b.xs, d, b.tids, b.toffsets, kc, coarse, b.cc64, b.obj_list,
                                   coarse_objective ? coarse_objective + it : nullptr, s)))
      return rc;
  }
  // 3. final sample labels, residuals, residual PQ fit
  if ((rc = coarse_assign_any(b.xs, n_train, d, coarse, kc, precision, b.cw, b.tlabels, nullptr, s))) return rc;
  if ((rc = launch_residuals(b.xs, n_train, d, b.tlabels, coarse, kc, b.rtrain, s))) return rc;
  if ((rc = mipq_pq_fit(b.rtrain, n_train, nullptr, 0, d, m, ks, pq_iters, pq_init, nullptr, precision, 0,
                        pq_codebook, nullptr, nullptr, nullptr, nullptr, b.sub, b.sub_bytes, stream)))
    return rc;
  // 4. labels and residual codes of all rows (residuals formed chunk by chunk)
  if ((rc = coarse_assign_any(x, n, d, coarse, kc, precision, b.cw, lab, nullptr, s))) return rc;
  for (int64_t a = 0; a < n; a += b.chunk) {
    const int64_t cnt = (n - a) < b.chunk ? (n - a) : b.chunk;
    if ((rc = launch_residuals(x + a * d, cnt, d, lab + a, coarse, kc, b.rbuf, s))) return rc;
    if ((rc = mipq_pq_encode(b.rbuf, cnt, d, m, ks, pq_codebook, precision, 0, b.codes + a * m, nullptr, nullptr,
                             nullptr, b.sub, b.sub_bytes, stream)))
      return rc;
  }
  // 5. stable bucketing by label, codes in list order
  if ((rc = launch_sort_by_label(lab, n, kc, b.keys_a, b.keys_b, b.vals_a, b.vals_b, b.hist, ids, b.keys_sorted,
                                 offsets, s)))
    return rc;
  return launch_gather_codes(b.codes, n, m, ids, codes_sorted, s);
}

namespace {
struct AddWs {
  CoarseWs cw;
  uint32_t *keys_a, *keys_b, *keys_sorted, *hist;
  int32_t *vals_a, *vals_b, *lab;
  uint8_t* codes;
  float* rbuf;
  int64_t chunk;
  void* sub;
  size_t sub_bytes;
  size_t bytes;
};

AddWs carve_add(void* ws, int64_t n, int d, int kc, int m, int ks, int precision, bool need_labels) {
  Carver c(ws);
  AddWs a;
  const int64_t nn = n > 0 ? n : 1;
  a.cw = carve_coarse(c, d, kc, precision);
  a.keys_a = c.take<uint32_t>(nn);
  a.keys_b = c.take<uint32_t>(nn);
  a.keys_sorted = c.take<uint32_t>(nn);
  a.hist = c.take<uint32_t>(sort_hist_entries(nn));
  a.vals_a = c.take<int32_t>(nn);
  a.vals_b = c.take<int32_t>(nn);
  a.lab = need_labels ? c.take<int32_t>(nn) : nullptr;
  a.codes = c.take<uint8_t>((size_t)nn * m);
  a.chunk = nn < (int64_t(1) << 20) ? nn : (int64_t(1) << 20);
  a.rbuf = c.take<float>((size_t)a.chunk * d);
  a.sub_bytes = mipq_pq_encode_workspace_size(a.chunk, d, m, ks, precision);
  a.sub = a.sub_bytes ? c.take<char>(a.sub_bytes) : nullptr;
  a.bytes = c.bytes();
  return a;
}
}  // namespace

size_t mipq_ii_add_workspace_size(int64_t n, int d, int kc, int m, int ks, int precision) {
  if (check_coarse(n, d, kc, precision) != MIPQ_OK || check_shape(n, d, m, ks, precision, false) != MIPQ_OK)
    return 0;
  return carve_add(nullptr, n, d, kc, m, ks, precision, true).bytes;
}

int mipq_ii_add(const float* x, int64_t n, int d, const float* coarse, int kc, const float* pq_codebook, int m,
                int ks, int precision, int64_t* offsets, int32_t* ids, uint8_t* codes_sorted, int32_t* labels,
                void* ws, size_t ws_bytes, void* stream) {
  int rc;
  if ((rc = check_coarse(n, d, kc, precision))) return rc;
  if ((rc = check_shape(n, d, m, ks, precision, false))) return rc;
  if (!coarse || !pq_codebook || !offsets || (n > 0 && (!x || !ids || !codes_sorted)))
    return fail(MIPQ_EINVAL, "a required pointer is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  AddWs a = carve_add(ws, n, d, kc, m, ks, precision, labels == nullptr);
  if ((rc = check_ws(ws, ws_bytes, a.bytes))) return rc;
  int32_t* lab = labels ? labels : a.lab;
  if (n == 0) return launch_zero_u32(reinterpret_cast<uint32_t*>(offsets), 2 * (kc + 1), s);
  // labels and residual codes of the rows, then stable bucketing by label
  if ((rc = coarse_assign_any(x, n, d, coarse, kc, precision, a.cw, lab, nullptr, s))) return rc;
  for (int64_t r = 0; r < n; r += a.chunk) {
    const int64_t cnt = (n - r) < a.chunk ? (n - r) : a.chunk;
    if ((rc = launch_residuals(x + r * d, cnt, d, lab + r, coarse, kc, a.rbuf, s))) return rc;
    if ((rc = mipq_pq_encode(a.rbuf, cnt, d, m, ks, pq_codebook, precision, 0, a.codes + r * m, nullptr, nullptr,
                             nullptr, a.sub, a.sub_bytes, stream)))
      return rc;
  }
  if ((rc = launch_sort_by_label(lab, n, kc, a.keys_a, a.keys_b, a.vals_a, a.vals_b, a.hist, ids, a.keys_sorted,
                                 offsets, s)))
    return rc;
  return launch_gather_codes(a.codes, n, m, ids, codes_sorted, s);
}

size_t mipq_ii_merge_workspace_size(int nparts, int kc) {
  if (nparts < 1 || kc < 1 || kc > 65536) return 0;
  Carver c(nullptr);
  c.take<char>(merge_part_bytes() * (size_t)nparts);
  c.take<int64_t>((size_t)nparts * kc);
  c.take<int64_t>(kc);
  return c.bytes();
}

int mipq_ii_merge(const int64_t* const* part_offsets, const int32_t* const* part_ids,
                  const uint8_t* const* part_codes, const int64_t* part_n, int nparts, int kc, int m,
                  int64_t* offsets, int32_t* ids, uint8_t* codes_sorted, void* ws, size_t ws_bytes, void* stream) {
  if (nparts < 1) return fail(MIPQ_EINVAL, "nparts must be positive");
  if (kc < 1 || kc > 65536) return fail(MIPQ_EINVAL, "kc must be in [1, 65536] (got %d)", kc);
  if (m < 1 || m > 256) return fail(MIPQ_EINVAL, "m must be in [1, 256] (got %d)", m);
  if (!part_offsets || !part_ids || !part_codes || !part_n || !offsets)
    return fail(MIPQ_EINVAL, "a required pointer is NULL");
  struct Part {
    const int64_t* off;
    const int32_t* ids;
    const uint8_t* codes;
    int64_t n;
    int64_t base;
  };
  static_assert(sizeof(Part) == 40, "part record");
  if (merge_part_bytes() != sizeof(Part)) return fail(MIPQ_EINVAL, "part record size mismatch");
  std::vector<Part> table((size_t)nparts);
  int64_t total = 0;
  bool vec16 = (m % 16) == 0 && (reinterpret_cast<uintptr_t>(codes_sorted) % 16) == 0;
  for (int p = 0; p < nparts; ++p) {
    const int64_t np = part_n[p];
    if (np < 0) return fail(MIPQ_EINVAL, "part %d has a negative row count", p);
    if (!part_offsets[p] || (np > 0 && (!part_ids[p] || !part_codes[p])))
      return fail(MIPQ_EINVAL, "part %d: a required pointer is NULL", p);
    vec16 = vec16 && (reinterpret_cast<uintptr_t>(part_codes[p]) % 16) == 0;
    table[p] = Part{part_offsets[p], part_ids[p], part_codes[p], np, total};
    total += np;
    if (total >= (int64_t(1) << 31)) return fail(MIPQ_EINVAL, "merged index exceeds 2^31 - 1 rows");
  }
  if (total > 0 && (!ids || !codes_sorted)) return fail(MIPQ_EINVAL, "ids and codes_sorted are required");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Carver c(ws);
  void* dtab = c.take<char>(sizeof(Part) * (size_t)nparts);
  int64_t* pre = c.take<int64_t>((size_t)nparts * kc);
  int64_t* tot = c.take<int64_t>(kc);
  int rc;
  if ((rc = check_ws(ws, ws_bytes, c.bytes()))) return rc;
  // the table lives in this call's host memory: copy it and wait
  hipError_t e = hipMemcpyAsync(dtab, table.data(), sizeof(Part) * (size_t)nparts, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(part table)");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  return launch_merge_lists(dtab, nparts, total, kc, m, pre, tot, offsets, ids, codes_sorted, vec16, s);
}

namespace {
struct AdcWs {
  CoarseWs cw;
  float* est;
  int32_t* probes;
  unsigned long long* qthr;
  uint64_t* pair_out;
  void* order_ws;
  size_t bytes;
};
AdcWs carve_adc(void* ws, int nq, int d, int kc, int nprobe, int topk) {
  Carver c(ws);
  AdcWs a;
  a.cw = carve_coarse(c, d, kc, MIPQ_BF16);
  a.est = c.take<float>((size_t)nq * kc);
  a.probes = c.take<int32_t>((size_t)nq * nprobe);
  a.qthr = c.take<unsigned long long>((size_t)nq);
  a.pair_out = c.take<uint64_t>((size_t)nq * nprobe * topk);
  a.order_ws = c.take<char>(adc_order_bytes((int64_t)nq * nprobe, nprobe, kc));
  a.bytes = c.bytes();
  return a;
}
}  // namespace

size_t mipq_adc_search_workspace_size(int nq, int d, int kc, int nprobe, int topk) {
  if (nq < 0 || check_coarse(0, d, kc, MIPQ_BF16) != MIPQ_OK || nprobe < 1 || topk < 1 || topk > 1024) return 0;
  return carve_adc(nullptr, nq, d, kc, nprobe, topk).bytes;
}

int mipq_adc_search(const float* q, int nq, int d, const float* coarse, int kc, const float* pq_codebook,
                    int m, int ks, const int64_t* offsets, const int32_t* ids, const uint8_t* codes_sorted,
                    int nprobe, int topk, int32_t* out_ids, float* out_dist, int64_t* wide, int64_t* work,
                    void* ws, size_t ws_bytes, void* stream) {
  int rc;
  if (nq < 0) return fail(MIPQ_EINVAL, "nq must be >= 0");
  if ((rc = check_coarse(0, d, kc, MIPQ_BF16))) return rc;
  if ((rc = check_shape(0, d, m, ks, MIPQ_FP32, false))) return rc;
  const int ds = d / m;
  if (!(ds == 1 || ds == 2 || ds == 4 || ds == 8 || ds == 16))
    return fail(MIPQ_EUNSUPPORTED, "ADC supports d/m in {1, 2, 4, 8, 16} (got %d)", ds);
  if (topk >= 1 && topk <= 1024 && !adc_fits_lds(d, m, ks, topk))
    return fail(MIPQ_EUNSUPPORTED, "ADC table of m x ks = %d x %d floats does not fit one block's LDS", m, ks);
  if (nprobe < 1 || nprobe > kc || nprobe > 256) return fail(MIPQ_EINVAL, "nprobe must be in [1, min(kc, 256)]");
  if (topk < 1 || topk > 1024) return fail(MIPQ_EINVAL, "topk must be in [1, 1024]");
  if (nq > 0 && (!q || !coarse || !pq_codebook || !offsets || !ids || !codes_sorted || !out_ids || !out_dist))
    return fail(MIPQ_EINVAL, "a required pointer is NULL");
  if ((int64_t)nq * nprobe >= (1ll << 31)) return fail(MIPQ_EUNSUPPORTED, "nq * nprobe must be < 2^31");
  hipStream_t s = static_cast<hipStream_t>(stream);
  AdcWs a = carve_adc(ws, nq, d, kc, nprobe, topk);
  if ((rc = check_ws(ws, ws_bytes, a.bytes))) return rc;
  if (wide && (rc = launch_zero_u32(reinterpret_cast<uint32_t*>(wide), 2, s))) return rc;
  if (work && (rc = launch_zero_u32(reinterpret_cast<uint32_t*>(work), 8, s))) return rc;
  if (nq == 0) return MIPQ_OK;
  if ((rc = launch_coarse_prepare(coarse, kc, d, a.cw.mu, a.cw.cmax, a.cw.aop, s))) return rc;
  return launch_adc(q, nq, d, coarse, kc, a.cw.aop, a.cw.mu, a.cw.cmax, pq_codebook, m, ks, offsets, ids,
                    codes_sorted, nprobe, topk, a.est, a.probes, a.qthr, a.pair_out, a.order_ws, wide, out_ids,
                    out_dist, work, s);
}

}  // extern "C"

// ---------------------------------------------------------------- optimized PQ
namespace {
constexpr int kPolarSweeps = 64;

struct ProcWs {
  double *part, *m, *a, *v, *m0, *rj, *vj;
  void* rlog;
  int* sweeps;
  int nch;
  size_t bytes;
};

ProcWs carve_proc(void* ws, int64_t n, int d, bool need_m, bool need_sweeps) {
  Carver c(ws);
  ProcWs w;
  const size_t dd = (size_t)d * d;
  w.nch = n > 0 ? cross_chunks(n, d) : 0;
  w.part = w.nch ? c.take<double>((size_t)w.nch * dd) : nullptr;
  w.m = need_m ? c.take<double>(dd) : nullptr;
  w.a = c.take<double>(dd);
  w.v = c.take<double>(dd);
  w.m0 = c.take<double>(dd);
  w.rj = c.take<double>(dd);
  w.vj = c.take<double>(dd);
  const size_t lb = polar_log_bytes(d, kPolarSweeps);
  w.rlog = lb ? c.take<char>(lb) : nullptr;
  w.sweeps = need_sweeps ? c.take<int>(1) : nullptr;
  w.bytes = c.bytes();
  return w;
}
}  // namespace

int mipq_rotate(const float* x, int64_t n, int d, const double* rotation, float* y, void* stream) {
  if (n < 0) return fail(MIPQ_EINVAL, "n must be >= 0");
  if (d < 1 || d > 4096) return fail(MIPQ_EINVAL, "d must be in [1, 4096] (got %d)", d);
  if (!rotation || (n > 0 && (!x || !y))) return fail(MIPQ_EINVAL, "x, rotation and y are required");
  if (n > 0) {
    const char* xb = reinterpret_cast<const char*>(x);
    const char* yb = reinterpret_cast<const char*>(y);
    const size_t bytes = (size_t)n * d * sizeof(float);
    if (xb < yb + bytes && yb < xb + bytes) return fail(MIPQ_EINVAL, "y must not overlap x");
  }
  return launch_rotate(x, n, d, rotation, y, static_cast<hipStream_t>(stream));
}

size_t mipq_opq_procrustes_workspace_size(int64_t n, int d) {
  if (n < 0 || d < 1 || d > 256) return 0;
  return carve_proc(nullptr, n, d, true, true).bytes;
}

int mipq_opq_procrustes(const float* x, const float* y_hat, int64_t n, int d, const double* v_init,
                        double* rotation, double* v_out, double* cross, int* sweeps, void* ws, size_t ws_bytes,
                        void* stream) {
  if (n < 0) return fail(MIPQ_EINVAL, "n must be >= 0");
  if (d < 1 || d > 256) return fail(MIPQ_EUNSUPPORTED, "the rotation fit supports 1 <= d <= 256 (got %d)", d);
  if (!rotation || (n > 0 && (!x || !y_hat))) return fail(MIPQ_EINVAL, "x, y_hat and rotation are required");
  hipStream_t s = static_cast<hipStream_t>(stream);
  ProcWs w = carve_proc(ws, n, d, cross == nullptr, sweeps == nullptr);
  int rc;
  if ((rc = check_ws(ws, ws_bytes, w.bytes))) return rc;
  double* m = cross ? cross : w.m;
  int* sw = sweeps ? sweeps : w.sweeps;
  if (n == 0) {
    if ((rc = launch_zero_u32(reinterpret_cast<uint32_t*>(m), (size_t)d * d * 2, s))) return rc;
  } else if ((rc = launch_cross(x, y_hat, n, d, w.nch, w.part, m, s))) {
    return rc;
  }
  return launch_polar(m, d, kPolarSweeps, v_init, w.m0, w.a, w.v, w.rj, w.vj, w.rlog, rotation, v_out, sw, s);
}
