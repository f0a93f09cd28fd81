// C-ABI entry points of libmipq: argument checks, workspace carving and the
// launch sequence of each call.  See include/mipq.h for the contract.
#include <stdarg.h>
#include <stdio.h>

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
  } else if (precision == MIPQ_BF16) {
    if (ds > kMaxDsBf16) return fail(MIPQ_EUNSUPPORTED, "BF16 path supports d/m <= %d (got %d)", kMaxDsBf16, ds);
    if ((uint64_t)n * (uint64_t)m >= (1ull << 32))
      return fail(MIPQ_EUNSUPPORTED, "BF16 path needs n*m < 2^32");
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

EncodeWs carve_encode(void* ws, int m, int ks, int ds, int precision) {
  Carver c(ws);
  EncodeWs e;
  if (precision == MIPQ_BF16) {
    e.aop = c.take<uint4>(bf16_operand_count(m, ks, ds));
    e.cmax = c.take<float>(m);
    e.mu = c.take<float>((size_t)m * kMaxDsBf16);
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
  int nch = 1;
  EncodeWs enc;
  size_t bytes = 0;
};

FitWs carve_fit(void* ws, int64_t n_train, bool gather, int d, int m, int ks, int iters,
                int precision, bool need_codes, bool need_c64) {
  Carver c(ws);
  FitWs f;
  const int ds = d / m;
  f.nch = update_chunks(n_train, m);
  if (gather) f.xs = c.take<float>((size_t)n_train * d);
  if (need_codes) f.codes = c.take<uint8_t>((size_t)n_train * m);
  if (need_c64) f.c64 = c.take<double>((size_t)m * ks * ds);
  f.part_s = c.take<double>((size_t)f.nch * m * ks * ds);
  f.part_cnt = c.take<uint32_t>((size_t)f.nch * m * ks);
  f.part_j = c.take<double>((size_t)f.nch * m);
  f.j_sub = c.take<double>((size_t)(iters > 0 ? iters : 1) * m);
  f.bad = c.take<uint32_t>(4);
  const size_t off = c.bytes();
  EncodeWs e = carve_encode(ws ? static_cast<char*>(ws) + off : nullptr, m, ks, ds, precision);
  f.enc = e;
  f.bytes = off + e.bytes;
  return f;
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
  return launch_assign_bf16(x, n, d, m, ks, e.aop, e.cmax, e.mu, c32, codes, rescored, s);
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
                int precision, float* codebook, double* codebook64, uint8_t* labels,
                double* objective, void* ws, size_t ws_bytes, void* stream) {
  int rc;
  const int64_t nt = train_rows ? n_train : n;
  if ((rc = check_shape(nt, d, m, ks, precision, true))) return rc;
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
  uint8_t* codes = labels ? labels : f.codes;
  double* c64 = codebook64 ? codebook64 : f.c64;
  float* c32 = codebook;   // working float32 codebook, final value on return
  if ((rc = launch_init_codebook(train, nt, d, m, ks, init_codebook ? nullptr : init_rows, init_codebook,
                                 c64, c32, f.bad, nullptr, s)))
    return rc;
  const bool bf = precision == MIPQ_BF16;
  if (bf && iters > 0 && (rc = launch_pack_bf16(c32, m, ks, ds, f.enc.aop, f.enc.cmax, f.enc.mu, s))) return rc;
  for (int it = 0; it < iters; ++it) {
    if ((rc = assign_any(train, nt, d, m, ks, c32, precision, codes, f.enc, nullptr, s))) return rc;
    // the update also packs the next round's operands (BF16)
    if ((rc = launch_update(train, nt, d, m, ks, codes, c32, c64, f.nch, f.part_s, f.part_cnt, f.part_j,
                            f.j_sub + (size_t)it * m, bf ? f.enc.aop : nullptr, f.enc.cmax, f.enc.mu, s)))
      return rc;
  }
  if (objective && (rc = launch_objective(f.j_sub, iters, m, objective, s))) return rc;
  return MIPQ_OK;
}

size_t mipq_pq_encode_workspace_size(int64_t n, int d, int m, int ks, int precision) {
  if (check_shape(n, d, m, ks, precision, false) != MIPQ_OK) return 0;
  return carve_encode(nullptr, m, ks, d / m, precision).bytes;
}

int mipq_pq_encode(const float* x, int64_t n, int d, int m, int ks, const float* codebook,
                   int precision, uint8_t* codes, int64_t* rescored, void* ws, size_t ws_bytes,
                   void* stream) {
  int rc;
  if ((rc = check_shape(n, d, m, ks, precision, false))) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (n > 0 && (!x || !codebook || !codes)) return fail(MIPQ_EINVAL, "x, codebook and codes are required");
  EncodeWs e = carve_encode(ws, m, ks, d / m, precision);
  if (n > 0 && (rc = check_ws(ws, ws_bytes, e.bytes))) return rc;
  if (rescored && (rc = launch_zero_u32(reinterpret_cast<uint32_t*>(rescored), 2, s))) return rc;
  if (n == 0) return MIPQ_OK;
  if (precision == MIPQ_BF16 && (rc = launch_pack_bf16(codebook, m, ks, d / m, e.aop, e.cmax, e.mu, s)))
    return rc;
  return assign_any(x, n, d, m, ks, codebook, precision, codes, e, rescored, s);
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

}  // extern "C"
