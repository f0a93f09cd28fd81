// Issue-rate and bandwidth probes behind the roofline peaks.
//
// The roofline fractions of the hot path are quoted against peaks derived from
// the chip's unit counts and clock (256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz for
// unpacked vector instructions; the published matrix-core and HBM figures).
// These kernels measure what one launch of each instruction kind actually
// sustains on the device, so that the derivation can be checked:
//   * every lane runs kChains independent chains of one vector instruction
//     (float32 add with a scalar or a vector operand, float32 fused
//     multiply-add, float32 2- and 3-input minimum, float64 fused
//     multiply-add; or 3-input minima and vector adds alternating), long
//     enough that latency is hidden by the chains and the 8 waves per SIMD.
//     The vector-vector add issues two instructions per quad-cycle on gfx950
//     (counter SQ_ACTIVE_INST_VALU2), minima do not, and a minimum and an add
//     of different waves can issue together;
//   * the matrix-core probes run four independent accumulators of one MFMA
//     shape per wave;
//   * the copy probe streams a buffer's first half into its second half with
//     16-byte loads and stores.
// Each launch writes one value per lane (or the copy) so that no work can be
// removed by the compiler.  This file is compiled with -fno-honor-nans so that
// the minimum chains become v_min3_f32.
#include "mipq_internal.h"

namespace mipq {

namespace {

constexpr int kChains = 8;
constexpr int kIter = 2048;
constexpr int kMfmaIter = 512;
constexpr int kThreads = 256;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__global__ __launch_bounds__(kThreads) void k_probe_add(float* out, float b) {
  float a[kChains];
#pragma unroll
  for (int j = 0; j < kChains; ++j) a[j] = threadIdx.x * 0.001f + j;
  for (int i = 0; i < kIter; ++i)
#pragma unroll
    for (int j = 0; j < kChains; ++j) a[j] = a[j] + b;
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < kChains; ++j) s = s + a[j];
  out[blockIdx.x * kThreads + threadIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void k_probe_fma(float* out, float b, float c) {
  float a[kChains];
#pragma unroll
  for (int j = 0; j < kChains; ++j) a[j] = threadIdx.x * 0.001f + j;
  for (int i = 0; i < kIter; ++i)
#pragma unroll
    for (int j = 0; j < kChains; ++j) a[j] = __builtin_fmaf(a[j], b, c);
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < kChains; ++j) s = s + a[j];
  out[blockIdx.x * kThreads + threadIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void k_probe_min3(float* out, float b) {
  float a[kChains];
#pragma unroll
  for (int j = 0; j < kChains; ++j) a[j] = threadIdx.x * 0.001f + j;
  for (int i = 0; i < kIter; ++i)
#pragma unroll
    for (int j = 0; j < kChains; ++j) a[j] = fminf(fminf(a[j], a[(j + 1) % kChains]), b);
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < kChains; ++j) s = s + a[j];
  out[blockIdx.x * kThreads + threadIdx.x] = s;
}

// vector-vector forms: every operand in a VGPR (e differs per chain)
__global__ __launch_bounds__(kThreads) void k_probe_add_vv(float* out) {
  float a[kChains], e[kChains];
#pragma unroll
  for (int j = 0; j < kChains; ++j) {
    a[j] = threadIdx.x * 0.001f + j;
    e[j] = 0.5f + j;
  }
  for (int i = 0; i < kIter; ++i)
#pragma unroll
    for (int j = 0; j < kChains; ++j) a[j] = a[j] + e[j];
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < kChains; ++j) s = s + a[j];
  out[blockIdx.x * kThreads + threadIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void k_probe_min_vv(float* out) {
  float a[kChains];
#pragma unroll
  for (int j = 0; j < kChains; ++j) a[j] = threadIdx.x * 0.001f + j;
  for (int i = 0; i < kIter; ++i)
#pragma unroll
    for (int j = 0; j < kChains; ++j) a[j] = fminf(a[j], a[(j + 1) % kChains]);
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < kChains; ++j) s = s + a[j];
  out[blockIdx.x * kThreads + threadIdx.x] = s;
}

// half the chains 3-input minima, half vector-vector adds
__global__ __launch_bounds__(kThreads) void k_probe_min3_add(float* out) {
  float a[kChains], e[kChains];
#pragma unroll
  for (int j = 0; j < kChains; ++j) {
    a[j] = threadIdx.x * 0.001f + j;
    e[j] = 0.5f + j;
  }
  for (int i = 0; i < kIter; ++i)
#pragma unroll
    for (int j = 0; j < kChains; ++j)
      a[j] = (j & 1) ? fminf(fminf(a[j], a[j - 1]), e[j]) : a[j] + e[j];
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < kChains; ++j) s = s + a[j];
  out[blockIdx.x * kThreads + threadIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void k_probe_fma64(double* out, double b, double c) {
  double a[kChains];
#pragma unroll
  for (int j = 0; j < kChains; ++j) a[j] = threadIdx.x * 0.001 + j;
  for (int i = 0; i < kIter; ++i)
#pragma unroll
    for (int j = 0; j < kChains; ++j) a[j] = __builtin_fma(a[j], b, c);
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < kChains; ++j) s = s + a[j];
  out[blockIdx.x * kThreads + threadIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void k_probe_mfma_bf16(float* out) {
  bf16x8 a, b;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    a[e] = (__bf16)(0.001f * (threadIdx.x + e));
    b[e] = (__bf16)(0.002f * e);
  }
  f32x16 c0 = {}, c1 = {}, c2 = {}, c3 = {};
  for (int i = 0; i < kMfmaIter; ++i) {
    c0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c3, 0, 0, 0);
  }
  float s = 0.0f;
#pragma unroll
  for (int r = 0; r < 16; ++r) s = s + c0[r] + c1[r] + c2[r] + c3[r];
  out[blockIdx.x * kThreads + threadIdx.x] = s;
}

// 32x32x64 OCP E4M3 x E4M3, the instruction of the FP8 assignment
__global__ __launch_bounds__(kThreads) void k_probe_mfma_f8(float* out) {
  i32x8 a, b;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    a[e] = 0x38383838 + (int)((threadIdx.x + e) & 7);
    b[e] = 0x30303030 + e;
  }
  f32x16 c0 = {}, c1 = {}, c2 = {}, c3 = {};
  for (int i = 0; i < kMfmaIter; ++i) {
    c0 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c0, 0, 0, 0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c1, 0, 0, 0, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c2, 0, 0, 0, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c3, 0, 0, 0, 0, 0, 0);
  }
  float s = 0.0f;
#pragma unroll
  for (int r = 0; r < 16; ++r) s = s + c0[r] + c1[r] + c2[r] + c3[r];
  out[blockIdx.x * kThreads + threadIdx.x] = s;
}

// first half of buf -> second half, 16 bytes per lane per step
__global__ __launch_bounds__(kThreads) void k_probe_copy(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                         int64_t count) {
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < count; i += stride) dst[i] = src[i];
}

}  // namespace

}  // namespace mipq

extern "C" {

int mipq_peak_probe(int kind, int blocks, void* out, size_t out_bytes, double* work, void* stream) {
  using namespace mipq;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (blocks < 1 || blocks > (1 << 20) || !out) return fail(MIPQ_EINVAL, "peak_probe: bad blocks or buffer");
  const double lanes = (double)blocks * kThreads;
  const size_t lane_bytes = (size_t)blocks * kThreads * sizeof(double);
  double w = 0.0;
  switch (kind) {
    case MIPQ_PROBE_ADD_F32:
    case MIPQ_PROBE_FMA_F32:
    case MIPQ_PROBE_MIN3_F32:
    case MIPQ_PROBE_FMA_F64:
    case MIPQ_PROBE_MFMA_BF16:
    case MIPQ_PROBE_MFMA_F8:
    case MIPQ_PROBE_ADD_VV:
    case MIPQ_PROBE_MIN_VV:
    case MIPQ_PROBE_MIN3_ADD:
      if (out_bytes < lane_bytes) return fail(MIPQ_EINVAL, "peak_probe: buffer below blocks*256*8 bytes");
      break;
    case MIPQ_PROBE_COPY:
      if (out_bytes < 2 * 16 * (size_t)kThreads || (reinterpret_cast<uintptr_t>(out) & 15))
        return fail(MIPQ_EINVAL, "peak_probe: copy buffer too small or not 16-byte aligned");
      break;
    default:
      return fail(MIPQ_EINVAL, "peak_probe: unknown kind %d", kind);
  }
  switch (kind) {
    case MIPQ_PROBE_ADD_F32:
      k_probe_add<<<blocks, kThreads, 0, s>>>(static_cast<float*>(out), 1.0f);
      w = lanes * kIter * kChains;
      break;
    case MIPQ_PROBE_FMA_F32:
      k_probe_fma<<<blocks, kThreads, 0, s>>>(static_cast<float*>(out), 0.999f, 0.5f);
      w = lanes * kIter * kChains;
      break;
    case MIPQ_PROBE_MIN3_F32:
      k_probe_min3<<<blocks, kThreads, 0, s>>>(static_cast<float*>(out), 0.5f);
      w = lanes * kIter * kChains;
      break;
    case MIPQ_PROBE_FMA_F64:
      k_probe_fma64<<<blocks, kThreads, 0, s>>>(static_cast<double*>(out), 0.999, 0.5);
      w = lanes * kIter * kChains;
      break;
    case MIPQ_PROBE_MFMA_BF16:
      k_probe_mfma_bf16<<<blocks, kThreads, 0, s>>>(static_cast<float*>(out));
      w = (double)blocks * (kThreads / 64) * kMfmaIter * 4 * (2.0 * 32 * 32 * 16);
      break;
    case MIPQ_PROBE_MFMA_F8:
      k_probe_mfma_f8<<<blocks, kThreads, 0, s>>>(static_cast<float*>(out));
      w = (double)blocks * (kThreads / 64) * kMfmaIter * 4 * (2.0 * 32 * 32 * 64);
      break;
    case MIPQ_PROBE_ADD_VV:
      k_probe_add_vv<<<blocks, kThreads, 0, s>>>(static_cast<float*>(out));
      w = lanes * kIter * kChains;
      break;
    case MIPQ_PROBE_MIN_VV:
      k_probe_min_vv<<<blocks, kThreads, 0, s>>>(static_cast<float*>(out));
      w = lanes * kIter * kChains;
      break;
    case MIPQ_PROBE_MIN3_ADD:
      k_probe_min3_add<<<blocks, kThreads, 0, s>>>(static_cast<float*>(out));
      w = lanes * kIter * kChains;
      break;
    case MIPQ_PROBE_COPY: {
      const int64_t count = (int64_t)(out_bytes / 2 / 16);
      const uint4* src = static_cast<const uint4*>(out);
      k_probe_copy<<<blocks, kThreads, 0, s>>>(src, static_cast<uint4*>(out) + count, count);
      w = 2.0 * 16.0 * (double)count;
      break;
    }
  }
  MIPQ_LAUNCHED("k_probe");
  if (work) *work = w;
  return MIPQ_OK;
}

}  // extern "C"
