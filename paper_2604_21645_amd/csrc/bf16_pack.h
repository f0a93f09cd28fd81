// Centroid-side operands of the matrix-core assignment (shared by the packing
// kernels and, for the layout, by the assignment kernel).
//
// For a subspace with NB 8-dimension blocks, each 32-centroid tile t uses
// NMF = bf16_nmfma(NB) MFMAs of shape 32x32x16 (bfloat16 in, float32 out).
// MFMA f of a tile, lane l (half = l / 32 selects K columns 0-7 or 8-15):
//   f <  NB           : A = [hi_f | lo_f]         B = [xh_f | xh_f]
//   f <  NB+(NB+1)/2  : pair p = f-NB, block b = 2p + half
//                       b < NB: A = hi_b, B = xl_b ; else A = normA, B = normB
//   otherwise         : A = [normA | 0]           B = [normB | 0]
// hi/lo: bfloat16 high and low parts of -2(c - mu); xh/xl: those of (x - mu);
// normA = [c2h, c2m, c2l, 1, 1, 1, 0, 0], normB = [1, 1, 1, x2h, x2m, x2l, 0, 0],
// the pieces summing to ||c - mu||^2 and ||x - mu||^2.  mu is the subspace
// centre: per dimension, the bfloat16-rounded midpoint of the smallest and
// largest centroid coordinate.  Operand slot ((sub*nt + t)*NMF + f)*64 + l
// holds lane l's 8 bfloat16 values of A.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "mipq_internal.h"

namespace mipq {

__device__ __forceinline__ uint16_t bf16_bits_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_bits_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

constexpr uint16_t kBf16One = 0x3F80u;

struct Pack8 {
  uint16_t v[8];
};

__device__ __forceinline__ void store_pack(uint4* dst, const Pack8& p) {
  uint4 q;
  q.x = (uint32_t)p.v[0] | ((uint32_t)p.v[1] << 16);
  q.y = (uint32_t)p.v[2] | ((uint32_t)p.v[3] << 16);
  q.z = (uint32_t)p.v[4] | ((uint32_t)p.v[5] << 16);
  q.w = (uint32_t)p.v[6] | ((uint32_t)p.v[7] << 16);
  *dst = q;
}

// Operand slot f of lane half `half` for centroid ck (its ds float32 values;
// nullptr for a padded centroid) centred by mu; cn: its float64 centred norm.
template <int NB>
__device__ __forceinline__ Pack8 slot_value(const float* ck, const float* mu, int ds, int f, int half, double& cn) {
  constexpr int DW = NB * 8;
  const bool real = ck != nullptr;
  float hv[DW], lv[DW];
  cn = 0.0;
#pragma unroll
  for (int e = 0; e < DW; ++e) {
    const float c = (real && e < ds) ? ck[e] - mu[e] : 0.0f;
    cn += (double)c * (double)c;
    const float v = -2.0f * c;
    hv[e] = bf16_bits_to_f32(bf16_bits_rne(v));
    lv[e] = bf16_bits_to_f32(bf16_bits_rne(v - hv[e]));
  }
  Pack8 norm = {};
  if (real) {
    const uint16_t h = bf16_bits_rne((float)cn);
    const double r1 = cn - (double)bf16_bits_to_f32(h);
    const uint16_t md = bf16_bits_rne((float)r1);
    const double r2 = r1 - (double)bf16_bits_to_f32(md);
    norm.v[0] = h;
    norm.v[1] = md;
    norm.v[2] = bf16_bits_rne((float)r2);
  } else {
    norm.v[0] = 0x7F80u;   // +inf: padded centroids never win
  }
  norm.v[3] = norm.v[4] = norm.v[5] = kBf16One;
  Pack8 out = {};
  auto block_of = [&](const float* src, int b) {
#pragma unroll
    for (int e = 0; e < 8; ++e) out.v[e] = bf16_bits_rne(src[b * 8 + e]);
  };
  if (f < NB) {
    block_of(half ? lv : hv, f);
  } else if (f < NB + (NB + 1) / 2) {
    const int b = 2 * (f - NB) + half;
    if (b < NB) block_of(hv, b);
    else out = norm;
  } else {
    if (!half) out = norm;
  }
  return out;
}

// Block-wide packing of one subspace's tiles [t_begin, t_end).  cb points to
// the subspace's float32 centroids ([ks][ds], global or LDS).  All threads of
// the block must call it (it synchronises).  red must hold 2*16*16 + 16 + 16
// floats of LDS.  With write_stats the block also stores mu (kMaxDsBf16
// floats at mu_out) and the largest centred norm rounded up (*cmax_out).
template <int NB>
__device__ void pack_subspace(const float* cb, int ks, int ds, int nt, int sub, int t_begin, int t_end,
                              uint4* __restrict__ aop, float* __restrict__ cmax_out,
                              float* __restrict__ mu_out, bool write_stats, float* red) {
  constexpr int NMF = bf16_nmfma(NB);
  constexpr int DW = NB * 8;
  const int nthr = blockDim.x;
  const int nw = nthr >> 6;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  float* lo_s = red;              // [16][16]
  float* hi_s = red + 256;        // [16][16]
  float* mu_s = red + 512;        // [16]
  float* mx_s = red + 528;        // [16]
  // centre: per-dimension min and max (exact in any order)
  float lo[DW], hi[DW];
#pragma unroll
  for (int e = 0; e < DW; ++e) {
    lo[e] = INFINITY;
    hi[e] = -INFINITY;
  }
  for (int k = threadIdx.x; k < ks; k += nthr)
#pragma unroll
    for (int e = 0; e < DW; ++e)
      if (e < ds) {
        const float v = cb[k * ds + e];
        lo[e] = fminf(lo[e], v);
        hi[e] = fmaxf(hi[e], v);
      }
#pragma unroll
  for (int e = 0; e < DW; ++e) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      lo[e] = fminf(lo[e], __shfl_xor(lo[e], off, 64));
      hi[e] = fmaxf(hi[e], __shfl_xor(hi[e], off, 64));
    }
    if (lane == 0) {
      lo_s[wv * 16 + e] = lo[e];
      hi_s[wv * 16 + e] = hi[e];
    }
  }
  __syncthreads();
  if (threadIdx.x < DW) {
    const int e = threadIdx.x;
    float a = lo_s[e], b = hi_s[e];
    for (int i = 1; i < nw; ++i) {
      a = fminf(a, lo_s[i * 16 + e]);
      b = fmaxf(b, hi_s[i * 16 + e]);
    }
    const float mu = (e < ds) ? bf16_bits_to_f32(bf16_bits_rne(0.5f * (a + b))) : 0.0f;
    mu_s[e] = mu;
    if (write_stats) mu_out[e] = mu;
  }
  __syncthreads();
  // largest centred norm
  float mx = 0.0f;
  for (int k = threadIdx.x; k < ks; k += nthr) {
    double cn = 0.0;
    for (int e = 0; e < ds; ++e) {
      const double c = (double)(cb[k * ds + e] - mu_s[e]);
      cn += c * c;
    }
    mx = fmaxf(mx, (float)(sqrt(cn) * (1.0 + 1e-6)));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
  if (lane == 0) mx_s[wv] = mx;
  __syncthreads();
  if (write_stats && threadIdx.x == 0) {
    float a = mx_s[0];
    for (int i = 1; i < nw; ++i) a = fmaxf(a, mx_s[i]);
    *cmax_out = a;
  }
  // operand slots
  const int slots = (t_end - t_begin) * NMF * 64;
  for (int s = threadIdx.x; s < slots; s += nthr) {
    const int l = s & 63;
    const int f = (s >> 6) % NMF;
    const int t = t_begin + s / (NMF * 64);
    const int k = t * 32 + (l & 31);
    double cn;
    const Pack8 out = slot_value<NB>(k < ks ? cb + k * ds : nullptr, mu_s, ds, f, l >> 5, cn);
    store_pack(aop + ((size_t)(sub * nt + t) * NMF + f) * 64 + l, out);
  }
}

}  // namespace mipq
