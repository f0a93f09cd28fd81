// Inverted file (paper Section 2.2: row ids stored per bucket for fast lookup;
// buckets here are coarse k-means lists, see the inverted-index reading).
//
//  * coarse assignment: label = argmin_l ||x - c_l||^2 over Kc full-dimension
//    centroids.  Exact rule: float32 differences, squared and summed in
//    float64 in ascending dimension order, lowest index on ties.  Ranked on
//    matrix cores (32x32x16 bfloat16 MFMA, centred operands, squared norms
//    folded into the contraction), each lane keeps its best two candidates;
//    rows whose best two are not separated by the proven error bound are
//    re-decided by the whole wave with the exact rule;
//  * stable counting sort of ids by label (least-significant-digit radix sort,
//    6-bit digits, ranks from wave ballots), list offsets by binary search;
//  * coarse Lloyd update from the sorted order: one block per list sums its
//    rows in id order (float64), so centroids are deterministic;
//  * residuals r = x - c_label (float32) for the residual PQ.
#include <math.h>

#include "bf16_pack.h"
#include "mipq_internal.h"

namespace mipq {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kT = 256;

__device__ __forceinline__ bf16x8 to_bf16x8(const float* v) {
  bf16x8 r;
#pragma unroll
  for (int e = 0; e < 8; e += 2) {
    f32x2 p = {v[e], v[e + 1]};
    bf16x2 q = __builtin_convertvector(p, bf16x2);
    r[e] = q[0];
    r[e + 1] = q[1];
  }
  return r;
}

// ---------------------------------------------------------------- centre
// mu[t] = bfloat16-rounded midpoint of min and max of centroid coordinate t;
// one block per dimension.  Also clears the norm bound cell.
__global__ __launch_bounds__(kT) void k_coarse_centre(const float* __restrict__ cc, int kc, int d,
                                                      float* __restrict__ mu, unsigned int* __restrict__ cmax_bits) {
  __shared__ float lo_s[kT / 64], hi_s[kT / 64];
  const int t = blockIdx.x;
  float lo = INFINITY, hi = -INFINITY;
  for (int l = threadIdx.x; l < kc; l += blockDim.x) {
    const float v = cc[(int64_t)l * d + t];
    lo = fminf(lo, v);
    hi = fmaxf(hi, v);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    lo = fminf(lo, __shfl_xor(lo, off, 64));
    hi = fmaxf(hi, __shfl_xor(hi, off, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    lo_s[threadIdx.x >> 6] = lo;
    hi_s[threadIdx.x >> 6] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) {
      lo = fminf(lo, lo_s[i]);
      hi = fmaxf(hi, hi_s[i]);
    }
    lo = fminf(lo, lo_s[0]);
    hi = fmaxf(hi, hi_s[0]);
    mu[t] = bf16_bits_to_f32(bf16_bits_rne(0.5f * (lo + hi)));
    if (t == 0) *cmax_bits = 0u;
  }
}

// ---------------------------------------------------------------- packing
// Operand slot ((t*NK + s)*64 + l) = lane l's 8 bfloat16 values of A for tile t
// (32 centroids), K-step s: s < S: bf16(-2(c - mu)) of dimensions 16s + 8h ..
// +7 (h = l/32, zero past d); s = S: [c2h, c2m, c2l, 1, 1, 1, 0, 0] for h = 0
// (||c - mu||^2 in three pieces), zeros for h = 1.  Padded centroids get
// c2h = +inf.  Also the largest centred norm (float bits, atomic max).
__global__ __launch_bounds__(kT) void k_coarse_pack(const float* __restrict__ cc, int kc, int d, int S,
                                                    const float* __restrict__ mu, uint4* __restrict__ aop,
                                                    unsigned int* __restrict__ cmax_bits) {
  const int NK = S + 1;
  const int nt = (kc + 31) / 32;
  const int total = nt * NK * 64;
  for (int slot = blockIdx.x * blockDim.x + threadIdx.x; slot < total; slot += gridDim.x * blockDim.x) {
    const int l = slot & 63;
    const int s = (slot >> 6) % NK;
    const int t = slot / (NK * 64);
    const int i = l & 31, h = l >> 5;
    const int k = t * 32 + i;
    const bool real = k < kc;
    Pack8 out = {};
    if (s < S) {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int dim = 16 * s + 8 * h + e;
        const float c = (real && dim < d) ? cc[(int64_t)k * d + dim] - mu[dim] : 0.0f;
        out.v[e] = bf16_bits_rne(-2.0f * c);
      }
    } else if (h == 0) {
      if (real) {
        double cn = 0.0;
        for (int dim = 0; dim < d; ++dim) {
          const double c = (double)(cc[(int64_t)k * d + dim] - mu[dim]);
          cn += c * c;
        }
        const uint16_t hb = bf16_bits_rne((float)cn);
        const double r1 = cn - (double)bf16_bits_to_f32(hb);
        const uint16_t mb = bf16_bits_rne((float)r1);
        const double r2 = r1 - (double)bf16_bits_to_f32(mb);
        out.v[0] = hb;
        out.v[1] = mb;
        out.v[2] = bf16_bits_rne((float)r2);
        const float nrm = (float)(sqrt(cn) * (1.0 + 1e-6));
        atomicMax(cmax_bits, __float_as_uint(nrm));
      } else {
        out.v[0] = 0x7F80u;
      }
      out.v[3] = out.v[4] = out.v[5] = kBf16One;
    }
    store_pack(aop + slot, out);
  }
}

// ---------------------------------------------------------------- exact rule
// float32 differences, float64 squares and sums in ascending dimension order
// (rows of 16-float multiples at 16-byte alignment are read 16 floats at a
// time, the next 16 in flight; the order of the sum is the same)
__device__ __forceinline__ double coarse_exact_dist(const float* __restrict__ xr, const float* __restrict__ c, int d) {
  double acc = 0.0;
  if ((d & 15) == 0 && ((reinterpret_cast<uintptr_t>(xr) | reinterpret_cast<uintptr_t>(c)) & 15) == 0) {
    const float4* x4 = reinterpret_cast<const float4*>(xr);
    const float4* c4 = reinterpret_cast<const float4*>(c);
    const int nch = d >> 4;
    float4 xc[4], cc4[4], xn[4], cn[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      xc[k] = x4[k];
      cc4[k] = c4[k];
    }
    for (int ch = 0; ch < nch; ++ch) {
      if (ch + 1 < nch) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          xn[k] = x4[(ch + 1) * 4 + k];
          cn[k] = c4[(ch + 1) * 4 + k];
        }
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float xv[4] = {xc[k].x, xc[k].y, xc[k].z, xc[k].w};
        const float cv[4] = {cc4[k].x, cc4[k].y, cc4[k].z, cc4[k].w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const double df = (double)(xv[i] - cv[i]);
          acc = acc + df * df;
        }
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        xc[k] = xn[k];
        cc4[k] = cn[k];
      }
    }
    return acc;
  }
  for (int t = 0; t < d; ++t) {
    const double df = (double)(xr[t] - c[t]);
    acc = acc + df * df;
  }
  return acc;
}

// whole wave: lane i scans centroids i, i+64, ...; lexicographic minimum
__device__ int coarse_exact_wave(const float* __restrict__ xr, const float* __restrict__ cc, int kc, int d,
                                 int lane) {
  double best = INFINITY;
  int bk = 0x7FFFFFFF;
  for (int k = lane; k < kc; k += 64) {
    const double dk = coarse_exact_dist(xr, cc + (int64_t)k * d, d);
    if (dk < best) {
      best = dk;
      bk = k;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double ob = __shfl_xor(best, off, 64);
    const int ok = __shfl_xor(bk, off, 64);
    if (ob < best || (ob == best && ok < bk)) {
      best = ob;
      bk = ok;
    }
  }
  return bk < kc ? bk : 0;
}

// One lane per row, plain exact rule (small problems and reference).
__global__ __launch_bounds__(kT) void k_coarse_assign_exact(const float* __restrict__ x, int64_t n, int d,
                                                            const float* __restrict__ cc, int kc,
                                                            int32_t* __restrict__ labels) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= n) return;
  const float* xr = x + row * d;
  double best = INFINITY;
  int bk = 0;
  for (int k = 0; k < kc; ++k) {
    const double dk = coarse_exact_dist(xr, cc + (int64_t)k * d, d);
    if (dk < best) {
      best = dk;
      bk = k;
    }
  }
  labels[row] = bk;
}

// ---------------------------------------------------------------- MFMA assign
// One wave = RG groups of 32 rows; lane l holds row l%32 of each group and the
// dimensions 16s + 8h .. +7 (h = l/32) of every K-step s.  For each
// 32-centroid tile the wave loads the tile's S+1 operands once and runs S+1
// MFMAs per row group; lane l receives 16 distance estimates of its row
// (centroids 8(r/4) + 4h + r%4 of the tile) and keeps its best two and the
// best index.
//
// A row whose best two estimates are not separated by the proven bound is
// ambiguous.  The wave then recomputes the estimates of its row groups that
// hold ambiguous rows, collects every (row, centroid) whose estimate is within
// the bound of the row's best (the exact winner is always among them) in an
// LDS list, and decides each such row by the exact rule over its candidates
// only.  Rows whose candidates do not fit the list are decided by the exact
// rule over all centroids.
constexpr int kCandCap = 256;   // candidate pairs per wave

// (registers capped for three waves per SIMD: at d = 128 the two waves the
// uncapped kernel allowed took 35 ms on 10M rows x Kc = 4096, three 30 ms)
template <int S, int RG>
__global__ __launch_bounds__(kT, 3) void k_coarse_assign_mfma(
    const float* __restrict__ x, int64_t n, int d, int kc, const bf16x8* __restrict__ aop,
    const float* __restrict__ mu, const unsigned int* __restrict__ cmax_bits, const float* __restrict__ cc,
    int32_t* __restrict__ labels, unsigned long long* __restrict__ rescored, float e_cross, float e_norm,
    float g_exact) {
  constexpr int NK = S + 1;
  __shared__ uint32_t cand_rk_all[kT / 64][kCandCap];   // (row in wave) << 16 | centroid
  __shared__ double cand_d_all[kT / 64][kCandCap];
  __shared__ bf16x8 a_lds[2][NK * 64];
  const int lane = threadIdx.x & 63;
  const int h = lane >> 5;
  const int w = threadIdx.x >> 6;
  const int64_t r0 = ((int64_t)blockIdx.x * (kT / 64) + w) * (32 * RG);
  // waves past the last row still stage operands and meet the block's
  // barriers; their rows read row n - 1 and write nothing
  uint32_t* cand_rk = cand_rk_all[w];
  double* cand_d = cand_d_all[w];
  const float cm = __uint_as_float(*cmax_bits);
  // every row slice is whole and 16-byte aligned (mu is a workspace buffer)
  const bool vec = d == 16 * S && (reinterpret_cast<uintptr_t>(x) & 15) == 0 &&
                   (reinterpret_cast<uintptr_t>(mu) & 15) == 0;

  // row operands (centred), ||x - mu||^2
  bf16x8 B[RG][NK];
  float xn[RG];
#pragma unroll
  for (int g = 0; g < RG; ++g) {
    const int64_t row = r0 + 32 * g + (lane & 31);
    const float* xr = x + (row < n ? row : n - 1) * d;
    float xn_part = 0.0f;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      float v[8];
      if (vec) {   // the 8 dimensions 16 s + 8 h .. + 7 as two float4
        const float4 xa = *reinterpret_cast<const float4*>(xr + 16 * s + 8 * h);
        const float4 xb = *reinterpret_cast<const float4*>(xr + 16 * s + 8 * h + 4);
        const float4 ma = *reinterpret_cast<const float4*>(mu + 16 * s + 8 * h);
        const float4 mb = *reinterpret_cast<const float4*>(mu + 16 * s + 8 * h + 4);
        const float xs[8] = {xa.x, xa.y, xa.z, xa.w, xb.x, xb.y, xb.z, xb.w};
        const float ms[8] = {ma.x, ma.y, ma.z, ma.w, mb.x, mb.y, mb.z, mb.w};
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          v[e] = xs[e] - ms[e];
          xn_part = xn_part + v[e] * v[e];
        }
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int dim = 16 * s + 8 * h + e;
          const float xv = xr[dim < d ? dim : d - 1];
          v[e] = dim < d ? xv - mu[dim] : 0.0f;
          xn_part = xn_part + v[e] * v[e];
        }
      }
      B[g][s] = to_bf16x8(v);
    }
    const auto sw = __builtin_amdgcn_permlane32_swap(__float_as_int(xn_part), __float_as_int(xn_part), false, false);
    xn[g] = __int_as_float((int)sw[0]) + __int_as_float((int)sw[1]);
    bf16x8 nb = {};
    if (h == 0) {
      const __bf16 hb = (__bf16)xn[g];
      const float r1 = xn[g] - (float)hb;
      const __bf16 mb = (__bf16)r1;
      nb[0] = nb[1] = nb[2] = (__bf16)1.0f;
      nb[3] = hb;
      nb[4] = mb;
      nb[5] = (__bf16)(r1 - (float)mb);
    }
    B[g][S] = nb;
  }

  float v1[RG], v2[RG];
  int i1[RG];
#pragma unroll
  for (int g = 0; g < RG; ++g) {
    v1[g] = INFINITY;
    v2[g] = INFINITY;
    i1[g] = 0;
  }
  const int nt = (kc + 31) / 32;
  // centroid operands of a tile: staged in LDS once for the block's four
  // waves (two buffers); the next tile's chunks are loaded into registers
  // while the current tile is scored, and stored after it
  constexpr int CH = NK * 64;               // 16-byte operand chunks per tile
  constexpr int PT = (CH + kT - 1) / kT;    // chunks per thread
  bf16x8 pre[PT];
  auto fetch = [&](int t) {
#pragma unroll
    for (int i = 0; i < PT; ++i) {
      const int c = threadIdx.x + i * kT;
      if (c < CH) pre[i] = aop[(size_t)t * CH + c];
    }
  };
  auto put = [&](int buf) {
#pragma unroll
    for (int i = 0; i < PT; ++i) {
      const int c = threadIdx.x + i * kT;
      if (c < CH) a_lds[buf][c] = pre[i];
    }
  };
  fetch(0);
  put(0);
  __syncthreads();
  for (int t = 0; t < nt; ++t) {
    const int cur = t & 1;
    if (t + 1 < nt) fetch(t + 1);
#pragma unroll
    for (int g = 0; g < RG; ++g) {
      f32x16 acc = {};
#pragma unroll
      for (int s = 0; s < NK; ++s)
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_lds[cur][s * 64 + lane], B[g][s], acc, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float v = acc[r];
        const int k = t * 32 + (r >> 2) * 8 + h * 4 + (r & 3);
        v2[g] = __builtin_amdgcn_fmed3f(v1[g], v2[g], v);   // runner-up of {v1, v2, v}, v1 <= v2
        const bool lt = v < v1[g];
        i1[g] = lt ? k : i1[g];
        v1[g] = lt ? v : v1[g];
      }
    }
    if (t + 1 < nt) put(cur ^ 1);
    __syncthreads();
  }

  // merge the two lanes of each row; separation test
  float f1[RG], beta[RG];
  bool amb[RG];
  uint64_t any_amb = 0;
#pragma unroll
  for (int g = 0; g < RG; ++g) {
    const auto a = __builtin_amdgcn_permlane32_swap(__float_as_int(v1[g]), __float_as_int(v1[g]), false, false);
    const auto b = __builtin_amdgcn_permlane32_swap(__float_as_int(v2[g]), __float_as_int(v2[g]), false, false);
    const auto c = __builtin_amdgcn_permlane32_swap(i1[g], i1[g], false, false);
    const float v1l = __int_as_float((int)a[0]), v1h = __int_as_float((int)a[1]);
    const float v2l = __int_as_float((int)b[0]), v2h = __int_as_float((int)b[1]);
    const int i1l = (int)c[0], i1h = (int)c[1];
    const bool hiw = (v1h < v1l) || (v1h == v1l && i1h < i1l);
    f1[g] = fminf(v1l, v1h);
    const float f2 = fminf(fmaxf(v1l, v1h), fminf(v2l, v2h));
    const int code = hiw ? i1h : i1l;
    beta[g] = e_cross * sqrtf(xn[g]) * 1.0001f * cm + e_norm * (cm * cm + xn[g]);
    const float gap = f2 - f1[g];
    const float thr = 2.0f * beta[g] + g_exact * (fabsf(f1[g]) + fabsf(f2) + 2.0f * beta[g] + 2.0f * xn[g] * g_exact);
    const int64_t row = r0 + 32 * g + (lane & 31);
    const bool valid = row < n;
    amb[g] = valid && (!(gap > thr) || code >= kc);
    if (h == 0 && valid) labels[row] = code;
    any_amb |= __ballot(h == 0 && amb[g]);
    if (rescored && lane == 0) {
      const int c2 = __popcll(__ballot(h == 0 && amb[g]));
      if (c2) atomicAdd(rescored, (unsigned long long)c2);
    }
  }
  if (!any_amb) return;

  // candidates of the ambiguous rows: est_k - f1 within the bound
  int nc = 0;
  bool ovf[RG];
#pragma unroll
  for (int g = 0; g < RG; ++g) ovf[g] = false;
  uint64_t gmask = 0;
#pragma unroll
  for (int g = 0; g < RG; ++g)
    if (__ballot(amb[g])) gmask |= 1ull << g;
  for (int t = 0; t < nt; ++t) {
    bf16x8 A[NK];
#pragma unroll
    for (int s = 0; s < NK; ++s) A[s] = aop[((size_t)t * NK + s) * 64 + lane];
#pragma unroll
    for (int g = 0; g < RG; ++g) {
      if (!((gmask >> g) & 1)) continue;   // wave-uniform
      f32x16 acc = {};
#pragma unroll
      for (int s = 0; s < NK; ++s) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[s], B[g][s], acc, 0, 0, 0);
      uint32_t mine = 0;   // bit r: candidate in accumulator register r
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float v = acc[r];
        const int k = t * 32 + (r >> 2) * 8 + h * 4 + (r & 3);
        const float lim = 2.0f * beta[g] + g_exact * (fabsf(f1[g]) + fabsf(v) + 2.0f * beta[g] +
                                                      2.0f * xn[g] * g_exact);
        const bool cand = amb[g] && k < kc && !(v - f1[g] > lim);
        mine |= cand ? (1u << r) : 0u;
      }
      if (!__ballot(mine != 0)) continue;
      const uint32_t rl = (uint32_t)(32 * g + (lane & 31)) << 16;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const bool cand = (mine >> r) & 1u;
        const uint64_t m = __ballot(cand);
        if (!m) continue;
        if (cand) {
          const int pos = nc + __popcll(m & ((1ull << lane) - 1ull));
          const int k = t * 32 + (r >> 2) * 8 + h * 4 + (r & 3);
          if (pos < kCandCap) cand_rk[pos] = rl | (uint32_t)k;
          else ovf[g] = true;
        }
        nc += __popcll(m);
      }
    }
  }
  const int ncl = nc < kCandCap ? nc : kCandCap;
  __builtin_amdgcn_wave_barrier();
  for (int i = lane; i < ncl; i += 64) {
    const uint32_t rk = cand_rk[i];
    const int64_t row = r0 + (rk >> 16);
    cand_d[i] = coarse_exact_dist(x + row * d, cc + (int64_t)(rk & 0xFFFFu) * d, d);
  }
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int g = 0; g < RG; ++g) {
    // a row overflowed when either of its two lanes dropped a candidate
    const uint64_t ob = __ballot(ovf[g]);
    const uint32_t rows_full = (uint32_t)(ob | (ob >> 32));
    const int64_t row = r0 + 32 * g + (lane & 31);
    if (h == 0 && amb[g] && !((rows_full >> (lane & 31)) & 1u)) {
      const uint32_t rl = (uint32_t)(32 * g + (lane & 31));
      double best = INFINITY;
      int bk = 0x7FFFFFFF;
      for (int i = 0; i < ncl; ++i) {
        const uint32_t rk = cand_rk[i];
        if ((rk >> 16) != rl) continue;
        const double dv = cand_d[i];
        const int k = (int)(rk & 0xFFFFu);
        if (dv < best || (dv == best && k < bk)) {
          best = dv;
          bk = k;
        }
      }
      labels[row] = bk;
    }
    uint32_t fm = rows_full & (uint32_t)__ballot(h == 0 && amb[g]);
    while (fm) {   // wave-uniform
      const int l = __ffs(fm) - 1;
      fm &= fm - 1;
      const int ec = coarse_exact_wave(x + (r0 + 32 * g + l) * d, cc, kc, d, lane);
      if (lane == 0) labels[r0 + 32 * g + l] = ec;
    }
  }
}

// ---------------------------------------------------------------- radix sort
// Stable LSD radix sort of (key, value) by key, 6-bit digits.  Tile = kRsTile
// consecutive elements per block; a round = 64 elements per wave, waves in
// element order.
constexpr int kRsBits = 6;
constexpr int kRsBuckets = 1 << kRsBits;
constexpr int kRsTile = 4096;

__global__ __launch_bounds__(kT) void k_rs_hist(const uint32_t* __restrict__ keys, int64_t n, int shift,
                                                uint32_t* __restrict__ hist, int nblk) {
  __shared__ uint32_t cnt[kRsBuckets];
  if (threadIdx.x < kRsBuckets) cnt[threadIdx.x] = 0u;
  __syncthreads();
  const int64_t b0 = (int64_t)blockIdx.x * kRsTile;
  const int64_t b1 = min(n, b0 + kRsTile);
  for (int64_t i = b0 + threadIdx.x; i < b1; i += blockDim.x)
    atomicAdd(&cnt[(keys[i] >> shift) & (kRsBuckets - 1)], 1u);
  __syncthreads();
  if (threadIdx.x < kRsBuckets) hist[(size_t)threadIdx.x * nblk + blockIdx.x] = cnt[threadIdx.x];
}

// exclusive scan of hist (bucket-major) in place, one block of kT threads
__global__ __launch_bounds__(kT) void k_rs_scan(uint32_t* __restrict__ hist, int total) {
  __shared__ uint32_t part[kT];
  const int per = (total + kT - 1) / kT;
  const int s0 = threadIdx.x * per;
  uint32_t run = 0;
  for (int i = 0; i < per; ++i)
    if (s0 + i < total) run += hist[s0 + i];
  part[threadIdx.x] = run;
  __syncthreads();
  for (int off = 1; off < kT; off <<= 1) {
    const uint32_t v = (int)threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  uint32_t acc = part[threadIdx.x] - run;
  for (int i = 0; i < per; ++i)
    if (s0 + i < total) {
      const uint32_t c = hist[s0 + i];
      hist[s0 + i] = acc;
      acc += c;
    }
}

// scatter in element order; vals_in == NULL means value = element index
__global__ __launch_bounds__(kT) void k_rs_scatter(const uint32_t* __restrict__ keys_in,
                                                   const int32_t* __restrict__ vals_in, int64_t n, int shift,
                                                   const uint32_t* __restrict__ offs, int nblk,
                                                   uint32_t* __restrict__ keys_out, int32_t* __restrict__ vals_out) {
  __shared__ uint32_t base[kRsBuckets];
  __shared__ uint32_t wcnt[kT / 64][kRsBuckets];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  if (threadIdx.x < kRsBuckets) base[threadIdx.x] = offs[(size_t)threadIdx.x * nblk + blockIdx.x];
  const int64_t b0 = (int64_t)blockIdx.x * kRsTile;
  const int64_t b1 = min(n, b0 + kRsTile);
  const uint64_t below = (1ull << lane) - 1ull;
  for (int64_t r0 = b0; r0 < b1; r0 += (int64_t)nw * 64) {
    const int64_t i = r0 + (int64_t)w * 64 + lane;
    const bool ok = i < b1;
    const uint32_t key = ok ? keys_in[i] : 0u;
    const int32_t val = ok ? (vals_in ? vals_in[i] : (int32_t)i) : 0;
    const int dig = ok ? (int)((key >> shift) & (kRsBuckets - 1)) : -1;
    int rank = 0;
    for (int b = 0; b < kRsBuckets; ++b) {
      const uint64_t m = __ballot(dig == b);
      if (dig == b) rank = __popcll(m & below);
      if (lane == b) wcnt[w][b] = (uint32_t)__popcll(m);
    }
    __syncthreads();
    if (ok) {
      uint32_t pos = base[dig] + (uint32_t)rank;
      for (int ww = 0; ww < w; ++ww) pos += wcnt[ww][dig];
      keys_out[pos] = key;
      vals_out[pos] = val;
    }
    __syncthreads();
    if (threadIdx.x < kRsBuckets) {
      uint32_t add = 0;
      for (int ww = 0; ww < nw; ++ww) add += wcnt[ww][threadIdx.x];
      base[threadIdx.x] += add;
    }
    __syncthreads();
  }
}

// offsets[l] = first position whose sorted key is >= l, l = 0..kc
__global__ __launch_bounds__(kT) void k_list_offsets(const uint32_t* __restrict__ sorted_keys, int64_t n, int kc,
                                                     int64_t* __restrict__ offsets) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l > kc) return;
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (sorted_keys[mid] < (uint32_t)l) lo = mid + 1;
    else hi = mid;
  }
  offsets[l] = lo;
}

// ---------------------------------------------------------------- coarse update
// One block per list: float64 sums of its rows in id order (thread t owns
// dimensions t, t+blockDim, ...); centroid = sum / count (empty keeps its
// value); also the list's objective sum of (x - c_old)^2 in float64.
__global__ __launch_bounds__(kT) void k_coarse_update(const float* __restrict__ x, int d,
                                                      const int32_t* __restrict__ ids,
                                                      const int64_t* __restrict__ offsets,
                                                      float* __restrict__ cc, double* __restrict__ cc64,
                                                      double* __restrict__ obj_list) {
  __shared__ double red[kT / 64];
  const int l = blockIdx.x;
  const int64_t a = offsets[l], b = offsets[l + 1];
  double jl = 0.0;
  for (int t = threadIdx.x; t < d; t += blockDim.x) {
    const float cold = cc[(int64_t)l * d + t];
    double s = 0.0;
    for (int64_t p = a; p < b; ++p) {
      const float xv = x[(int64_t)ids[p] * d + t];
      s += (double)xv;
      const double df = (double)xv - (double)cold;
      jl += df * df;
    }
    if (b > a) {
      const double v = s / (double)(b - a);
      cc64[(int64_t)l * d + t] = v;
      cc[(int64_t)l * d + t] = (float)v;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) jl += __shfl_xor(jl, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = jl;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
    obj_list[l] = s;
  }
}

// objective of a round: fixed pairwise tree over the lists, one block
__global__ __launch_bounds__(kT) void k_sum_lists(const double* __restrict__ v, int k, double* __restrict__ out) {
  __shared__ double red[kT];
  double s = 0.0;
  for (int i = threadIdx.x; i < k; i += blockDim.x) s += v[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

__global__ void k_gather_coarse(const float* __restrict__ x, int64_t n, int d, const int64_t* __restrict__ rows,
                                int kc, float* __restrict__ cc, double* __restrict__ cc64) {
  const int64_t total = (int64_t)kc * d;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t l = i / d;
    const int t = int(i - l * d);
    const int64_t r = rows[l];
    const float v = (r >= 0 && r < n) ? x[r * d + t] : NAN;
    cc[i] = v;
    cc64[i] = (double)v;
  }
}

// r = x - c_label, float32
// r = x - c_label, float32.  Block-stride over rows, the block's threads over
// the row's elements (16-byte accesses when d % 4 == 0).
__global__ void k_residuals(const float* __restrict__ x, int64_t n, int d, const int32_t* __restrict__ labels,
                            const float* __restrict__ cc, int kc, float* __restrict__ r, int vec4) {
  const int per = vec4 ? d / 4 : d;
  const int rpb = blockDim.x / per > 0 ? blockDim.x / per : 1;   // rows per block step
  const int lr = threadIdx.x / per;
  for (int64_t row0 = (int64_t)blockIdx.x * rpb; row0 < n; row0 += (int64_t)gridDim.x * rpb) {
    const int64_t row = row0 + lr;
    if (lr >= rpb || row >= n) continue;
    const int l = labels[row];
    const bool ok = l >= 0 && l < kc;
    const float* c = cc + (int64_t)(ok ? l : 0) * d;
    for (int e = threadIdx.x - lr * per; e < per; e += (per > (int)blockDim.x ? blockDim.x : per)) {
      if (vec4) {
        const float4 a = reinterpret_cast<const float4*>(x + row * d)[e];
        const float4 b = reinterpret_cast<const float4*>(c)[e];
        reinterpret_cast<float4*>(r + row * d)[e] =
            ok ? make_float4(a.x - b.x, a.y - b.y, a.z - b.z, a.w - b.w) : make_float4(NAN, NAN, NAN, NAN);
      } else {
        r[row * d + e] = ok ? x[row * d + e] - c[e] : NAN;
      }
    }
  }
}

// codes_sorted[i] = codes[ids[i]] (m bytes per row); one thread per row
__global__ void k_gather_codes(const uint8_t* __restrict__ codes, int64_t n, int m, const int32_t* __restrict__ ids,
                               uint8_t* __restrict__ out, int vec16) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint8_t* src = codes + (int64_t)ids[i] * m;
    uint8_t* dst = out + i * m;
    if (vec16) {
      for (int j = 0; j < m; j += 16) *reinterpret_cast<uint4*>(dst + j) = *reinterpret_cast<const uint4*>(src + j);
    } else {
      for (int j = 0; j < m; ++j) dst[j] = src[j];
    }
  }
}

// ---------------------------------------------------------------- list merge
// Merge of inverted lists built over consecutive row ranges ("parts"): list l
// of the result is the concatenation, in part order, of list l of every
// part, ids shifted by the part's first row.  Ids ascend inside every part's
// list and the parts cover increasing row ranges, so merged lists ascend.
struct MergePart {
  const int64_t* off;
  const int32_t* ids;
  const uint8_t* codes;
  int64_t n;
  int64_t base;   // first row of the part
};

// thread per list: rows of list l in the parts before p (pre[p*kc + l]) and in all
__global__ void k_merge_prefix(const MergePart* __restrict__ parts, int nparts, int kc, int64_t* __restrict__ pre,
                               int64_t* __restrict__ total) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= kc) return;
  int64_t acc = 0;
  for (int p = 0; p < nparts; ++p) {
    pre[(size_t)p * kc + l] = acc;
    acc += parts[p].off[l + 1] - parts[p].off[l];
  }
  total[l] = acc;
}

// exclusive scan of total[0..kc) into offsets[0..kc], one block
__global__ __launch_bounds__(kT) void k_merge_scan(const int64_t* __restrict__ total, int kc,
                                                   int64_t* __restrict__ offsets) {
  __shared__ int64_t part[kT];
  const int per = (kc + kT - 1) / kT;
  const int s0 = threadIdx.x * per;
  int64_t run = 0;
  for (int i = 0; i < per; ++i)
    if (s0 + i < kc) run += total[s0 + i];
  part[threadIdx.x] = run;
  __syncthreads();
  for (int off = 1; off < kT; off <<= 1) {
    const int64_t v = (int)threadIdx.x >= off ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  int64_t acc = part[threadIdx.x] - run;
  for (int i = 0; i < per; ++i)
    if (s0 + i < kc) {
      offsets[s0 + i] = acc;
      acc += total[s0 + i];
    }
  if (threadIdx.x == kT - 1) offsets[kc] = part[kT - 1];
}

// thread per row of all parts: its list by binary search in the part's offsets
__global__ void k_merge_copy(const MergePart* __restrict__ parts, int nparts, int64_t total_rows, int kc, int m,
                             const int64_t* __restrict__ pre, const int64_t* __restrict__ offsets,
                             int32_t* __restrict__ ids, uint8_t* __restrict__ codes, int vec16) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total_rows;
       g += (int64_t)gridDim.x * blockDim.x) {
    int lo = 0, hi = nparts - 1;
    while (lo < hi) {   // last part with base <= g
      const int mid = (lo + hi + 1) >> 1;
      if (parts[mid].base <= g) lo = mid;
      else hi = mid - 1;
    }
    const MergePart& P = parts[lo];
    const int64_t i = g - P.base;
    int a = 0, b = kc - 1;
    while (a < b) {   // last list l with off[l] <= i
      const int mid = (a + b + 1) >> 1;
      if (P.off[mid] <= i) a = mid;
      else b = mid - 1;
    }
    const int64_t dst = offsets[a] + pre[(size_t)lo * kc + a] + (i - P.off[a]);
    ids[dst] = (int32_t)(P.ids[i] + P.base);
    const uint8_t* src = P.codes + i * m;
    uint8_t* out = codes + dst * m;
    if (vec16) {
      for (int j = 0; j < m; j += 16) *reinterpret_cast<uint4*>(out + j) = *reinterpret_cast<const uint4*>(src + j);
    } else {
      for (int j = 0; j < m; ++j) out[j] = src[j];
    }
  }
}

int grid_cap(int64_t work, int cap) {
  int64_t g = (work + kT - 1) / kT;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return int(g);
}

}  // namespace

// ---------------------------------------------------------------- host side
int coarse_ksteps(int d) { return (d + 15) / 16; }

size_t coarse_operand_count(int kc, int d) { return (size_t)((kc + 31) / 32) * (coarse_ksteps(d) + 1) * 64; }

int launch_coarse_prepare(const float* cc, int kc, int d, float* mu, unsigned int* cmax_bits, void* aop,
                          hipStream_t s) {
  ProfScope ps(MIPQ_K_COARSE_PACK, s);
  k_coarse_centre<<<d, kT, 0, s>>>(cc, kc, d, mu, cmax_bits);
  MIPQ_LAUNCHED("k_coarse_centre");
  const int S = coarse_ksteps(d);
  k_coarse_pack<<<grid_cap((int64_t)coarse_operand_count(kc, d), 4096), kT, 0, s>>>(cc, kc, d, S, mu,
                                                                                    (uint4*)aop, cmax_bits);
  MIPQ_LAUNCHED("k_coarse_pack");
  return MIPQ_OK;
}

int launch_coarse_assign(const float* x, int64_t n, int d, const float* cc, int kc, const void* aop,
                         const float* mu, const unsigned int* cmax_bits, int32_t* labels, int64_t* rescored,
                         bool exact_only, hipStream_t s) {
  if (n == 0) return MIPQ_OK;
  ProfScope ps(MIPQ_K_COARSE_ASSIGN, s);
  if (exact_only) {
    k_coarse_assign_exact<<<ceil_div(n, kT), kT, 0, s>>>(x, n, d, cc, kc, labels);
    MIPQ_LAUNCHED("k_coarse_assign_exact");
    return MIPQ_OK;
  }
  const int S = coarse_ksteps(d);
  // error bound: single bfloat16 products 2(2u + u^2) with u = 2^-8, twice for
  // the -2 factor, float32 accumulation over 16(S+1) terms at 2^-23 each, the
  // norm pieces and the centring; g_exact: float32 differences squared (2^-23)
  const float e_cross = 0.0165f;
  const float e_norm = 16.0f * (S + 1) * 1.2e-7f + 2.4e-7f;
  const float g_exact = 1.3e-7f;
  unsigned long long* resc = reinterpret_cast<unsigned long long*>(rescored);
  // two row groups per wave (operands loaded once per tile for 64 rows) while
  // the row operands fit the registers
#define CA(SV)                                                                                                  \
  do {                                                                                                          \
    constexpr int RGV = SV <= 8 ? 2 : 1;                                                                        \
    const int blocks = ceil_div((n + 32 * RGV - 1) / (32 * RGV), kT / 64);                                      \
    k_coarse_assign_mfma<SV, RGV><<<blocks, kT, 0, s>>>(x, n, d, kc, (const bf16x8*)aop, mu, cmax_bits, cc,     \
                                                        labels, resc, e_cross, e_norm, g_exact);                \
  } while (0)
  switch (S) {
    case 1: CA(1); break;
    case 2: CA(2); break;
    case 4: CA(4); break;
    case 6: CA(6); break;
    case 8: CA(8); break;
    case 12: CA(12); break;
    case 16: CA(16); break;
    default: return fail(MIPQ_EUNSUPPORTED, "coarse matrix-core path supports d in {<=16, 32, 64, 96, 128, 192, 256} (got %d)", d);
  }
#undef CA
  MIPQ_LAUNCHED("k_coarse_assign_mfma");
  return MIPQ_OK;
}

int sort_blocks(int64_t n) { return n > 0 ? ceil_div(n, kRsTile) : 1; }

int launch_sort_by_label(const int32_t* labels, int64_t n, int kc, uint32_t* keys_a, uint32_t* keys_b,
                         int32_t* vals_a, int32_t* vals_b, uint32_t* hist, int32_t* ids_out,
                         uint32_t* keys_out_sorted, int64_t* offsets, hipStream_t s) {
  ProfScope ps(MIPQ_K_SORT, s);
  const int nblk = sort_blocks(n);
  int bits = 1;
  while ((1 << bits) < kc) ++bits;
  const int passes = (bits + kRsBits - 1) / kRsBits;
  const uint32_t* kin = reinterpret_cast<const uint32_t*>(labels);
  const int32_t* vin = nullptr;
  for (int p = 0; p < passes; ++p) {
    const bool last = p == passes - 1;
    uint32_t* kout = last ? keys_out_sorted : (p % 2 == 0 ? keys_a : keys_b);
    int32_t* vout = last ? ids_out : (p % 2 == 0 ? vals_a : vals_b);
    if (n > 0) {
      k_rs_hist<<<nblk, kT, 0, s>>>(kin, n, p * kRsBits, hist, nblk);
      MIPQ_LAUNCHED("k_rs_hist");
      k_rs_scan<<<1, kT, 0, s>>>(hist, kRsBuckets * nblk);
      MIPQ_LAUNCHED("k_rs_scan");
      k_rs_scatter<<<nblk, kT, 0, s>>>(kin, vin, n, p * kRsBits, hist, nblk, kout, vout);
      MIPQ_LAUNCHED("k_rs_scatter");
    }
    kin = kout;
    vin = vout;
  }
  k_list_offsets<<<ceil_div(kc + 1, kT), kT, 0, s>>>(keys_out_sorted, n, kc, offsets);
  MIPQ_LAUNCHED("k_list_offsets");
  return MIPQ_OK;
}

int launch_coarse_update(const float* x, int d, const int32_t* ids, const int64_t* offsets, int kc, float* cc,
                         double* cc64, double* obj_list, double* obj_out, hipStream_t s) {
  ProfScope ps(MIPQ_K_COARSE_UPDATE, s);
  k_coarse_update<<<kc, d >= kT ? kT : (d >= 128 ? 128 : 64), 0, s>>>(x, d, ids, offsets, cc, cc64, obj_list);
  MIPQ_LAUNCHED("k_coarse_update");
  if (obj_out) {
    k_sum_lists<<<1, kT, 0, s>>>(obj_list, kc, obj_out);
    MIPQ_LAUNCHED("k_sum_lists");
  }
  return MIPQ_OK;
}

int launch_gather_coarse(const float* x, int64_t n, int d, const int64_t* rows, int kc, float* cc, double* cc64,
                         hipStream_t s) {
  k_gather_coarse<<<grid_cap((int64_t)kc * d, 4096), kT, 0, s>>>(x, n, d, rows, kc, cc, cc64);
  MIPQ_LAUNCHED("k_gather_coarse");
  return MIPQ_OK;
}

int launch_residuals(const float* x, int64_t n, int d, const int32_t* labels, const float* cc, int kc, float* r,
                     hipStream_t s) {
  if (n == 0) return MIPQ_OK;
  const int vec4 = (d % 4 == 0) && (((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(cc) |
                                       reinterpret_cast<uintptr_t>(r)) & 15) == 0);
  k_residuals<<<grid_cap(n, 8192), kT, 0, s>>>(x, n, d, labels, cc, kc, r, vec4);
  MIPQ_LAUNCHED("k_residuals");
  return MIPQ_OK;
}

int launch_gather_codes(const uint8_t* codes, int64_t n, int m, const int32_t* ids, uint8_t* out, hipStream_t s) {
  if (n == 0) return MIPQ_OK;
  const int vec16 = (m % 16 == 0) && (((reinterpret_cast<uintptr_t>(codes) | reinterpret_cast<uintptr_t>(out)) & 15) == 0);
  k_gather_codes<<<grid_cap(n, 8192), kT, 0, s>>>(codes, n, m, ids, out, vec16);
  MIPQ_LAUNCHED("k_gather_codes");
  return MIPQ_OK;
}

size_t merge_part_bytes() { return sizeof(MergePart); }

int launch_merge_lists(const void* parts, int nparts, int64_t total_rows, int kc, int m, int64_t* pre,
                       int64_t* total, int64_t* offsets, int32_t* ids, uint8_t* codes, bool vec16, hipStream_t s) {
  const MergePart* P = static_cast<const MergePart*>(parts);
  k_merge_prefix<<<ceil_div(kc, kT), kT, 0, s>>>(P, nparts, kc, pre, total);
  MIPQ_LAUNCHED("k_merge_prefix");
  k_merge_scan<<<1, kT, 0, s>>>(total, kc, offsets);
  MIPQ_LAUNCHED("k_merge_scan");
  if (total_rows > 0) {
    k_merge_copy<<<grid_cap(total_rows, 8192), kT, 0, s>>>(P, nparts, total_rows, kc, m, pre, offsets, ids, codes,
                                                          vec16 ? 1 : 0);
    MIPQ_LAUNCHED("k_merge_copy");
  }
  return MIPQ_OK;
}

}  // namespace mipq
