// Lloyd update (paper Section 2.1: k-means in every subspace): float64
// centroid sums per row chunk, then per subspace the centroid means, the
// round's objective and, for the matrix-core path, the packed centroid
// operands of the next round.  Also the stand-alone operand packing used
// before the first round and by encoding.
#include <math.h>

#include "bf16_pack.h"
#include "mipq_internal.h"

namespace mipq {

namespace {

constexpr int kUpdThreads = 512;   // accumulation blocks: several per CU overlap their set-up and stores
constexpr int kPackThreads = 256;
constexpr int kPackRed = 544;   // floats of LDS scratch for pack_subspace

// Block (c, j) adds the rows of chunk c to subspace j's float64 sums and counts
// in LDS (lane l takes dimension l % ds of row l / ds; sums centroid-major with
// a padded stride ds + 1 so that one centroid's dimensions sit in different
// banks) and the float64 squared distance of each row to its centroid, then
// stores them as the chunk's partials.
// With GX the block also writes dL/dx = 2 g (x - c) (float64 product rounded to
// float32, g = *gscale) for the reconstruction loss L = sum (x - x_hat)^2.
template <bool GX, bool OBJ, bool CHECK>
__device__ __forceinline__ void accumulate_chunk(
    const float* __restrict__ x, int64_t n, int d, int m, int ks, int ds,
    const uint8_t* __restrict__ codes, const float* __restrict__ c32, int64_t rpc, int c, int sub,
    double* __restrict__ part_s, uint32_t* __restrict__ part_cnt, double* __restrict__ part_j,
    const double* __restrict__ gscale, float* __restrict__ grad_x, double* smem, double* redj) {
  const int stride = ds + 1;
  double* S = smem;
  uint32_t* cnt = reinterpret_cast<uint32_t*>(S + (size_t)ks * stride);
  float* cbs = reinterpret_cast<float*>(S + (size_t)ks * stride + (ks + 1) / 2);
  const int per = ks * ds;
  for (int i = threadIdx.x; i < ks * stride; i += blockDim.x) S[i] = 0.0;
  for (int i = threadIdx.x; i < ks; i += blockDim.x) cnt[i] = 0u;
  if (OBJ)
    for (int i = threadIdx.x; i < per; i += blockDim.x) cbs[i] = c32[(int64_t)sub * per + i];
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int rpw = 64 / ds;                 // rows per wave step
  const int g = lane / ds, t = lane - g * ds;
  const int64_t r0 = (int64_t)c * rpc;
  const int64_t r1 = min(n, r0 + rpc);
  const int64_t step = (int64_t)(blockDim.x >> 6) * rpw;   // rows between a lane's consecutive rows
  const int64_t first = r0 + (int64_t)wave * rpw + g;
  // this lane's rows: first, first + step, ... below r1
  const int64_t nrows = (g < rpw && first < r1) ? (r1 - first + step - 1) / step : 0;
  const float* xp = x + first * d + (int64_t)sub * ds + t;
  const uint8_t* cp = codes + first * m + sub;
  float* gp = GX ? grad_x + first * d + (int64_t)sub * ds + t : nullptr;
  const int64_t xs = step * d, cs = step * m;
  double jl = 0.0;
  const double g2 = GX ? 2.0 * (gscale ? *gscale : 1.0) : 0.0;
  auto add_row = [&](int code, float xv, int64_t off) {
    if (CHECK && code >= ks) {   // corrupt code: poison the objective, touch no sum
      jl += NAN;
      if (GX) gp[off] = NAN;
      return;
    }
    if (OBJ) {
      const double df = (double)xv - (double)cbs[code * ds + t];
      jl += df * df;
      if (GX) gp[off] = (float)(g2 * df);
    }
    atomicAdd(&S[code * stride + t], (double)xv);
    if (t == 0) atomicAdd(&cnt[code], 1u);
  };
  constexpr int U = 8;   // rows in flight per lane
  int64_t i = 0;
  for (; i + U <= nrows; i += U) {
    int code[U];
    float xv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      code[u] = (int)cp[u * cs];
      xv[u] = xp[u * xs];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) add_row(code[u], xv[u], u * xs);
    xp += U * xs;
    cp += U * cs;
    if (GX) gp += U * xs;
  }
  for (; i < nrows; ++i) {
    add_row((int)cp[0], xp[0], 0);
    xp += xs;
    cp += cs;
    if (GX) gp += xs;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) jl += __shfl_xor(jl, off, 64);
  if (lane == 0) redj[wave] = jl;
  __syncthreads();
  const size_t base = (size_t)c * m + sub;
  for (int i = threadIdx.x; i < per; i += blockDim.x) {
    const int k = i / ds;
    part_s[base * per + i] = S[k * stride + (i - k * ds)];
  }
  for (int i = threadIdx.x; i < ks; i += blockDim.x) part_cnt[base * ks + i] = cnt[i];
  if (threadIdx.x == 0) {
    double js = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) js += redj[i];
    part_j[base] = js;
  }
}

// Vector form of accumulate_chunk for d/m and d multiples of 4 and 16-byte
// aligned rows: lane l takes the 4 dimensions 4q..4q+3 (q = l % (ds/4)) of
// row l / (ds/4) with one 16-byte load, and keeps U such rows in flight, so a
// wave has 16 times the bytes of the scalar form outstanding.  The sums, the
// counts and the order of the objective terms within a lane are those of the
// scalar form applied to the lane's elements; the atomic additions make the
// sums' last bits depend on their order, as there.
template <bool GX, bool OBJ, bool CHECK>
__device__ __forceinline__ void accumulate_chunk4(
    const float* __restrict__ x, int64_t n, int d, int m, int ks, int ds,
    const uint8_t* __restrict__ codes, const float* __restrict__ c32, int64_t rpc, int c, int sub,
    double* __restrict__ part_s, uint32_t* __restrict__ part_cnt, double* __restrict__ part_j,
    const double* __restrict__ gscale, float* __restrict__ grad_x, double* smem, double* redj) {
  const int stride = ds + 1;
  double* S = smem;
  uint32_t* cnt = reinterpret_cast<uint32_t*>(S + (size_t)ks * stride);
  float* cbs = reinterpret_cast<float*>(S + (size_t)ks * stride + (ks + 1) / 2);
  const int per = ks * ds;
  for (int i = threadIdx.x; i < ks * stride; i += blockDim.x) S[i] = 0.0;
  for (int i = threadIdx.x; i < ks; i += blockDim.x) cnt[i] = 0u;
  if (OBJ)
    for (int i = threadIdx.x; i < per; i += blockDim.x) cbs[i] = c32[(int64_t)sub * per + i];
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int lpr = ds >> 2;                 // lanes per row
  const int rpw = 64 / lpr;                // rows per wave step
  const int g = lane / lpr, t = (lane - g * lpr) * 4;
  const int64_t r0 = (int64_t)c * rpc;
  const int64_t r1 = min(n, r0 + rpc);
  const int64_t step = (int64_t)(blockDim.x >> 6) * rpw;
  const int64_t first = r0 + (int64_t)wave * rpw + g;
  const int64_t nrows = (g < rpw && first < r1) ? (r1 - first + step - 1) / step : 0;
  const float* xp = x + first * d + (int64_t)sub * ds + t;
  const uint8_t* cp = codes + first * m + sub;
  float* gp = GX ? grad_x + first * d + (int64_t)sub * ds + t : nullptr;
  const int64_t xs = step * d, cs = step * m;
  double jl = 0.0;
  const double g2 = GX ? 2.0 * (gscale ? *gscale : 1.0) : 0.0;
  auto add_row = [&](int code, const float4& v, int64_t off) {
    const float xv[4] = {v.x, v.y, v.z, v.w};
    if (CHECK && code >= ks) {
      jl += NAN;
      if (GX) *reinterpret_cast<float4*>(gp + off) = make_float4(NAN, NAN, NAN, NAN);
      return;
    }
    if (OBJ) {
      float gv[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const double df = (double)xv[e] - (double)cbs[code * ds + t + e];
        jl += df * df;
        gv[e] = (float)(g2 * df);
      }
      if (GX) *reinterpret_cast<float4*>(gp + off) = make_float4(gv[0], gv[1], gv[2], gv[3]);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) atomicAdd(&S[code * stride + t + e], (double)xv[e]);
    if (t == 0) atomicAdd(&cnt[code], 1u);
  };
  constexpr int U = 8;   // rows in flight per lane
  int64_t i = 0;
  for (; i + U <= nrows; i += U) {
    int code[U];
    float4 xv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      code[u] = (int)cp[u * cs];
      xv[u] = *reinterpret_cast<const float4*>(xp + u * xs);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) add_row(code[u], xv[u], u * xs);
    xp += U * xs;
    cp += U * cs;
    if (GX) gp += U * xs;
  }
  for (; i < nrows; ++i) {
    add_row((int)cp[0], *reinterpret_cast<const float4*>(xp), 0);
    xp += xs;
    cp += cs;
    if (GX) gp += xs;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) jl += __shfl_xor(jl, off, 64);
  if (lane == 0) redj[wave] = jl;
  __syncthreads();
  const size_t base = (size_t)c * m + sub;
  for (int i = threadIdx.x; i < per; i += blockDim.x) {
    const int k = i / ds;
    part_s[base * per + i] = S[k * stride + (i - k * ds)];
  }
  for (int i = threadIdx.x; i < ks; i += blockDim.x) part_cnt[base * ks + i] = cnt[i];
  if (threadIdx.x == 0) {
    double js = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) js += redj[i];
    part_j[base] = js;
  }
}

// As accumulate_chunk4, for G consecutive subspaces sub0 .. sub0 + G - 1 of
// chunk c in one block, so that a row's G ds floats (G ds / 4 lanes, 16 bytes
// each) are one contiguous read and one contiguous write: with one subspace
// per block, the blocks of a chunk each read and write a 32-byte piece of a
// row's cache lines at different times, and the lines went to and from HBM
// about 1.5 times.  LDS: per subspace the sums S [ks][ds + 1], counts [ks]
// and (OBJ) the float32 centroids.  The objective partial of each subspace is
// reduced in a fixed order (lanes of one subspace by xor steps, then the
// waves in order), as in accumulate_chunk4.
template <bool GX, bool OBJ, bool CHECK, int G>
__device__ __forceinline__ void accumulate_group4(
    const float* __restrict__ x, int64_t n, int d, int m, int ks, int ds,
    const uint8_t* __restrict__ codes, const float* __restrict__ c32, int64_t rpc, int c, int sub0,
    double* __restrict__ part_s, uint32_t* __restrict__ part_cnt, double* __restrict__ part_j,
    const double* __restrict__ gscale, float* __restrict__ grad_x, double* smem, double* redj) {
  const int stride = ds + 1;
  const int per = ks * ds;
  double* S0 = smem;                                                          // [G][ks * stride]
  uint32_t* cnt0 = reinterpret_cast<uint32_t*>(S0 + (size_t)G * ks * stride);   // [G][ks]
  float* cbs0 = reinterpret_cast<float*>(cnt0 + (size_t)G * ks);               // [G][per]
  for (int i = threadIdx.x; i < G * ks * stride; i += blockDim.x) S0[i] = 0.0;
  for (int i = threadIdx.x; i < G * ks; i += blockDim.x) cnt0[i] = 0u;
  if (OBJ)
    for (int i = threadIdx.x; i < G * per; i += blockDim.x) cbs0[i] = c32[(int64_t)sub0 * per + i];
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int lps = ds >> 2;                 // lanes per subspace slice
  const int lpr = G * lps;                 // lanes per row (a power of two <= 64)
  const int rpw = 64 / lpr;                // rows per wave step
  const int g = lane / lpr, li = lane - g * lpr;
  const int j = li / lps, t = (li - j * lps) * 4;
  double* S = S0 + (size_t)j * ks * stride;
  uint32_t* cnt = cnt0 + (size_t)j * ks;
  const float* cbs = cbs0 + (size_t)j * per;
  const int64_t r0 = (int64_t)c * rpc;
  const int64_t r1 = min(n, r0 + rpc);
  const int64_t step = (int64_t)(blockDim.x >> 6) * rpw;
  const int64_t first = r0 + (int64_t)wave * rpw + g;
  const int64_t nrows = first < r1 ? (r1 - first + step - 1) / step : 0;
  const float* xp = x + first * d + (int64_t)sub0 * ds + li * 4;
  const uint8_t* cp = codes + first * m + sub0 + j;
  float* gp = GX ? grad_x + first * d + (int64_t)sub0 * ds + li * 4 : nullptr;
  const int64_t xs = step * d, cs = step * m;
  double jl = 0.0;
  const double g2 = GX ? 2.0 * (gscale ? *gscale : 1.0) : 0.0;
  auto add_row = [&](int code, const float4& v, int64_t off) {
    const float xv[4] = {v.x, v.y, v.z, v.w};
    if (CHECK && code >= ks) {
      jl += NAN;
      if (GX) *reinterpret_cast<float4*>(gp + off) = make_float4(NAN, NAN, NAN, NAN);
      return;
    }
    if (OBJ) {
      float gv[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const double df = (double)xv[e] - (double)cbs[code * ds + t + e];
        jl += df * df;
        gv[e] = (float)(g2 * df);
      }
      if (GX) *reinterpret_cast<float4*>(gp + off) = make_float4(gv[0], gv[1], gv[2], gv[3]);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) atomicAdd(&S[code * stride + t + e], (double)xv[e]);
    if (t == 0) atomicAdd(&cnt[code], 1u);
  };
  constexpr int U = 6;   // rows in flight per lane (8 spills at 1024 threads)
  int64_t i = 0;
  for (; i + U <= nrows; i += U) {
    int code[U];
    float4 xv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      code[u] = (int)cp[u * cs];
      xv[u] = *reinterpret_cast<const float4*>(xp + u * xs);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) add_row(code[u], xv[u], u * xs);
    xp += U * xs;
    cp += U * cs;
    if (GX) gp += U * xs;
  }
  for (; i < nrows; ++i) {
    add_row((int)cp[0], *reinterpret_cast<const float4*>(xp), 0);
    xp += xs;
    cp += cs;
    if (GX) gp += xs;
  }
  // the lanes of subspace j differ in their row (bits at and above lpr) and
  // their slice (bits below lps): xor steps over those bits only
  for (int off = 1; off < lps; off <<= 1) jl += __shfl_xor(jl, off, 64);
  for (int off = lpr; off < 64; off <<= 1) jl += __shfl_xor(jl, off, 64);
  if (g == 0 && t == 0) redj[wave * G + j] = jl;
  __syncthreads();
  const size_t base = (size_t)c * m + sub0;
  for (int i2 = threadIdx.x; i2 < G * per; i2 += blockDim.x) {
    const int jj = i2 / per, r = i2 - jj * per;
    const int k = r / ds;
    part_s[(base + jj) * per + r] = S0[(size_t)jj * ks * stride + k * stride + (r - k * ds)];
  }
  for (int i2 = threadIdx.x; i2 < G * ks; i2 += blockDim.x) {
    const int jj = i2 / ks;
    part_cnt[(base + jj) * ks + (i2 - jj * ks)] = cnt0[i2];
  }
  if (threadIdx.x < G) {
    double js = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) js += redj[w * G + threadIdx.x];
    part_j[base + threadIdx.x] = js;
  }
}

// LDS of accumulate_group4 for G subspaces (OBJ: with the float32 centroids)
__host__ __device__ constexpr size_t group4_lds_bytes(int ks, int ds, int G) {
  return (size_t)G * ks * (ds + 1) * sizeof(double) + (size_t)G * ks * sizeof(uint32_t) +
         (size_t)G * ks * ds * sizeof(float);
}

// rows of x can be read 16 bytes at a time in every subspace
__host__ __device__ __forceinline__ bool rows_vec4(const float* x, int d, int ds) {
  return ds % 4 == 0 && d % 4 == 0 && (reinterpret_cast<uintptr_t>(x) & 15) == 0;
}

// Deterministic variant (MIPQ_DETERMINISTIC): no floating-point atomics.  The
// chunk's rows are taken in pieces of kDetPiece rows; each piece's positions
// are sorted by code with a stable two-pass counting sort on 4-bit digits
// (low, then high; ranks inside 64 consecutive elements from wave ballots),
// then thread q owns the sums of pair q = (centroid k, dimension t) and adds
// x[row][t] of the piece's rows coded k in row order, pieces in order.  The
// objective terms are added by the same threads in the same order.  Every sum
// therefore depends only on the inputs.
constexpr int kDetPiece = 1024;
constexpr int kDetBatches = kDetPiece / 64;

__host__ __device__ constexpr size_t det_lds_bytes(int ks, int ds, bool obj) {
  return (size_t)ks * ds * sizeof(double) + (obj ? (size_t)ks * ds * sizeof(float) : 0) +
         ((size_t)3 * ks + 1 + 16 * kDetBatches + 32) * sizeof(uint32_t) + 2 * kDetPiece * sizeof(uint16_t) +
         kDetPiece;
}

template <bool OBJ>
__device__ __forceinline__ void accumulate_chunk_det(
    const float* __restrict__ x, int64_t n, int d, int m, int ks, int ds, const uint8_t* __restrict__ codes,
    const float* __restrict__ c32, int64_t rpc, int c, int sub, double* __restrict__ part_s,
    uint32_t* __restrict__ part_cnt, double* __restrict__ part_j, char* smem, double* redj) {
  const int per = ks * ds;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6;
  double* S = reinterpret_cast<double*>(smem);                     // [per]
  float* cbs = reinterpret_cast<float*>(S + per);                  // [per] (OBJ)
  uint32_t* cnt = reinterpret_cast<uint32_t*>(cbs + (OBJ ? per : 0));   // [ks]
  uint32_t* cntp = cnt + ks;                                       // [ks] histogram of the piece
  uint32_t* off = cntp + ks;                                       // [ks + 1]
  uint32_t* bcount = off + ks + 1;                                 // [kDetBatches][16]
  uint32_t* dtot = bcount + 16 * kDetBatches;                      // [16] digit totals
  uint32_t* dbase = dtot + 16;                                     // [16]
  uint16_t* permA = reinterpret_cast<uint16_t*>(dbase + 16);       // [kDetPiece]
  uint16_t* permB = permA + kDetPiece;                             // [kDetPiece]
  uint8_t* pc = reinterpret_cast<uint8_t*>(permB + kDetPiece);     // [kDetPiece]
  for (int i = tid; i < per; i += nthr) {
    S[i] = 0.0;
    if (OBJ) cbs[i] = c32[(int64_t)sub * per + i];
  }
  for (int i = tid; i < ks; i += nthr) cnt[i] = 0u;
  const int64_t r0 = (int64_t)c * rpc;
  const int64_t r1 = min(n, r0 + rpc);
  const float* xs = x + (int64_t)sub * ds;
  double jl = 0.0;
  for (int64_t p0 = r0; p0 < r1; p0 += kDetPiece) {
    const int L = (int)min((int64_t)kDetPiece, r1 - p0);
    for (int i = tid; i < ks; i += nthr) cntp[i] = 0u;
    __syncthreads();
    for (int i = tid; i < L; i += nthr) {
      const int cd = codes[(p0 + i) * m + sub];
      pc[i] = (uint8_t)cd;
      if (cd < ks) atomicAdd(&cntp[cd], 1u);   // integer counts: order-independent
    }
    __syncthreads();
    // exclusive scan of the piece histogram (one wave, 4 bins per lane)
    if (wave == 0) {
      uint32_t v[4], run = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = lane * 4 + q;
        v[q] = k < ks ? cntp[k] : 0u;
        run += v[q];
      }
      uint32_t inc = run;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
      }
      uint32_t e = inc - run;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = lane * 4 + q;
        if (k < ks) off[k] = e;
        e += v[q];
      }
      if (lane == 63) off[ks] = inc;
    }
    // stable sort of the piece's positions by code
    for (int pass = 0; pass < 2; ++pass) {
      const int shift = 4 * pass;
      uint16_t* dst = pass ? permB : permA;
      for (int i = tid; i < 16 * kDetBatches; i += nthr) bcount[i] = 0u;
      __syncthreads();
      constexpr int kPer = 4;   // elements per thread (kDetPiece / 256 threads at most)
      int rank[kPer], dig[kPer], pos[kPer];
#pragma unroll
      for (int j = 0; j < kPer; ++j) {
        const int e = j * nthr + tid;   // batch e / 64: lanes hold consecutive elements
        const bool live = e < L;
        pos[j] = live ? (pass ? (int)permA[e] : e) : 0;
        dig[j] = live ? ((pc[pos[j]] >> shift) & 15) : 0;
        uint64_t eq = __ballot(live);
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const uint64_t bm = __ballot(live && ((dig[j] >> b) & 1));
          eq &= ((dig[j] >> b) & 1) ? bm : ~bm;
        }
        rank[j] = __popcll(eq & ((1ull << lane) - 1ull));
        if (live && rank[j] == 0) bcount[(e >> 6) * 16 + dig[j]] = (uint32_t)__popcll(eq);
        if (!live) rank[j] = -1;
      }
      __syncthreads();
      if (tid < 16) {   // per digit: batches in order
        uint32_t run = 0;
        for (int b = 0; b < kDetBatches; ++b) {
          const uint32_t v = bcount[b * 16 + tid];
          bcount[b * 16 + tid] = run;
          run += v;
        }
        dtot[tid] = run;
      }
      __syncthreads();
      if (tid == 0) {
        uint32_t run = 0;
        for (int g = 0; g < 16; ++g) {
          dbase[g] = run;
          run += dtot[g];
        }
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < kPer; ++j) {
        const int e = j * nthr + tid;
        if (rank[j] >= 0) dst[dbase[dig[j]] + bcount[(e >> 6) * 16 + dig[j]] + rank[j]] = (uint16_t)pos[j];
      }
      __syncthreads();
    }
    // sums of the piece: pair q = (k, t), rows of code k in row order
    for (int q = tid; q < per; q += nthr) {
      const int k = q / ds, t = q - k * ds;
      const uint32_t b = off[k], e = off[k + 1];
      double acc = S[q];
      const double cv = OBJ ? (double)cbs[q] : 0.0;
      const float* xc = xs + p0 * d + t;
      uint32_t i = b;
      for (; i + 4 <= e; i += 4) {
        float v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = xc[(int64_t)permB[i + u] * d];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          acc += (double)v[u];
          if (OBJ) {
            const double df = (double)v[u] - cv;
            jl += df * df;
          }
        }
      }
      for (; i < e; ++i) {
        const float v = xc[(int64_t)permB[i] * d];
        acc += (double)v;
        if (OBJ) {
          const double df = (double)v - cv;
          jl += df * df;
        }
      }
      S[q] = acc;
    }
    for (int k = tid; k < ks; k += nthr) cnt[k] += cntp[k];
    __syncthreads();
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) jl += __shfl_xor(jl, o, 64);
  if (lane == 0) redj[wave] = jl;
  __syncthreads();
  const size_t base = (size_t)c * m + sub;
  for (int i = tid; i < per; i += nthr) part_s[base * per + i] = S[i];
  for (int i = tid; i < ks; i += nthr) part_cnt[base * ks + i] = cnt[i];
  if (tid == 0) {
    double js = 0.0;
    for (int i = 0; i < (nthr >> 6); ++i) js += redj[i];
    part_j[base] = js;
  }
}

// Block -> (chunk, subspace) so that the m blocks of one chunk run on one XCD
// (hardware block id mod 8) next to each other: they read the same rows, which
// then come from that XCD's L2.  Chunks go round-robin over the XCDs.
struct ChunkMap {
  int64_t chunk;
  int sub;
};
__device__ __forceinline__ ChunkMap chunk_map(int64_t b, int m) {
  const int64_t xcd = b & 7, slot = b >> 3;
  ChunkMap r;
  r.chunk = (slot / m) * 8 + xcd;
  r.sub = (int)(slot - (slot / m) * m);
  return r;
}

// One problem: chunk c, subspace j (see chunk_map).  NT threads per block:
// kUpdThreads for the fit; the backward, which also writes dL/dx, runs
// kBwdThreads.
constexpr int kBwdThreads = 1024;
constexpr int kDetThreads = 256;   // four elements per thread in the piece sort

template <bool GX, bool OBJ, bool CHECK, int NT>
__global__ __launch_bounds__(NT) void k_accumulate(
    const float* __restrict__ x, int64_t n, int d, int m, int ks, int ds,
    const uint8_t* __restrict__ codes, const float* __restrict__ c32, int64_t rpc, int nch,
    double* __restrict__ part_s, uint32_t* __restrict__ part_cnt, double* __restrict__ part_j,
    const double* __restrict__ gscale, float* __restrict__ grad_x, float* __restrict__ cmax_zero) {
  extern __shared__ double smem[];
  __shared__ double redj[NT / 64];
  // the next finalize raises cmax[j] tile by tile from zero (the round's
  // assignment, which read it, has finished)
  if (cmax_zero && blockIdx.x == 0)
    for (int j = threadIdx.x; j < m; j += blockDim.x) cmax_zero[j] = 0.0f;
  const ChunkMap cm = chunk_map(blockIdx.x, m);
  if (cm.chunk >= nch) return;   // padding of the grid (every chunk's partials are written)
  if (rows_vec4(x, d, ds) && (!GX || rows_vec4(grad_x, d, ds)))
    accumulate_chunk4<GX, OBJ, CHECK>(x, n, d, m, ks, ds, codes, c32, rpc, (int)cm.chunk, cm.sub, part_s, part_cnt,
                                      part_j, gscale, grad_x, smem, redj);
  else
    accumulate_chunk<GX, OBJ, CHECK>(x, n, d, m, ks, ds, codes, c32, rpc, (int)cm.chunk, cm.sub, part_s, part_cnt,
                                     part_j, gscale, grad_x, smem, redj);
}

// Deterministic accumulation (see accumulate_chunk_det), one problem.
template <bool OBJ>
__global__ __launch_bounds__(kDetThreads) void k_accumulate_det(
    const float* __restrict__ x, int64_t n, int d, int m, int ks, int ds, const uint8_t* __restrict__ codes,
    const float* __restrict__ c32, int64_t rpc, int nch, double* __restrict__ part_s,
    uint32_t* __restrict__ part_cnt, double* __restrict__ part_j, float* __restrict__ cmax_zero) {
  extern __shared__ double smem[];
  __shared__ double redj[kDetThreads / 64];
  if (cmax_zero && blockIdx.x == 0)
    for (int j = threadIdx.x; j < m; j += blockDim.x) cmax_zero[j] = 0.0f;
  const ChunkMap cm = chunk_map(blockIdx.x, m);
  if (cm.chunk >= nch) return;
  accumulate_chunk_det<OBJ>(x, n, d, m, ks, ds, codes, c32, rpc, (int)cm.chunk, cm.sub, part_s, part_cnt, part_j,
                            reinterpret_cast<char*>(smem), redj);
}

// the last problem p with key(p) <= i (problems in ascending key order)
template <class Key>
__device__ __forceinline__ int find_problem(const BatchProb* __restrict__ probs, int nprob, int64_t i, Key key) {
  int lo = 0, hi = nprob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (key(probs[mid]) <= i) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Many problems: block i is accumulation item i = (problem p, chunk c,
// subspace j) with items problem-major, then chunk, then subspace; problem p's
// partials use the single-problem layout at offset item0.
// The reconstruction-loss backward with G consecutive subspaces per block
// (accumulate_group4): block -> (chunk, group of G) as chunk_map does for
// single subspaces.
template <bool GX, int G>
__global__ __launch_bounds__(kBwdThreads) void k_backward_group(
    const float* __restrict__ x, int64_t n, int d, int m, int ks, int ds, const uint8_t* __restrict__ codes,
    const float* __restrict__ c32, int64_t rpc, int nch, double* __restrict__ part_s,
    uint32_t* __restrict__ part_cnt, double* __restrict__ part_j, const double* __restrict__ gscale,
    float* __restrict__ grad_x) {
  extern __shared__ double smem[];
  __shared__ double redj[kBwdThreads / 64 * G];
  const ChunkMap cm = chunk_map(blockIdx.x, m / G);
  if (cm.chunk >= nch) return;   // padding of the grid
  accumulate_group4<GX, true, true, G>(x, n, d, m, ks, ds, codes, c32, rpc, (int)cm.chunk, cm.sub * G, part_s,
                                       part_cnt, part_j, gscale, grad_x, smem, redj);
}

template <bool DET, int NT>
__global__ __launch_bounds__(NT) void k_accumulate_batched(const BatchProb* __restrict__ probs, int nprob,
                                                           int64_t items, int d, int m, int ks, int ds,
                                                           double* __restrict__ part_s,
                                                           uint32_t* __restrict__ part_cnt,
                                                           double* __restrict__ part_j) {
  extern __shared__ double smem[];
  __shared__ double redj[NT / 64];
  const ChunkMap cmap = chunk_map(blockIdx.x, m);
  const int64_t i = cmap.chunk * m + cmap.sub;   // item: chunks of all problems in order, then subspace
  if (i >= items) return;
  const int p = find_problem(probs, nprob, i, [](const BatchProb& b) { return b.item0; });
  const int64_t item0 = probs[p].item0;
  const int local = (int)(i - item0);
  const int c = local / m, sub = local - (local / m) * m;
  const size_t per = (size_t)ks * ds;
  // the deterministic sums run with the single-problem block size, so that
  // every result (the objective too) equals the single call's
  if (DET)
    accumulate_chunk_det<true>(probs[p].x, probs[p].n, d, m, ks, ds, probs[p].codes, probs[p].c32, probs[p].rpc, c,
                               sub, part_s + item0 * per, part_cnt + item0 * ks, part_j + item0,
                               reinterpret_cast<char*>(smem), redj);
  else if (rows_vec4(probs[p].x, d, ds))
    accumulate_chunk4<false, true, false>(probs[p].x, probs[p].n, d, m, ks, ds, probs[p].codes, probs[p].c32,
                                          probs[p].rpc, c, sub, part_s + item0 * per, part_cnt + item0 * ks,
                                          part_j + item0, nullptr, nullptr, smem, redj);
  else
    accumulate_chunk<false, true, false>(probs[p].x, probs[p].n, d, m, ks, ds, probs[p].codes, probs[p].c32,
                                         probs[p].rpc, c, sub, part_s + item0 * per, part_cnt + item0 * ks,
                                         part_j + item0, nullptr, nullptr, smem, redj);
}

// Subspace sub (paths without matrix-core operands): sums the chunk partials
// in chunk order, centroid = sum / count (an empty centroid keeps its value),
// float32 copy by round-to-nearest, and the subspace objective (*j_out).
__device__ __forceinline__ void finalize_sub(int sub, int m, int ks, int ds, int nch,
                                             const double* __restrict__ part_s,
                                             const uint32_t* __restrict__ part_cnt,
                                             const double* __restrict__ part_j, float* __restrict__ c32,
                                             double* __restrict__ c64, double* __restrict__ j_out) {
  const int per = ks * ds;
  for (int e = threadIdx.x; e < per; e += blockDim.x) {
    const int k = e / ds;
    double sacc = 0.0;
    uint64_t cacc = 0;
    constexpr int V = 16;   // partials in flight, added in chunk order
    for (int c0 = 0; c0 < nch; c0 += V) {
      double sv[V];
      uint32_t cv[V];
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const int cc = c0 + v < nch ? c0 + v : nch - 1;
        const size_t b2 = (size_t)cc * m + sub;
        sv[v] = part_s[b2 * per + e];
        cv[v] = part_cnt[b2 * ks + k];
      }
#pragma unroll
      for (int v = 0; v < V; ++v)
        if (c0 + v < nch) {
          sacc += sv[v];
          cacc += cv[v];
        }
    }
    const size_t o = (size_t)sub * per + e;
    const double v = cacc ? sacc / (double)cacc : c64[o];
    c64[o] = v;
    const float f = (float)v;
    c32[o] = f;
  }
  if (threadIdx.x < 64) {   // objective: lane-strided chunk sums, then a fixed xor tree
    double js = 0.0;
    for (int cc = threadIdx.x; cc < nch; cc += 64) js += part_j[(size_t)cc * m + sub];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) js += __shfl_xor(js, off, 64);
    if (threadIdx.x == 0 && j_out) *j_out = js;
  }
}

// One block per subspace.
__global__ __launch_bounds__(kUpdThreads) void k_finalize(int m, int ks, int ds, int nch,
                                                          const double* __restrict__ part_s,
                                                          const uint32_t* __restrict__ part_cnt,
                                                          const double* __restrict__ part_j,
                                                          float* __restrict__ c32, double* __restrict__ c64,
                                                          double* __restrict__ j_sub) {
  finalize_sub(blockIdx.x, m, ks, ds, nch, part_s, part_cnt, part_j, c32, c64, j_sub + blockIdx.x);
}

// One problem, block (tile t, subspace j): the means of the tile's 32
// centroids (chunk partials summed in chunk order, float64; empty keeps its
// value), then the tile's operand slots for the next round, centred by the
// subspace centre mu fixed at the start of the fit, and the tile's largest
// centred norm raised into cmax[j] (zeroed by the accumulation).  Block t = 0
// also sums the round's objective.  All tiles of all subspaces run at once.
constexpr int kFinTileThreads = 256;

template <int NB>
__device__ __forceinline__ void finalize_tile(int t, int sub, int m, int ks, int ds, int nch,
                                              const double* __restrict__ part_s,
                                              const uint32_t* __restrict__ part_cnt,
                                              const double* __restrict__ part_j, float* __restrict__ c32,
                                              double* __restrict__ c64, double* __restrict__ j_out,
                                              uint4* __restrict__ aop, float* __restrict__ cmax,
                                              const float* __restrict__ mu, int nt, float* newc, float* mus,
                                              float* wmax, float* __restrict__ tmax = nullptr) {
  constexpr int NMF = bf16_nmfma(NB);
  const int per = ks * ds;
  const int k0 = t * 32;
  const int kn = min(32, ks - k0);
  // the centre, loaded while the partials are summed
  const float mu_t = threadIdx.x < NB * 8 ? mu[sub * kMaxDsBf16 + threadIdx.x] : 0.0f;
  for (int le = threadIdx.x; le < kn * ds; le += blockDim.x) {
    const int e = k0 * ds + le;
    const int k = e / ds;
    double sacc = 0.0;
    uint64_t cacc = 0;
    constexpr int V = 16;   // partials in flight, added in chunk order
    for (int c0 = 0; c0 < nch; c0 += V) {
      double sv[V];
      uint32_t cv[V];
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const int cc = c0 + v < nch ? c0 + v : nch - 1;
        const size_t b2 = (size_t)cc * m + sub;
        sv[v] = part_s[b2 * per + e];
        cv[v] = part_cnt[b2 * ks + k];
      }
#pragma unroll
      for (int v = 0; v < V; ++v)
        if (c0 + v < nch) {
          sacc += sv[v];
          cacc += cv[v];
        }
    }
    const size_t o = (size_t)sub * per + e;
    const double v = cacc ? sacc / (double)cacc : c64[o];
    c64[o] = v;
    const float f = (float)v;
    c32[o] = f;
    newc[le] = f;
  }
  if (threadIdx.x < NB * 8) mus[threadIdx.x] = mu_t;
  if (t == 0 && j_out && threadIdx.x < 64) {   // objective: lane-strided chunk sums, then a fixed xor tree
    double js = 0.0;
    for (int cc = threadIdx.x; cc < nch; cc += 64) js += part_j[(size_t)cc * m + sub];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) js += __shfl_xor(js, off, 64);
    if (threadIdx.x == 0) *j_out = js;
  }
  __syncthreads();
  float mx = 0.0f;
  for (int s = threadIdx.x; s < NMF * 64; s += blockDim.x) {
    const int l = s & 63;
    const int f = s >> 6;
    const int i = l & 31;
    double cn;
    const Pack8 out = slot_value<NB>(i < kn ? newc + i * ds : nullptr, mus, ds, f, l >> 5, cn);
    store_pack(aop + ((size_t)(sub * nt + t) * NMF + f) * 64 + l, out);
    if (i < kn) mx = fmaxf(mx, (float)(sqrt(cn) * (1.0 + 1e-6)));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    float a = wmax[0];
    for (int i = 1; i < kFinTileThreads / 64; ++i) a = fmaxf(a, wmax[i]);
    if (tmax)
      tmax[t] = a;   // the tile's own slot, reduced by k_next_round_batched
    else   // non-negative floats order as their bit patterns
      atomicMax(reinterpret_cast<unsigned int*>(cmax + sub), __float_as_uint(a));
  }
}

template <int NB>
__global__ __launch_bounds__(kFinTileThreads) void k_finalize_tiles(int m, int ks, int ds, int nch,
                                                                    const double* __restrict__ part_s,
                                                                    const uint32_t* __restrict__ part_cnt,
                                                                    const double* __restrict__ part_j,
                                                                    float* __restrict__ c32, double* __restrict__ c64,
                                                                    double* __restrict__ j_sub,
                                                                    uint4* __restrict__ aop,
                                                                    float* __restrict__ cmax,
                                                                    const float* __restrict__ mu, int nt) {
  __shared__ float newc[32 * NB * 8];
  __shared__ float mus[NB * 8];
  __shared__ float wmax[kFinTileThreads / 64];
  finalize_tile<NB>(blockIdx.x, blockIdx.y, m, ks, ds, nch, part_s, part_cnt, part_j, c32, c64,
                    j_sub ? j_sub + blockIdx.y : nullptr, aop, cmax, mu, nt, newc, mus, wmax);
}

// Many problems: block (tile t, subspace j, problem p), as k_finalize_tiles
// on problem p's partials; the round index comes from *round (see
// k_finalize_batched).  The tile's norm bound goes to its own slot
// tmax_all[(p m + j) kMaxTiles + t], so that no kernel of the round has to
// clear cmax while another may read it; k_next_round_batched reduces them.
template <int NB>
__global__ __launch_bounds__(kFinTileThreads) void k_finalize_tiles_batched(
    const BatchProb* __restrict__ probs, int nprob, int m, int ks, int ds, const double* __restrict__ part_s,
    const uint32_t* __restrict__ part_cnt, const double* __restrict__ part_j, double* __restrict__ c64_all,
    double* __restrict__ j_all, const uint32_t* __restrict__ round, int iters, uint4* __restrict__ aop_all,
    size_t aop_stride, float* __restrict__ cmax_all, const float* __restrict__ mu_all, int nt,
    float* __restrict__ tmax_all) {
  __shared__ float newc[32 * NB * 8];
  __shared__ float mus[NB * 8];
  __shared__ float wmax[kFinTileThreads / 64];
  const int t = blockIdx.x, sub = blockIdx.y, p = blockIdx.z;
  const int64_t item0 = probs[p].item0;
  const size_t per = (size_t)ks * ds;
  const uint32_t r = *round;
  double* j_out = r < (uint32_t)iters ? j_all + ((size_t)r * nprob + p) * m + sub : nullptr;
  finalize_tile<NB>(t, sub, m, ks, ds, probs[p].nch, part_s + item0 * per, part_cnt + item0 * ks, part_j + item0,
                    probs[p].c32, c64_all + (size_t)p * m * per, j_out, aop_all + (size_t)p * aop_stride,
                    cmax_all + (size_t)p * m, mu_all + (size_t)p * m * kMaxDsBf16, nt, newc, mus, wmax,
                    tmax_all + ((size_t)p * m + sub) * kMaxTiles);
}

__global__ void k_next_round(uint32_t* round) {
  if (threadIdx.x == 0) round[0] = round[0] + 1u;
}

// Many problems: cmax[i] = the largest of subspace i's nt tile bounds (every
// slot written by this round's finalize), then the round counter advances.
__global__ __launch_bounds__(256) void k_next_round_batched(uint32_t* __restrict__ round,
                                                            const float* __restrict__ tmax_all,
                                                            float* __restrict__ cmax_all, int count, int nt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) {
    float a = tmax_all[(size_t)i * kMaxTiles];
    for (int t = 1; t < nt; ++t) a = fmaxf(a, tmax_all[(size_t)i * kMaxTiles + t]);
    cmax_all[i] = a;
  }
  if (i == 0) round[0] = round[0] + 1u;
}

// dL/dC_j[k] = 2 g (cnt_jk C_j[k] - S_jk) with the chunk partials summed in
// chunk order (float64), rounded to float32; also subspace j's loss.
__global__ __launch_bounds__(kUpdThreads) void k_grad_codebook(int m, int ks, int ds, int nch,
                                                               const double* __restrict__ part_s,
                                                               const uint32_t* __restrict__ part_cnt,
                                                               const double* __restrict__ part_j,
                                                               const float* __restrict__ c32,
                                                               const double* __restrict__ gscale,
                                                               float* __restrict__ grad_c,
                                                               double* __restrict__ loss_sub) {
  const int sub = blockIdx.x;
  const int per = ks * ds;
  const double g2 = 2.0 * (gscale ? *gscale : 1.0);
  if (grad_c)
    for (int e = threadIdx.x; e < per; e += blockDim.x) {
      const int k = e / ds;
      double sacc = 0.0;
      uint64_t cacc = 0;
      constexpr int V = 8;
      for (int c0 = 0; c0 < nch; c0 += V) {
        double sv[V];
        uint32_t cv[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
          const int cc = c0 + v < nch ? c0 + v : nch - 1;
          const size_t b2 = (size_t)cc * m + sub;
          sv[v] = part_s[b2 * per + e];
          cv[v] = part_cnt[b2 * ks + k];
        }
#pragma unroll
        for (int v = 0; v < V; ++v)
          if (c0 + v < nch) {
            sacc += sv[v];
            cacc += cv[v];
          }
      }
      const size_t o = (size_t)sub * per + e;
      grad_c[o] = (float)(g2 * ((double)cacc * (double)c32[o] - sacc));
    }
  if (threadIdx.x < 64) {
    double js = 0.0;
    for (int cc = threadIdx.x; cc < nch; cc += 64) js += part_j[(size_t)cc * m + sub];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) js += __shfl_xor(js, off, 64);
    if (threadIdx.x == 0) loss_sub[sub] = js;
  }
}

// Stand-alone packing: block (t, j) packs tile t of subspace j; block (0, j)
// also stores the subspace centre and norm bound.
template <int NB>
__global__ __launch_bounds__(kPackThreads) void k_pack_bf16(const float* __restrict__ c32, int ks, int ds,
                                                            int nt, uint4* __restrict__ aop,
                                                            float* __restrict__ cmax, float* __restrict__ mu) {
  __shared__ float red[kPackRed];
  const int t = blockIdx.x, sub = blockIdx.y;
  pack_subspace<NB>(c32 + (int64_t)sub * ks * ds, ks, ds, nt, sub, t, t + 1, aop, cmax + sub,
                    mu + sub * kMaxDsBf16, t == 0, red);
}

// Many problems: block (t, j, p) packs tile t of subspace j of problem p.
template <int NB>
__global__ __launch_bounds__(kPackThreads) void k_pack_bf16_batched(const BatchProb* __restrict__ probs, int ks,
                                                                    int ds, int m, int nt, uint4* __restrict__ aop_all,
                                                                    size_t aop_stride, float* __restrict__ cmax_all,
                                                                    float* __restrict__ mu_all) {
  __shared__ float red[kPackRed];
  const int t = blockIdx.x, sub = blockIdx.y, p = blockIdx.z;
  pack_subspace<NB>(probs[p].c32 + (int64_t)sub * ks * ds, ks, ds, nt, sub, t, t + 1,
                    aop_all + (size_t)p * aop_stride, cmax_all + (size_t)p * m + sub,
                    mu_all + ((size_t)p * m + sub) * kMaxDsBf16, t == 0, red);
}

}  // namespace

// at least 4096 rows per chunk (the block's fixed cost of clearing and
// storing its sums stays small), at most 256 (chunk, subspace) blocks
int update_chunks(int64_t n, int m) {
  int nch = ceil_div(n, 4096);
  int cap = 256 / m;
  if (cap < 1) cap = 1;
  if (nch > cap) nch = cap;
  return nch < 1 ? 1 : nch;
}

int launch_update(const float* x, int64_t n, int d, int m, int ks, const uint8_t* codes, float* c32,
                  double* c64, int nch, double* part_s, uint32_t* part_cnt, double* part_j,
                  double* j_sub, void* aop, float* cmax, float* mu, bool objective, bool det, hipStream_t s) {
  const int ds = d / m;
  const int64_t rpc = (n + nch - 1) / nch;
  if (det) {
    const unsigned grid = (unsigned)(((nch + 7) / 8) * 8 * m);
    ProfScope ps(MIPQ_K_UPDATE, s);
    float* cz = aop ? cmax : nullptr;
    if (objective)
      k_accumulate_det<true><<<grid, kDetThreads, det_lds_bytes(ks, ds, true), s>>>(
          x, n, d, m, ks, ds, codes, c32, rpc, nch, part_s, part_cnt, part_j, cz);
    else
      k_accumulate_det<false><<<grid, kDetThreads, det_lds_bytes(ks, ds, false), s>>>(
          x, n, d, m, ks, ds, codes, c32, rpc, nch, part_s, part_cnt, part_j, cz);
    MIPQ_LAUNCHED("k_accumulate_det");
  } else {
    const size_t shm = (size_t)ks * (ds + 1) * sizeof(double) + ((ks + 1) / 2) * sizeof(double) +
                       (size_t)ks * ds * sizeof(float);
    const unsigned grid = (unsigned)(((nch + 7) / 8) * 8 * m);
    ProfScope ps(MIPQ_K_UPDATE, s);
    float* cz = aop ? cmax : nullptr;
    if (objective)
      k_accumulate<false, true, false, kUpdThreads><<<grid, kUpdThreads, shm, s>>>(
          x, n, d, m, ks, ds, codes, c32, rpc, nch, part_s, part_cnt, part_j, nullptr, nullptr, cz);
    else
      k_accumulate<false, false, false, kUpdThreads><<<grid, kUpdThreads, shm, s>>>(
          x, n, d, m, ks, ds, codes, c32, rpc, nch, part_s, part_cnt, part_j, nullptr, nullptr, cz);
    MIPQ_LAUNCHED("k_accumulate");
  }
  return launch_finalize(m, ks, ds, nch, part_s, part_cnt, part_j, c32, c64, j_sub, aop, cmax, mu, s);
}

int launch_finalize(int m, int ks, int ds, int nch, const double* part_s, const uint32_t* part_cnt,
                    const double* part_j, float* c32, double* c64, double* j_sub, void* aop, float* cmax,
                    const float* mu, hipStream_t s) {
  const int nt = tiles_for(ks);
  ProfScope ps(MIPQ_K_FINALIZE, s);
  if (!aop) {
    k_finalize<<<m, kUpdThreads, 0, s>>>(m, ks, ds, nch, part_s, part_cnt, part_j, c32, c64, j_sub);
  } else {   // matrix-core operands: every (tile, subspace) block at once
    dim3 grid(nt, m);
    if (ds <= 8)
      k_finalize_tiles<1><<<grid, kFinTileThreads, 0, s>>>(m, ks, ds, nch, part_s, part_cnt, part_j, c32, c64, j_sub,
                                                            (uint4*)aop, cmax, mu, nt);
    else
      k_finalize_tiles<2><<<grid, kFinTileThreads, 0, s>>>(m, ks, ds, nch, part_s, part_cnt, part_j, c32, c64, j_sub,
                                                            (uint4*)aop, cmax, mu, nt);
  }
  MIPQ_LAUNCHED("k_finalize");
  return MIPQ_OK;
}

int backward_chunks(int64_t n, int m) {
  int nch = ceil_div(n, 2048);
  int cap = 2048 / m;
  if (cap < 1) cap = 1;
  if (nch > cap) nch = cap;
  return nch < 1 ? 1 : nch;
}

int launch_backward(const float* x, int64_t n, int d, int m, int ks, const uint8_t* codes,
                    const float* c32, const double* gscale, float* grad_x, float* grad_c, int nch,
                    double* part_s, uint32_t* part_cnt, double* part_j, double* loss_sub, hipStream_t s) {
  const int ds = d / m;
  const int64_t rpc = (n + nch - 1) / nch;
  // several subspaces per block when a row's slices of them are whole
  // 16-byte pieces and their LDS fits a block
  int G = 1;
  if (ds % 4 == 0 && rows_vec4(x, d, ds) && (!grad_x || rows_vec4(grad_x, d, ds))) {
    int dev = 0, lds_max = 65536;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      lds_max = 65536;
    for (int g = 4; g >= 2; g >>= 1)
      if (m % g == 0 && (g * ds / 4) <= 64 && group4_lds_bytes(ks, ds, g) <= (size_t)lds_max) {
        G = g;
        break;
      }
  }
  if (G > 1) {
    const unsigned grid = (unsigned)(((nch + 7) / 8) * 8 * (m / G));
    const size_t shm = group4_lds_bytes(ks, ds, G);
    ProfScope ps(MIPQ_K_BACKWARD, s);
#define BG(GV)                                                                                                 \
  do {                                                                                                         \
    if (grad_x)                                                                                                \
      k_backward_group<true, GV><<<grid, kBwdThreads, shm, s>>>(x, n, d, m, ks, ds, codes, c32, rpc, nch,        \
                                                              part_s, part_cnt, part_j, gscale, grad_x);       \
    else                                                                                                       \
      k_backward_group<false, GV><<<grid, kBwdThreads, shm, s>>>(x, n, d, m, ks, ds, codes, c32, rpc, nch,       \
                                                               part_s, part_cnt, part_j, nullptr, nullptr);    \
  } while (0)
    if (G == 4) BG(4);
    else BG(2);
#undef BG
    MIPQ_LAUNCHED("k_backward_group");
  } else {
    const size_t shm = (size_t)ks * (ds + 1) * sizeof(double) + ((ks + 1) / 2) * sizeof(double) +
                       (size_t)ks * ds * sizeof(float);
    const unsigned grid = (unsigned)(((nch + 7) / 8) * 8 * m);
    ProfScope ps(MIPQ_K_BACKWARD, s);
    if (grad_x)
      k_accumulate<true, true, true, kBwdThreads><<<grid, kBwdThreads, shm, s>>>(
          x, n, d, m, ks, ds, codes, c32, rpc, nch, part_s, part_cnt, part_j, gscale, grad_x, nullptr);
    else
      k_accumulate<false, true, true, kBwdThreads><<<grid, kBwdThreads, shm, s>>>(
          x, n, d, m, ks, ds, codes, c32, rpc, nch, part_s, part_cnt, part_j, nullptr, nullptr, nullptr);
    MIPQ_LAUNCHED("k_accumulate");
  }
  k_grad_codebook<<<m, kUpdThreads, 0, s>>>(m, ks, ds, nch, part_s, part_cnt, part_j, c32, gscale, grad_c,
                                            loss_sub);
  MIPQ_LAUNCHED("k_grad_codebook");
  return MIPQ_OK;
}

int launch_pack_bf16(const float* c32, int m, int ks, int ds, void* aop, float* cmax, float* mu,
                     hipStream_t s) {
  const int nt = tiles_for(ks);
  ProfScope ps(MIPQ_K_PACK_BF16, s);
  dim3 grid(nt, m);
  if (ds <= 8)
    k_pack_bf16<1><<<grid, kPackThreads, 0, s>>>(c32, ks, ds, nt, (uint4*)aop, cmax, mu);
  else
    k_pack_bf16<2><<<grid, kPackThreads, 0, s>>>(c32, ks, ds, nt, (uint4*)aop, cmax, mu);
  MIPQ_LAUNCHED("k_pack_bf16");
  return MIPQ_OK;
}

int launch_pack_bf16_batched(const BatchProb* probs, int nprob, int m, int ks, int ds, void* aop,
                             size_t aop_stride, float* cmax, float* mu, hipStream_t s) {
  const int nt = tiles_for(ks);
  ProfScope ps(MIPQ_K_PACK_BF16, s);
  dim3 grid(nt, m, nprob);
  if (ds <= 8)
    k_pack_bf16_batched<1><<<grid, kPackThreads, 0, s>>>(probs, ks, ds, m, nt, (uint4*)aop, aop_stride, cmax, mu);
  else
    k_pack_bf16_batched<2><<<grid, kPackThreads, 0, s>>>(probs, ks, ds, m, nt, (uint4*)aop, aop_stride, cmax, mu);
  MIPQ_LAUNCHED("k_pack_bf16_batched");
  return MIPQ_OK;
}

int launch_update_batched(const BatchProb* probs, int nprob, int64_t items, int d, int m, int ks, double* c64,
                          double* part_s, uint32_t* part_cnt, double* part_j, double* j_all,
                          const uint32_t* round, int iters, void* aop, size_t aop_stride, float* cmax, float* mu,
                          bool det, bool accumulate, float* tmax, hipStream_t s) {
  const int ds = d / m;
  if (accumulate) {
    const size_t shm = (size_t)ks * (ds + 1) * sizeof(double) + ((ks + 1) / 2) * sizeof(double) +
                       (size_t)ks * ds * sizeof(float);
    ProfScope ps(MIPQ_K_UPDATE, s);
    const int64_t chunks = items / m;
    const unsigned grid = (unsigned)(((chunks + 7) / 8) * 8 * m);
    if (det)
      k_accumulate_batched<true, kDetThreads><<<grid, kDetThreads, det_lds_bytes(ks, ds, true), s>>>(
          probs, nprob, items, d, m, ks, ds, part_s, part_cnt, part_j);
    else
      k_accumulate_batched<false, kUpdThreads><<<grid, kUpdThreads, shm, s>>>(probs, nprob, items, d, m, ks, ds,
                                                                              part_s, part_cnt, part_j);
    MIPQ_LAUNCHED("k_accumulate_batched");
  }
  const int nt = tiles_for(ks);
  ProfScope ps(MIPQ_K_FINALIZE, s);
  dim3 grid(nt, m, nprob);
  if (ds <= 8)
    k_finalize_tiles_batched<1><<<grid, kFinTileThreads, 0, s>>>(probs, nprob, m, ks, ds, part_s, part_cnt, part_j,
                                                                 c64, j_all, round, iters, (uint4*)aop, aop_stride,
                                                                 cmax, mu, nt, tmax);
  else
    k_finalize_tiles_batched<2><<<grid, kFinTileThreads, 0, s>>>(probs, nprob, m, ks, ds, part_s, part_cnt, part_j,
                                                                 c64, j_all, round, iters, (uint4*)aop, aop_stride,
                                                                 cmax, mu, nt, tmax);
  MIPQ_LAUNCHED("k_finalize_tiles_batched");
  const int count = nprob * m;
  k_next_round_batched<<<(count + 255) / 256, 256, 0, s>>>(const_cast<uint32_t*>(round), tmax, cmax, count, nt);
  MIPQ_LAUNCHED("k_next_round_batched");
  return MIPQ_OK;
}

}  // namespace mipq
