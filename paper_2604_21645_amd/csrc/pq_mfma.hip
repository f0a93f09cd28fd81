// Per-subspace nearest-centroid assignment on gfx950 matrix cores.
//
// Paper Section 2.1: every row of every subspace is assigned to its nearest
// of Ks subspace centroids (the inner step of the k-means fit and the whole
// of encoding).  For squared Euclidean distance the ranking of candidates k
// for a fixed row only needs
//     s_k = ||c_k||^2 - 2 x . c_k ,
// a dense contraction over the subspace dimensions, which runs here as
// 32x32x16 bfloat16 MFMAs with float32 accumulation:
//   * x and -2c are split into high and low bfloat16 parts (v = hi + lo + e,
//     |e| <= 2^-16 |v|); the MFMA sums hi*hi + hi*lo + lo*hi over the
//     dimensions, and ||c||^2 and ||x||^2 enter the same contraction as three
//     bfloat16 pieces each multiplied by ones, so the accumulator starts at
//     zero and ends at an estimate of the distance itself (>= -error);
//   * layout: A = centroid operands (32 centroids x K), B = row operands
//     (K x 32 rows); lane l receives row l%32 and, for each of the 8 tiles
//     of 32 centroids, 16 scores (centroids 8*(r/4) + 4*(l/32) + r%4);
//   * each lane reduces its 128 scores with two groupings -- by tile and by
//     accumulator register -- whose minima give the best score, its tile and
//     register (hence its index), and the runner-up (any two candidates of
//     one lane differ in tile or in register);
//   * the lane pair (l, l^32) merges; if the gap between best and runner-up
//     does not exceed a proven bound on the error of the scores plus the
//     rounding of the exact rule, the whole wave re-decides that (row,
//     subspace) with the exact float32 rule.  Otherwise the matrix-core winner
//     IS the exact rule's unique winner.
#include <math.h>

#include "bf16_pack.h"
#include "mipq_internal.h"

namespace mipq {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kThreads = 256;   // 4 waves, one subspace each
// row tiles per block of the assignment with fused outputs: its LDS (lists,
// the block's centroids, stashes) then fits three blocks per CU
constexpr int kOutTiles = 32;

// LDS of k_fit_round_bf16: sums [ks][ds + 1] float64 and counts [ks], then
// (16-byte aligned) the waves' stashes, the block's 16-bit pending list and
// two counters (the next 64-row step, the list's length)
__host__ __device__ constexpr size_t fit_lds_stash_offset(int ks, int ds) {
  return ((size_t)ks * (ds + 1) * sizeof(double) + (size_t)ks * sizeof(uint32_t) + 15) & ~size_t(15);
}
// its waves per block: three per SIMD for one 8-dimension block (about 168
// VGPRs), one per SIMD for two (up to 256 VGPRs)
__host__ __device__ constexpr int fit_waves(int nb) { return nb == 1 ? 12 : 4; }

// ---- row side --------------------------------------------------------------
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

__device__ __forceinline__ float min3f(float a, float b, float c) { return fminf(fminf(a, b), c); }

__device__ __forceinline__ float min16(const f32x16& a) {
  const float m0 = min3f(a[0], a[1], a[2]);
  const float m1 = min3f(a[3], a[4], a[5]);
  const float m2 = min3f(a[6], a[7], a[8]);
  const float m3 = min3f(a[9], a[10], a[11]);
  const float m4 = min3f(a[12], a[13], a[14]);
  return fminf(min3f(m0, m1, m2), min3f(m3, m4, a[15]));
}

// Lexicographic (value, index) minimum over the 64 lanes, returned on every
// lane: the smallest value (float minimum), then the smallest index among the
// lanes holding it.  Within 16-lane rows by DPP (quad swaps, half-row and row
// mirrors), across rows by v_permlane16_swap and v_permlane32_swap: no LDS
// round trips (ds_bpermute) on the re-decision's critical path.
__device__ __forceinline__ float dpp_minf(float v) {
  auto step = [](float a, int b) { return fminf(a, __int_as_float(b)); };
  v = step(v, __builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0xB1, 0xF, 0xF, false));  // quad [1,0,3,2]
  v = step(v, __builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0x4E, 0xF, 0xF, false));  // quad [2,3,0,1]
  v = step(v, __builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0x141, 0xF, 0xF, false)); // half-row mirror
  v = step(v, __builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0x140, 0xF, 0xF, false)); // row mirror
  const auto r16 = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  v = fminf(__uint_as_float(r16[0]), __uint_as_float(r16[1]));
  const auto r32 = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return fminf(__uint_as_float(r32[0]), __uint_as_float(r32[1]));
}
__device__ __forceinline__ int dpp_mini(int v) {
  v = min(v, __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false));
  v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xF, 0xF, false));
  v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x141, 0xF, 0xF, false));
  v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x140, 0xF, 0xF, false));
  const auto r16 = __builtin_amdgcn_permlane16_swap((unsigned)v, (unsigned)v, false, false);
  v = min((int)r16[0], (int)r16[1]);
  const auto r32 = __builtin_amdgcn_permlane32_swap((unsigned)v, (unsigned)v, false, false);
  return min((int)r32[0], (int)r32[1]);
}
__device__ __forceinline__ void wave_argmin(float& best, int& bk) {
  const float m = dpp_minf(best);
  bk = dpp_mini(best == m ? bk : 0x7FFFFFFF);
  best = m;
}

// set bits of a wave-wide mask below the calling lane (v_mbcnt: no lane mask
// kept in registers)
__device__ __forceinline__ int lanes_below(uint64_t mask) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// signed-integer key: the float's bits with its low bits replaced by an index;
// for non-negative floats integer order is float order (up to the replaced bits)
__device__ __forceinline__ int key_of(float v, int mask, int idx) {
  return (__float_as_int(v) & mask) | idx;
}

// median of three signed ints (v_med3_i32)
__device__ __forceinline__ int med3i(int a, int b, int c) { return max(min(a, b), min(max(a, b), c)); }

// values of lane l%32 (.x) and lane 32 + l%32 (.y), for every lane
__device__ __forceinline__ int2 halves(int v) {
  const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
  return make_int2((int)r[0], (int)r[1]);
}

// a wave-uniform 64-bit value moved to scalar registers
__device__ __forceinline__ int64_t uniform64(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

struct XcdMap {
  int rowblk, group;
};
__device__ __forceinline__ XcdMap xcd_map(int lin, int groups) {
  const int xcd = lin & 7;
  const int slot = lin >> 3;
  XcdMap r;
  r.group = slot % groups;
  r.rowblk = (slot / groups) * 8 + xcd;
  return r;
}

// Exact float32 rule for one (row, subspace) by the whole wave: lane i scans
// centroids i, i+64, ... in ascending order, then a lexicographic (distance,
// index) minimum over the lanes.  Dimensions t >= ds contribute exact zeros, so
// the sums equal the ds-term sums of the plain path bit for bit.
template <int DW>
__device__ __forceinline__ int exact_code_wave(const float* __restrict__ xr, const float* __restrict__ cb,
                                               int ds, int ks, int lane) {
  float xo[DW];
#pragma unroll
  for (int t = 0; t < DW; ++t) {
    const float v = xr[t < ds ? t : ds - 1];
    xo[t] = t < ds ? v : 0.0f;
  }
  float best = INFINITY;
  int bk = 0x7FFFFFFF;
  for (int k = lane; k < ks; k += 64) {
    const float* c = cb + (int64_t)k * ds;
    float acc = 0.0f;
#pragma unroll
    for (int t = 0; t < DW; ++t) {
      const float cv = c[t < ds ? t : ds - 1];
      const float df = xo[t] - (t < ds ? cv : 0.0f);
      const float sq = df * df;
      acc = acc + sq;
    }
    if (acc < best) {
      best = acc;
      bk = k;
    }
  }
  wave_argmin(best, bk);
  return bk < ks ? bk : 0;
}

// Centroid-side state of one subspace, held in registers while a wave walks a
// range of rows: the packed operands, the centre mu (scalar registers) and the
// bound on the centred centroid norms.
template <int NB, int NT>
struct SubOps {
  static constexpr int NMF = bf16_nmfma(NB);
  static constexpr int DW = NB * 8;
  bf16x8 A[NT][NMF];
  float muv[DW];
  float cm;
};

template <int NB, int NT>
__device__ __forceinline__ void load_sub_ops(SubOps<NB, NT>& o, const bf16x8* __restrict__ aop,
                                             const float* __restrict__ cmax, const float* __restrict__ mu,
                                             int sub, int lane) {
  constexpr int NMF = SubOps<NB, NT>::NMF;
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int f = 0; f < NMF; ++f) o.A[t][f] = aop[((size_t)(sub * NT + t) * NMF + f) * 64 + lane];
  o.cm = cmax[sub];
#pragma unroll
  for (int e = 0; e < NB * 8; ++e)
    o.muv[e] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(mu[sub * kMaxDsBf16 + e])));
}

// error-bound constants of the separation test (see launch_assign_bf16)
struct Band {
  float e_cross, e_norm, g_exact;
};

// Raw slice of row r0 + lane%32 (clamped to r0 past the end) of subspace sub.
template <int DW, bool FULL>
__device__ __forceinline__ void load_rows(float (&xv)[DW], const float* __restrict__ x, int64_t r0, int64_t rend,
                                          int d, int sub, int ds, int lane) {
  const int64_t row = r0 + (lane & 31);
  const float* xr = x + (row < rend ? row : r0) * d + (int64_t)sub * ds;
  if (FULL) {   // ds == DW and 16-byte aligned rows: vector loads
#pragma unroll
    for (int e = 0; e < DW; e += 4) {
      const float4 v = *reinterpret_cast<const float4*>(xr + e);
      xv[e] = v.x;
      xv[e + 1] = v.y;
      xv[e + 2] = v.z;
      xv[e + 3] = v.w;
    }
  } else {   // clamped loads, then zero the padding dimensions
#pragma unroll
    for (int e = 0; e < DW; ++e) {
      const float v = xr[e < ds ? e : ds - 1];
      xv[e] = (e < ds) ? v : 0.0f;
    }
  }
}

// Reduction of the NT tiles of 32-centroid estimates of one row (lanes l and
// l^32): the best estimate f1, the runner-up f2 and the index of the best.
// Each lane reduces its 16*NT values with two groupings -- by tile (amin) and
// by accumulator register (bmin) -- whose minima give the best value, its tile
// and register (hence its index), and the runner-up (two candidates of one
// lane differ in tile or in register); then the lane pair merges.
template <int NT, class TileFn>
__device__ __forceinline__ void lane_keys(TileFn tile, int& a1o, int& s2o, int& rlo) {
  float amin[NT];
  float bmin[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) bmin[r] = INFINITY;
#pragma unroll
  for (int t = 0; t < NT; t += 2) {
    const f32x16 c0 = tile(t);
    amin[t] = min16(c0);
    if (t + 1 < NT) {
      const f32x16 c1 = tile(t + 1 < NT ? t + 1 : 0);
      amin[t + 1] = min16(c1);
#pragma unroll
      for (int r = 0; r < 16; ++r) bmin[r] = min3f(bmin[r], c0[r], c1[r]);
    } else {
#pragma unroll
      for (int r = 0; r < 16; ++r) bmin[r] = fminf(bmin[r], c0[r]);
    }
  }

  // smallest two keys of each grouping; the low bits carry the tile
  // (3 bits) or the register (4 bits)
  int a1 = INT_MAX, a2 = INT_MAX, b1 = INT_MAX, b2 = INT_MAX;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int k = key_of(amin[t], ~7, t);
    a2 = min(a2, max(a1, k));
    a1 = min(a1, k);
  }
#pragma unroll
  for (int r = 0; r < 16; r += 2) {
    const int ka = key_of(bmin[r], ~15, r);
    const int kb = key_of(bmin[r + 1], ~15, r + 1);
    b2 = min(b2, med3i(ka, kb, b1));   // runner-up of {b1, b2, ka, kb}, b1 <= b2
    b1 = min(b1, min(ka, kb));
  }
  a1o = a1;
  s2o = min(a2, b2);
  rlo = b1 & 15;
}

// Merge of the keys of the two lanes holding one row's candidates (x: the
// lane of half 0, y: half 1): best estimate f1, runner-up f2, winning index.
__device__ __forceinline__ int merge_keys(int a1x, int a1y, int s2x, int s2y, int rlx, int rly, float& f1,
                                          float& f2) {
  const bool hiw = a1y < a1x;
  const int w1 = min(a1x, a1y);
  const int sec = min(max(a1x, a1y), min(s2x, s2y));
  const int tw = (hiw ? a1y : a1x) & 7;
  const int rw = hiw ? rly : rlx;
  f1 = __int_as_float(w1);
  f2 = __int_as_float(sec);
  return tw * 32 + (rw >> 2) * 8 + (hiw ? 4 : 0) + (rw & 3);
}

template <int NT, class TileFn>
__device__ __forceinline__ int reduce_scores(TileFn tile, float& f1, float& f2) {
  int a1, s2, rl;
  lane_keys<NT>(tile, a1, s2, rl);
  const int2 A1 = halves(a1);
  const int2 S2 = halves(s2);
  const int2 RL = halves(rl);
  return merge_keys(A1.x, A1.y, S2.x, S2.y, RL.x, RL.y, f1, f2);
}

// Separation test: true when the two best estimates f1 <= f2 (error at most
// beta each) may not order the exact rule's distances; q covers the key
// truncation and the exact rule's rounding (g relative), xn the row norm.
__device__ __forceinline__ bool not_separated(float f1, float f2, float beta, float g, float xn) {
  const float q = 3.815e-6f + g;   // 2^-18 + g
  const float thr = 2.0f * beta + q * (fabsf(f1) + fabsf(f2)) + 2.0f * g * (beta + g * xn);
  return !(f2 - f1 > thr);
}

// Fused Lloyd accumulation (k_fit_round_bf16): the block's float64 sums of
// its rows by code, S [ks][ds + 1] (one padding double per centroid spreads a
// centroid's dimensions over the LDS banks) and counts cnt [ks], and the
// wave's stash of its lanes' row slices, [DW / 4][64] float4 (lane-minor, so
// that a wave's 16-byte stores and loads are contiguous).
struct AccLds {
  double* S = nullptr;
  uint32_t* cnt = nullptr;
  float4* stash = nullptr;
};

// one row's slice v (dimensions t < ds) added to centroid code's sums
template <int DW>
__device__ __forceinline__ void acc_row(const AccLds& a, int code, const float (&v)[DW], int ds) {
  double* sc = a.S + code * (ds + 1);
#pragma unroll
  for (int t = 0; t < DW; ++t)
    if (t < ds) atomicAdd(sc + t, (double)v[t]);
  atomicAdd(a.cnt + code, 1u);
}

// The exact rule for the np pending rows (rows base + pend[i]) of subspace
// sub by the whole wave, one row after another; overwrites their codes.  Lane
// i holds centroids i, i+64, i+128, i+192 (ks <= 256) in registers for all the
// rows, and the next row's slice is loaded while the current one is decided:
// per row the wave computes the ks distances (float32, dimensions ascending,
// unfused; padding dimensions add exact zeros) and takes the lexicographic
// (distance, index) minimum over the lanes.
// REG false (kernels with no registers to spare): the rows one at a time with
// the centroids read for each row (exact_code_wave), the same arithmetic.
// OUT (REG only): also the exact distance of the winner (min_dist, optional)
// and the float64 squared error of the row's subspace block, added to *sse
// by lane 0.  ACC (REG only): lane 0 adds the row to the block's sums.
template <int DW, bool REG, bool OUT = false, bool ACC = false, class P = uint32_t>
__device__ __forceinline__ void redecide(const P* pend, int64_t base, int np, const float* __restrict__ x, int d,
                                         int m, int ks, int ds, int sub, const float* __restrict__ cbsub,
                                         uint8_t* __restrict__ codes, int lane, float* __restrict__ min_dist = nullptr,
                                         double* sse = nullptr, const AccLds& acc = AccLds()) {
  static_assert(REG || (!OUT && !ACC), "the fused outputs need the register form");
  if (np == 0) return;   // wave-uniform
  if (!REG) {
    for (int i = 0; i < np; ++i) {
      const int64_t prow = base + pend[i];
      const int ec = exact_code_wave<DW>(x + prow * d + (int64_t)sub * ds, cbsub, ds, ks, lane);
      if (lane == 0) codes[prow * m + sub] = (uint8_t)ec;
    }
    return;
  }
  constexpr int KPL = kMaxKs / 64;
  float cv[KPL][DW];
  // whole 16-byte centroid rows when ds fills the register block
  const bool vec = ds == DW && (reinterpret_cast<uintptr_t>(cbsub) & 15) == 0;
#pragma unroll
  for (int j = 0; j < KPL; ++j) {
    const int k = lane + 64 * j;
    const float* c = cbsub + (int64_t)(k < ks ? k : 0) * ds;
    if (vec) {
#pragma unroll
      for (int t = 0; t < DW; t += 4) {
        const float4 v = *reinterpret_cast<const float4*>(c + t);
        cv[j][t] = k < ks ? v.x : 0.0f;
        cv[j][t + 1] = k < ks ? v.y : 0.0f;
        cv[j][t + 2] = k < ks ? v.z : 0.0f;
        cv[j][t + 3] = k < ks ? v.w : 0.0f;
      }
    } else {
#pragma unroll
      for (int t = 0; t < DW; ++t) {
        const float v = c[t < ds ? t : ds - 1];
        cv[j][t] = (k < ks && t < ds) ? v : 0.0f;
      }
    }
  }
  auto load_x = [&](int64_t row, float (&xo)[DW]) {
    const float* xr = x + row * d + (int64_t)sub * ds;
#pragma unroll
    for (int t = 0; t < DW; ++t) {
      const float v = xr[t < ds ? t : ds - 1];
      xo[t] = t < ds ? v : 0.0f;
    }
  };
  float xn[DW];
  load_x(base + pend[0], xn);
  for (int i = 0; i < np; ++i) {
    const int64_t prow = base + pend[i];
    float xo[DW];
#pragma unroll
    for (int t = 0; t < DW; ++t) xo[t] = xn[t];
    if (i + 1 < np) load_x(base + pend[i + 1], xn);   // next row in flight
    float best = INFINITY;
    int bk = 0x7FFFFFFF;
#pragma unroll
    for (int j = 0; j < KPL; ++j) {
      const int k = lane + 64 * j;
      float acc = 0.0f;
#pragma unroll
      for (int t = 0; t < DW; ++t) {
        const float df = xo[t] - cv[j][t];
        const float sq = df * df;
        acc = acc + sq;
      }
      if (k < ks && acc < best) {
        best = acc;
        bk = k;
      }
    }
    wave_argmin(best, bk);
    const int code = bk < ks ? bk : 0;
    if (lane == 0) {
      if (codes) codes[prow * m + sub] = (uint8_t)code;
      if (ACC) acc_row<DW>(acc, code, xo, ds);
      if (OUT) {
        if (min_dist) min_dist[prow * m + sub] = best;
        const float* c = cbsub + (int64_t)code * ds;
        double sq = 0.0;
#pragma unroll
        for (int t = 0; t < DW; ++t)
          if (t < ds) {
            const double dd = (double)xo[t] - (double)c[t];
            sq = sq + dd * dd;
          }
        *sse += sq;
      }
    }
  }
}

// One wave assigns rows [rb, re) of subspace sub, 32 rows at a time (lane l
// and l^32 share row l%32), the next tile's rows in flight.  Ambiguous rows
// are queued in the wave's LDS list and re-decided with the exact rule after
// the loop (and, with MIDFLUSH, whenever more than flush_at are queued).
// Returns the number of re-decided rows.
template <int DW, bool FULL, bool MIDFLUSH, bool REG, class Decide>
__device__ __forceinline__ uint32_t assign_rows(const float* __restrict__ x, int d, int ds, int m, int ks, int sub,
                                                int64_t rb, int64_t re, Decide decide,
                                                const float* __restrict__ cbsub, uint8_t* __restrict__ codes,
                                                uint32_t* pend, int flush_at, int lane) {
  const int half = lane >> 5;
  uint32_t nres = 0;
  int np = 0;
  float xnext[DW];
  load_rows<DW, FULL>(xnext, x, rb, re, d, sub, ds, lane);
  for (int64_t r0 = rb; r0 < re; r0 += 32) {
    if (MIDFLUSH && np > flush_at) {
      redecide<DW, REG>(pend, 0, np, x, d, m, ks, ds, sub, cbsub, codes, lane);
      nres += (uint32_t)np;
      np = 0;
    }
    const int64_t row = r0 + (lane & 31);
    const bool valid = row < re;
    float xv[DW];
#pragma unroll
    for (int e = 0; e < DW; ++e) xv[e] = xnext[e];
    if (r0 + 32 < re) load_rows<DW, FULL>(xnext, x, r0 + 32, re, d, sub, ds, lane);   // next tile in flight
    bool amb;
    const int code = decide(xv, half, amb);
    // rows whose two best candidates are not separated are re-decided by the
    // whole wave with the exact rule (rare); their codes are overwritten then
    if (half == 0 && valid) codes[row * m + sub] = (uint8_t)code;
    const bool push = (half == 0) && valid && amb;
    const uint64_t mask = __ballot(push);
    if (mask) {
      if (push) pend[np + lanes_below(mask)] = (uint32_t)row;
      np += __popcll(mask);
    }
  }
  redecide<DW, REG>(pend, 0, np, x, d, m, ks, ds, sub, cbsub, codes, lane);
  return nres + (uint32_t)np;
}

typedef int i32x4 __attribute__((ext_vector_type(4)));

// Row-side operand parts of one row: its slice centred by mu, the squared
// norm xn of the centred slice (float32, dimensions ascending), the
// bfloat16 high parts XH and low parts XL (of the remainders), and normB =
// [1, 1, 1, xn_hi, xn_mid, xn_lo, 0, 0], the pieces of xn against the ones of
// the centroid norm slots (see bf16_pack.h for the operand layout).
template <int NB>
struct RowParts {
  bf16x8 XH[NB], XL[NB], normB;
  float xn;
};

template <int NB>
__device__ __forceinline__ void row_parts(const float (&xraw)[NB * 8], const float (&muv)[NB * 8],
                                          RowParts<NB>& r) {
  constexpr int DW = NB * 8;
  float xv[DW];
#pragma unroll
  for (int e = 0; e < DW; ++e) xv[e] = xraw[e] - muv[e];
  float xn = 0.0f;
#pragma unroll
  for (int e = 0; e < DW; ++e) xn = xn + xv[e] * xv[e];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    r.XH[b] = to_bf16x8(xv + b * 8);
    float rem[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) rem[e] = xv[b * 8 + e] - (float)r.XH[b][e];
    r.XL[b] = to_bf16x8(rem);
  }
  const __bf16 h = (__bf16)xn;
  const float r1 = xn - (float)h;
  const __bf16 md = (__bf16)r1;
  r.normB = bf16x8{};
  r.normB[0] = r.normB[1] = r.normB[2] = (__bf16)1.0f;
  r.normB[3] = h;
  r.normB[4] = md;
  r.normB[5] = (__bf16)(r1 - (float)md);
  r.xn = xn;
}

// [p.lo | q.lo] and [p.hi | q.hi] (lo: lanes 0-31, hi: lanes 32-63), one
// v_permlane32_swap per dword
__device__ __forceinline__ void swap_halves(const bf16x8& p, const bf16x8& q, bf16x8& lo, bf16x8& hi) {
  const i32x4 pi = __builtin_bit_cast(i32x4, p), qi = __builtin_bit_cast(i32x4, q);
  i32x4 a, b;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const auto r = __builtin_amdgcn_permlane32_swap(pi[w], qi[w], false, false);
    a[w] = (int)r[0];
    b[w] = (int)r[1];
  }
  lo = __builtin_bit_cast(bf16x8, a);
  hi = __builtin_bit_cast(bf16x8, b);
}
__device__ __forceinline__ void swap_halves(int p, int q, int& lo, int& hi) {
  const auto r = __builtin_amdgcn_permlane32_swap(p, q, false, false);
  lo = (int)r[0];
  hi = (int)r[1];
}

// Row operands of both 32-row groups of a 64-row step from the lanes' own
// rows (lanes 0-31: group A, 32-63: group B).  MFMA f takes P_f of the row
// on lanes 0-31 and Q_f on lanes 32-63 (bf16_pack.h: [xh | xh] for the
// first NB, [xl_b | xl_b+1 or normB] for the pairs, [normB | 0] last); a
// swap of P_f with Q_f leaves [P_f(A) | Q_f(A)] and [P_f(B) | Q_f(B)].
template <int NB>
__device__ __forceinline__ void row_operands(const RowParts<NB>& r, bf16x8 (&BA)[bf16_nmfma(NB)],
                                             bf16x8 (&BB)[bf16_nmfma(NB)]) {
  constexpr int NMF = bf16_nmfma(NB);
  const bf16x8 zero8 = {};
#pragma unroll
  for (int f = 0; f < NMF; ++f) {
    bf16x8 P, Q;
    if (f < NB) {
      P = r.XH[f];
      Q = r.XH[f];
    } else if (f < NB + (NB + 1) / 2) {
      const int b0 = 2 * (f - NB);
      P = r.XL[b0];
      Q = (b0 + 1 < NB) ? r.XL[b0 + 1 < NB ? b0 + 1 : 0] : r.normB;
    } else {
      P = r.normB;
      Q = zero8;
    }
    swap_halves(P, Q, BA[f], BB[f]);
  }
}

// Raw subspace slice of row r0 + lane (clamped to r0 past rend).  Without
// whole 8-dimension blocks, an even ds on 8-byte aligned rows is read in pairs
// of floats (the last pair repeated past ds), else one float at a time.
template <int DW, bool FULL>
__device__ __forceinline__ void load_own_row(float (&xv)[DW], const float* __restrict__ x, int64_t r0, int64_t rend,
                                             int d, int sub, int ds, int lane) {
  const int64_t row = r0 + lane;
  const float* xr = x + (row < rend ? row : r0) * d + (int64_t)sub * ds;
  if (FULL) {
#pragma unroll
    for (int e = 0; e < DW; e += 4) {
      const float4 v = *reinterpret_cast<const float4*>(xr + e);
      xv[e] = v.x;
      xv[e + 1] = v.y;
      xv[e + 2] = v.z;
      xv[e + 3] = v.w;
    }
  } else if ((ds & 1) == 0 && (reinterpret_cast<uintptr_t>(x) & 7) == 0) {
#pragma unroll
    for (int e = 0; e < DW; e += 2) {
      const float2 v = *reinterpret_cast<const float2*>(xr + (e < ds ? e : ds - 2));
      xv[e] = (e < ds) ? v.x : 0.0f;
      xv[e + 1] = (e < ds) ? v.y : 0.0f;
    }
  } else {
#pragma unroll
    for (int e = 0; e < DW; ++e) {
      const float v = xr[e < ds ? e : ds - 1];
      xv[e] = (e < ds) ? v : 0.0f;
    }
  }
}

// Rows [rb, re) of subspace sub by one wave, 64 rows per step; lane l owns
// row r0 + l (lanes 0-31 form the step's first 32-row group A, lanes 32-63
// the second, B).  Every lane prepares the operand parts of its own row;
// row_operands hands each lane its half's operands in both groups; both
// groups' tiles run on the matrix cores and each lane reduces its half of the
// candidates of group A's and group B's row (lane_keys); one swap per key
// brings the two halves of a row to the row's own lane, so the merge, the
// separation test, the code store (none with codes NULL) and (OUT) the
// distance of the chosen centroid and its float64 squared error run once per
// row.  Ambiguous rows
// are queued in the wave's LDS list `pend` as offsets from rb (room for
// re - rb <= 65536 entries) and re-decided by the whole wave after the loop.  Returns the number of
// re-decided rows; OUT adds the squared errors to *sse (lane-local sums); ACC
// adds every row, once its code is final, to the block's sums (AccLds).
// DYN: [rb, re) is the block's range, shared by its waves: each wave claims
// the next 64-row step from the counter dyn[0] (so the waves of a SIMD end
// together however the SIMD shares its issue slots among them) and appends
// its ambiguous rows to the block's list pend (count dyn[1]), which the waves
// re-decide together once all are done (a barrier: every wave of the block
// must call).  Returns the block's number of ambiguous rows.
__device__ __forceinline__ int claim_step(int* ctr, int lane) {
  int v = 0;
  if (lane == 0) v = atomicAdd(ctr, 1);
  return __builtin_amdgcn_readfirstlane(v);
}
template <int NB, int NT, bool FULL, bool OUT, bool REG, bool ACC = false, bool DYN = false>
__device__ __forceinline__ int assign_rows64(const SubOps<NB, NT>& o, const Band& bd, const float* __restrict__ x,
                                             int d, int ds, int m, int ks, int sub, int64_t rb, int64_t re,
                                             const float* __restrict__ cbsub, uint8_t* __restrict__ codes,
                                             uint16_t* pend, int lane, float* __restrict__ min_dist,
                                             double* sse, const AccLds& acc = AccLds(), int* dyn = nullptr) {
  static_assert(!(ACC && OUT), "one fused output at a time");
  static_assert(!DYN || ACC, "the shared steps are the fused round's");
  constexpr int DW = NB * 8;
  constexpr int NMF = bf16_nmfma(NB);
  int np = 0;
  const int nsteps = DYN ? (int)((re - rb + 63) / 64) : 0;
  int step = DYN ? claim_step(dyn, lane) : 0;
  float xnext[DW];
  if (!DYN || step < nsteps) load_own_row<DW, FULL>(xnext, x, rb + (int64_t)step * 64, re, d, sub, ds, lane);
  for (int64_t r0 = rb + (int64_t)step * 64; DYN ? step < nsteps : r0 < re;) {
    float xv[DW];
#pragma unroll
    for (int e = 0; e < DW; ++e) xv[e] = xnext[e];
    // the next step's row in flight
    int64_t rnext;
    if (DYN) {
      step = claim_step(dyn, lane);
      rnext = rb + (int64_t)step * 64;
      if (step < nsteps) load_own_row<DW, FULL>(xnext, x, rnext, re, d, sub, ds, lane);
    } else {
      rnext = r0 + 64;
      if (rnext < re) load_own_row<DW, FULL>(xnext, x, rnext, re, d, sub, ds, lane);
    }
    const int64_t row = r0 + lane;
    const bool valid = row < re;
    if (ACC || (OUT && NB == 1)) {   // the slice waits in LDS until the row's code is known
#pragma unroll
      for (int e = 0; e < DW; e += 4) acc.stash[(e >> 2) * 64 + lane] = make_float4(xv[e], xv[e + 1], xv[e + 2], xv[e + 3]);
    }
    RowParts<NB> rp;
    row_parts<NB>(xv, o.muv, rp);
    bf16x8 BA[NMF], BB[NMF];
    row_operands<NB>(rp, BA, BB);
    int a1A, s2A, rlA, a1B, s2B, rlB;
    lane_keys<NT>([&](int t) {
      f32x16 acc = {};
#pragma unroll
      for (int f = 0; f < NMF; ++f) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o.A[t][f], BA[f], acc, 0, 0, 0);
      return acc;
    }, a1A, s2A, rlA);
    lane_keys<NT>([&](int t) {
      f32x16 acc = {};
#pragma unroll
      for (int f = 0; f < NMF; ++f) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o.A[t][f], BB[f], acc, 0, 0, 0);
      return acc;
    }, a1B, s2B, rlB);
    // lanes 0-31: both halves of group A's row; lanes 32-63: group B's
    int a1x, a1y, s2x, s2y, rlx, rly;
    swap_halves(a1A, a1B, a1x, a1y);
    swap_halves(s2A, s2B, s2x, s2y);
    swap_halves(rlA, rlB, rlx, rly);
    float f1, f2;
    const int code = merge_keys(a1x, a1y, s2x, s2y, rlx, rly, f1, f2);
    const float xnorm = sqrtf(rp.xn) * 1.0001f;
    const float beta = bd.e_cross * xnorm * o.cm + bd.e_norm * (o.cm * o.cm + rp.xn);
    const bool amb = not_separated(f1, f2, beta, bd.g_exact, rp.xn) || code >= ks;
    if (valid && codes) codes[row * m + sub] = (uint8_t)code;
    const bool push = valid && amb;
    const uint64_t mask = __ballot(push);
    if (mask) {
      int at = np;
      if (DYN) {   // the block's list
        int b = 0;
        if (lane == 0) b = atomicAdd(dyn + 1, __popcll(mask));
        at = __builtin_amdgcn_readfirstlane(b);
      }
      if (push) pend[at + lanes_below(mask)] = (uint16_t)(row - rb);
      np += __popcll(mask);
    }
    if (ACC && valid && !amb) {
      float v[DW];
#pragma unroll
      for (int e = 0; e < DW; e += 4) {
        const float4 q = acc.stash[(e >> 2) * 64 + lane];
        v[e] = q.x;
        v[e + 1] = q.y;
        v[e + 2] = q.z;
        v[e + 3] = q.w;
      }
      acc_row<DW>(acc, code, v, ds);
    }
    if (OUT && valid && !amb) {   // the chosen centroid's distance and squared error
      // the row again, from the stash (one 8-dimension block) or from cache:
      // keeping it live through the matrix-core phase would cost registers
      // and occupancy
      if (NB == 1) {
#pragma unroll
        for (int e = 0; e < DW; e += 4) {
          const float4 q = acc.stash[(e >> 2) * 64 + lane];
          xv[e] = q.x;
          xv[e + 1] = q.y;
          xv[e + 2] = q.z;
          xv[e + 3] = q.w;
        }
      } else {
        load_own_row<DW, FULL>(xv, x, r0, re, d, sub, ds, lane);
      }
      const float* c = cbsub + (int64_t)code * ds;
      float cv[DW];
      if (FULL) {
#pragma unroll
        for (int e = 0; e < DW; e += 4) {
          const float4 v = *reinterpret_cast<const float4*>(c + e);
          cv[e] = v.x;
          cv[e + 1] = v.y;
          cv[e + 2] = v.z;
          cv[e + 3] = v.w;
        }
      } else {
#pragma unroll
        for (int e = 0; e < DW; ++e) cv[e] = c[e < ds ? e : ds - 1];
      }
      float dist = 0.0f;
      double sq = 0.0;
#pragma unroll
      for (int t = 0; t < DW; ++t)
        if (t < ds) {
          const float df = xv[t] - cv[t];
          const float s2 = df * df;
          dist = dist + s2;
          const double dd = (double)xv[t] - (double)cv[t];
          sq = sq + dd * dd;
        }
      if (min_dist) min_dist[row * m + sub] = dist;
      *sse += sq;
    }
    r0 = rnext;
  }
  if (DYN) {   // the block's list once every wave is done, split evenly over the waves
    __syncthreads();
    const int nw = (int)(blockDim.x >> 6), w = (int)(threadIdx.x >> 6);
    const int total = dyn[1];
    const int s0 = (int)((int64_t)total * w / nw), s1 = (int)((int64_t)total * (w + 1) / nw);
    redecide<DW, REG, OUT, ACC>(pend + s0, rb, s1 - s0, x, d, m, ks, ds, sub, cbsub, codes, lane, min_dist, sse, acc);
    return total;
  }
  redecide<DW, REG, OUT, ACC>(pend, rb, np, x, d, m, ks, ds, sub, cbsub, codes, lane, min_dist, sse, acc);
  return np;
}

// One problem: block = (row block, group of 4 subspaces), one subspace per
// wave (assign_rows64 over the block's rows).  OUT: min_dist (optional) and
// per-wave squared-error partials sse_part[block * 4 + wave] (every wave
// writes its slot).
template <int NB, int NT, bool FULL, bool OUT>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(NB == 1 ? 3 : 1, 8))) void k_assign_bf16(
    const float* __restrict__ x, int64_t n, int d, int m, int ks, int ds,
    const bf16x8* __restrict__ aop, const float* __restrict__ cmax, const float* __restrict__ mu,
    const float* __restrict__ c32, uint8_t* __restrict__ codes,
    unsigned long long* __restrict__ rescored, int groups, int rpb, float e_cross, float e_norm,
    float g_exact, float* __restrict__ min_dist, double* __restrict__ sse_part) {
  const XcdMap bm = xcd_map(blockIdx.x, groups);
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int sub = bm.group * 4 + w;
  const int64_t rbeg = (int64_t)bm.rowblk * rpb;
  double sse = 0.0;
  // LDS: rpb list entries per wave, so the list cannot overflow; with OUT
  // and one 8-dimension block (STAGE) also the float32 centroids of the
  // block's four subspaces (the chosen centroid of every row is read from
  // there) and the waves' stashes of their rows' slices (kept until the
  // rows' codes are known)
  constexpr bool STAGE = OUT && NB == 1;
  extern __shared__ __align__(16) uint16_t pend16[];
  float* cb_lds = reinterpret_cast<float*>(pend16 + (kThreads / 64) * rpb);
  const int s0 = bm.group * 4;
  if (STAGE) {
    const int nsub = min(4, m - s0);
    const int cnt = nsub * ks * ds;
    const float* src = c32 + (int64_t)s0 * ks * ds;
    if ((cnt & 3) == 0 && (reinterpret_cast<uintptr_t>(src) & 15) == 0) {
      for (int i = threadIdx.x; i < cnt / 4; i += blockDim.x)
        reinterpret_cast<float4*>(cb_lds)[i] = reinterpret_cast<const float4*>(src)[i];
    } else {
      for (int i = threadIdx.x; i < cnt; i += blockDim.x) cb_lds[i] = src[i];
    }
    __syncthreads();
  }
  if (sub < m && rbeg < n) {
    const int64_t rend = min(n, rbeg + rpb);
    SubOps<NB, NT> o;
    load_sub_ops<NB, NT>(o, aop, cmax, mu, sub, lane);
    const Band bd{e_cross, e_norm, g_exact};
    AccLds st;
    if (STAGE) st.stash = reinterpret_cast<float4*>(cb_lds + 4 * ks * ds) + w * 2 * 64;
    const float* cbsub = STAGE ? cb_lds + w * ks * ds : c32 + (int64_t)sub * ks * ds;
    const int np = assign_rows64<NB, NT, FULL, OUT, true>(o, bd, x, d, ds, m, ks, sub, rbeg, rend, cbsub, codes,
                                                          pend16 + w * rpb, lane, min_dist, &sse, st);
    if (rescored && lane == 0 && np) atomicAdd(rescored, (unsigned long long)np);
  }
  if (OUT && sse_part) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) sse += __shfl_xor(sse, off, 64);
    if (lane == 0) sse_part[blockIdx.x * 4 + w] = sse;
  }
}

// One Lloyd round of one problem in one launch: the assignment of
// k_assign_bf16 and the float64 sums of the rows by code (the accumulation
// of paper Section 2.1's centroid update), which k_accumulate would otherwise
// take in a second pass over the rows.  Block = (row chunk c, subspace j),
// W = fit_waves(NB) waves: all the waves one CU holds at the kernel's
// register use, so one block per CU shares one set of sums and the chunks
// (hence the finalize's partials) are few.  xcd_map with one subspace per
// group puts the m blocks of a chunk on one XCD and its L2.  Wave w takes
// rows [(c W + w) rpw, + rpw) of subspace j (its pending list has room for
// all of them; a loop over pieces would keep the operands live across the
// re-decisions and spill).
// The block's sums and counts are formed in
// LDS (lane atomics, as k_accumulate) and stored as chunk c's partials in
// k_accumulate's layout, for the finalize.  Block 0 also zeroes cmax_zero,
// the per-subspace norm bound that the finalize raises for the next round
// (a buffer other than the cmax this launch reads).
template <int NB, int NT, bool FULL>
__global__ __launch_bounds__(fit_waves(NB) * 64) __attribute__((amdgpu_waves_per_eu(NB == 1 ? 3 : 1, 8))) void
k_fit_round_bf16(const float* __restrict__ x, int64_t n, int d, int m, int ks, int ds, const bf16x8* __restrict__ aop,
                 const float* __restrict__ cmax, const float* __restrict__ mu, const float* __restrict__ c32,
                 uint8_t* __restrict__ codes, unsigned long long* __restrict__ rescored, int nch, int rpw,
                 float e_cross, float e_norm, float g_exact, double* __restrict__ part_s,
                 uint32_t* __restrict__ part_cnt, float* __restrict__ cmax_zero) {
  constexpr int DW = NB * 8;
  constexpr int W = fit_waves(NB);
  extern __shared__ __align__(16) unsigned char fit_lds[];
  if (cmax_zero && blockIdx.x == 0)
    for (int j = threadIdx.x; j < m; j += blockDim.x) cmax_zero[j] = 0.0f;
  const XcdMap bm = xcd_map(blockIdx.x, m);
  const int chunk = bm.rowblk, sub = bm.group;
  if (chunk >= nch) return;   // grid padding (block-uniform)
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // LDS: sums, counts, the waves' stashes and pending lists
  const int stride = ds + 1;
  AccLds acc;
  acc.S = reinterpret_cast<double*>(fit_lds);
  acc.cnt = reinterpret_cast<uint32_t*>(acc.S + (size_t)ks * stride);
  float4* stash0 = reinterpret_cast<float4*>(fit_lds + fit_lds_stash_offset(ks, ds));
  acc.stash = stash0 + w * (DW / 4) * 64;
  uint16_t* pend = reinterpret_cast<uint16_t*>(stash0 + W * (DW / 4) * 64);   // W rpw entries
  int* dyn = reinterpret_cast<int*>(pend + W * rpw + (W * rpw & 1));
  for (int i = threadIdx.x; i < ks * stride; i += blockDim.x) acc.S[i] = 0.0;
  for (int i = threadIdx.x; i < ks; i += blockDim.x) acc.cnt[i] = 0u;
  if (threadIdx.x < 2) dyn[threadIdx.x] = 0;
  __syncthreads();
  // the block's rows, claimed 64 at a time by its waves
  const int64_t rb = (int64_t)chunk * W * rpw;
  const int64_t re = min(n, rb + (int64_t)W * rpw);
  const float* cbsub = c32 + (int64_t)sub * ks * ds;
  if (rb < re) {   // block-uniform
    SubOps<NB, NT> o;
    load_sub_ops<NB, NT>(o, aop, cmax, mu, sub, lane);
    const Band bd{e_cross, e_norm, g_exact};
    const int total = assign_rows64<NB, NT, FULL, false, true, true, true>(o, bd, x, d, ds, m, ks, sub, rb, re, cbsub,
                                                                           codes, pend, lane, nullptr, nullptr, acc,
                                                                           dyn);
    if (rescored && threadIdx.x == 0 && total) atomicAdd(rescored, (unsigned long long)total);
  }
  __syncthreads();
  const int per = ks * ds;
  const size_t base = (size_t)chunk * m + sub;
  for (int i = threadIdx.x; i < per; i += blockDim.x) {
    const int k = i / ds;
    part_s[base * per + i] = acc.S[k * stride + (i - k * ds)];
  }
  for (int i = threadIdx.x; i < ks; i += blockDim.x) part_cnt[base * ks + i] = acc.cnt[i];
}

// Many problems, one Lloyd round in one launch: k_fit_round_bf16 on the
// accumulation items (problem p, chunk c, subspace j) of the batched update
// (chunks of all problems in order, then subspace; problem p's chunk c is
// rows [c rpc, (c + 1) rpc) of its own), so the partials keep that layout
// and the batched finalize reads them unchanged.  The block's W waves claim
// the chunk's 64-row steps; its pending list has room for W rpw >= rpc rows.
// No objective terms are formed (part_j gets zeros) and no codes are stored
// (codes NULL to assign_rows64): the final encode writes every code, and a
// byte column per block would make each code line travel to HBM many times.
// cmax is only read: the finalize writes per-tile maxima and the round's last
// kernel reduces them.
template <int NB, int NT, bool FULL>
__global__ __launch_bounds__(fit_waves(NB) * 64) __attribute__((amdgpu_waves_per_eu(NB == 1 ? 3 : 1, 8))) void
k_fit_round_bf16_batched(const BatchProb* __restrict__ probs, int nprob, int64_t items, int d, int m, int ks,
                         int ds, const bf16x8* __restrict__ aop, size_t aop_stride, const float* __restrict__ cmax,
                         const float* __restrict__ mu, int rpw, float e_cross, float e_norm, float g_exact,
                         double* __restrict__ part_s, uint32_t* __restrict__ part_cnt,
                         double* __restrict__ part_j) {
  constexpr int DW = NB * 8;
  constexpr int W = fit_waves(NB);
  extern __shared__ __align__(16) unsigned char fit_lds[];
  const XcdMap bm = xcd_map(blockIdx.x, m);
  const int64_t item = (int64_t)bm.rowblk * m + bm.group;
  if (item >= items) return;   // grid padding (block-uniform)
  // the problem holding the item: the last p with item0 <= item
  int lo = 0, hi = nprob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (probs[mid].item0 <= item) lo = mid;
    else hi = mid - 1;
  }
  const int p = lo;
  const int local = (int)(item - probs[p].item0);
  const int chunk = local / m, sub = local - chunk * m;
  const float* px = probs[p].x;
  const int64_t n = probs[p].n, rpc = probs[p].rpc;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int stride = ds + 1;
  AccLds acc;
  acc.S = reinterpret_cast<double*>(fit_lds);
  acc.cnt = reinterpret_cast<uint32_t*>(acc.S + (size_t)ks * stride);
  float4* stash0 = reinterpret_cast<float4*>(fit_lds + fit_lds_stash_offset(ks, ds));
  acc.stash = stash0 + w * (DW / 4) * 64;
  uint16_t* pend = reinterpret_cast<uint16_t*>(stash0 + W * (DW / 4) * 64);   // W rpw entries
  int* dyn = reinterpret_cast<int*>(pend + W * rpw + (W * rpw & 1));
  for (int i = threadIdx.x; i < ks * stride; i += blockDim.x) acc.S[i] = 0.0;
  for (int i = threadIdx.x; i < ks; i += blockDim.x) acc.cnt[i] = 0u;
  if (threadIdx.x < 2) dyn[threadIdx.x] = 0;
  __syncthreads();
  const int64_t rb = (int64_t)chunk * rpc;
  const int64_t re = min(n, rb + rpc);
  const float* cbsub = probs[p].c32 + (int64_t)sub * ks * ds;
  if (rb < re) {   // block-uniform
    SubOps<NB, NT> o;
    load_sub_ops<NB, NT>(o, aop + (size_t)p * aop_stride, cmax + (size_t)p * m, mu + (size_t)p * m * kMaxDsBf16,
                         sub, lane);
    const Band bd{e_cross, e_norm, g_exact};
    (void)assign_rows64<NB, NT, FULL, false, true, true, true>(o, bd, px, d, ds, m, ks, sub, rb, re, cbsub,
                                                               nullptr, pend, lane, nullptr, nullptr, acc, dyn);
  }
  __syncthreads();
  const int per = ks * ds;
  for (int i = threadIdx.x; i < per; i += blockDim.x) {
    const int k = i / ds;
    part_s[(size_t)item * per + i] = acc.S[k * stride + (i - k * ds)];
  }
  for (int i = threadIdx.x; i < ks; i += blockDim.x) part_cnt[(size_t)item * ks + i] = acc.cnt[i];
  if (threadIdx.x == 0) part_j[item] = 0.0;
}

// Many problems in one persistent launch.  The work is the list of units
// (problem, group of 4 subspaces, 32-row tile): problem-major, then group,
// then tile.  Logical block b takes the contiguous range [U b / G, U (b+1) / G)
// of the U units, so it crosses few (problem, group) segments and keeps one
// segment's operands in registers while it lasts.  Logical blocks are
// numbered so that each XCD (hardware block id mod 8) holds a contiguous
// eighth of the list: neighbouring segments share that XCD's L2.
// REG: how a piece's pending rows are re-decided (the register form, with the
// subspace's centroids held in registers across the piece's rows, or one row
// at a time with the centroids re-read); the register form is faster per row
// but raises the kernel's register count, so the plan chooses between them.
template <int NB, int NT, bool FULL, bool REG>
__global__ __launch_bounds__(kThreads) void k_assign_bf16_batched(
    const BatchProb* __restrict__ probs, int nprob, int64_t units, int d, int m, int ks, int ds,
    const bf16x8* __restrict__ aop, size_t aop_stride, const float* __restrict__ cmax,
    const float* __restrict__ mu, unsigned long long* __restrict__ rescored, float e_cross, float e_norm,
    float g_exact) {
  constexpr int PC = kBatchPend;
  __shared__ uint16_t pend_all[(kThreads / 64) * PC];
  const int G = gridDim.x;   // a multiple of 8
  const int lb = (int)(blockIdx.x & 7) * (G >> 3) + (int)(blockIdx.x >> 3);
  // block-uniform work indices, kept in scalar registers (the divisions
  // themselves run on the vector unit)
  int64_t u = uniform64(units * lb / G);
  const int64_t uend = uniform64(units * (lb + 1) / G);
  if (u >= uend) return;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int groups = (m + 3) >> 2;
  const Band bd{e_cross, e_norm, g_exact};
  // the problem holding unit u: the last p with unit0 <= u
  int lo = 0, hi = nprob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (probs[mid].unit0 <= u) lo = mid;
    else hi = mid - 1;
  }
  int p = lo;
  uint32_t nres = 0;
  while (u < uend) {
    while (p + 1 < nprob && probs[p + 1].unit0 <= u) ++p;
    const float* px = probs[p].x;
    const int64_t n = probs[p].n;
    const int64_t tiles = (n + 31) >> 5;
    const int64_t local = u - probs[p].unit0;   // < groups * tiles < 2^32
    const int group = __builtin_amdgcn_readfirstlane((int)((uint32_t)local / (uint32_t)tiles));
    const int64_t t0 = local - (int64_t)group * tiles;
    const int64_t t1 = min(tiles, t0 + (uend - u));
    u += t1 - t0;
    const int sub = group * 4 + w;
    if (group >= groups || sub >= m) continue;
    SubOps<NB, NT> o;
    load_sub_ops<NB, NT>(o, aop + (size_t)p * aop_stride, cmax + (size_t)p * m, mu + (size_t)p * m * kMaxDsBf16,
                         sub, lane);
    // rows in pieces of PC, so that a piece's pending list fits the wave's LDS
    const int64_t rb = t0 * 32, re = min(n, t1 * 32);
    for (int64_t pb = rb; pb < re; pb += PC)
      nres += (uint32_t)assign_rows64<NB, NT, FULL, false, REG>(o, bd, px, d, ds, m, ks, sub, pb,
                                                                  min(re, pb + PC),
                                                                  probs[p].c32 + (int64_t)sub * ks * ds,
                                                                  probs[p].codes, pend_all + w * PC, lane,
                                                                  nullptr, nullptr);
  }
  if (rescored && lane == 0 && nres) atomicAdd(rescored, (unsigned long long)nres);
}

// ---- FP8 (OCP E4M3) matrix-core path ----------------------------------------
// One v_mfma_f32_32x32x64_f8f6f4 per 32-centroid tile.  Per subspace a power of
// two sigma maps the centred centroids into [-16, 16] (x~ = (x - mu)/sigma,
// c^ = -2 (c - mu)/sigma); each value v is split into fp8 parts vh = fp8(v),
// vl = fp8(v - vh), with residual ev = v - vh - vl.  K slots (same for A, B):
//   hh: ch.xh   lh: cl.xh   hl: ch.xl   (DW slots each)
//   4 slots: pieces of ||c~||^2 times 16, 1, 1/16, 1/256 (row side holds the
//   multipliers), 4 slots: 256, 16, 1, 1/16 times pieces of ||x~||^2.
// DW = 8: all 32 slots in lane half 0 (half 1 zero); DW = 16: hh, lh in half
// 0, hl and the norm slots in half 1.  The estimate is ||x~ - c~||^2 up to the
// dropped terms xl.cl + (xh + xl).ec + ex.c^, the norm residuals and the
// float32 accumulation; the bound uses the measured norms of the parts, so it
// holds for any rounding of the conversions.  Values are clamped to the fp8
// range first; a clamped row gets a large residual and goes to the exact rule.
typedef int i32x8 __attribute__((ext_vector_type(8)));
constexpr int kFp8Stats = 24;   // per subspace: mu[16], 1/sigma, sigma^2, Lc, Ec, Cc, Rc, ncmax, pad
constexpr float kFp8Max = 448.0f;

__device__ __forceinline__ float clamp8(float v) { return fminf(fmaxf(v, -kFp8Max), kFp8Max); }
// two floats to two fp8 bytes (low 16 bits), then back to float
__device__ __forceinline__ uint32_t pk8(float a, float b) {
  return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(clamp8(a), clamp8(b), 0, false) & 0xFFFFu;
}
__device__ __forceinline__ f32x2 unpk8(uint32_t w) { return __builtin_amdgcn_cvt_pk_f32_fp8((int)w, false); }

struct Split8 {   // fp8 high/low parts of a DW-vector, packed 4 per dword
  uint32_t h[4], l[4];   // DW <= 16
  float nl, ne;          // ||vl||, ||v - vh - vl||
};
template <int DW>
__device__ __forceinline__ Split8 split8(const float (&v)[DW]) {
  Split8 s;
  float sl = 0.0f, se = 0.0f;
#pragma unroll
  for (int i = 0; i < DW; i += 4) {
    const uint32_t h01 = pk8(v[i], v[i + 1]), h23 = pk8(v[i + 2], v[i + 3]);
    const f32x2 fh01 = unpk8(h01), fh23 = unpk8(h23);
    const float r0 = v[i] - fh01[0], r1 = v[i + 1] - fh01[1], r2 = v[i + 2] - fh23[0], r3 = v[i + 3] - fh23[1];
    const uint32_t l01 = pk8(r0, r1), l23 = pk8(r2, r3);
    const f32x2 fl01 = unpk8(l01), fl23 = unpk8(l23);
    const float e0 = r0 - fl01[0], e1 = r1 - fl01[1], e2 = r2 - fl23[0], e3 = r3 - fl23[1];
    s.h[i >> 2] = h01 | (h23 << 16);
    s.l[i >> 2] = l01 | (l23 << 16);
    sl = __builtin_fmaf(fl01[0], fl01[0], sl);
    sl = __builtin_fmaf(fl01[1], fl01[1], sl);
    sl = __builtin_fmaf(fl23[0], fl23[0], sl);
    sl = __builtin_fmaf(fl23[1], fl23[1], sl);
    se = __builtin_fmaf(e0, e0, se);
    se = __builtin_fmaf(e1, e1, se);
    se = __builtin_fmaf(e2, e2, se);
    se = __builtin_fmaf(e3, e3, se);
  }
  s.nl = sqrtf(sl) * 1.0001f;
  s.ne = sqrtf(se) * 1.0001f;
  return s;
}

// four fp8 pieces of v against the multipliers 2^k0, 2^(k0-4), 2^(k0-8),
// 2^(k0-12): packed bytes and the remaining residual |v - sum|
__device__ __forceinline__ uint32_t pieces8(float v, float inv0, float& resid) {
  float r = v, m = inv0, mul = 1.0f / inv0;
  uint32_t out = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t b = pk8(r * m, 0.0f) & 0xFFu;
    const float pf = unpk8(b)[0];
    r = r - pf * mul;   // exact while the pieces track the residual
    out |= b << (8 * i);
    m *= 16.0f;
    mul *= 0.0625f;
  }
  resid = fabsf(r);
  return out;
}

template <int NT>
struct SubOps8 {
  i32x8 A[NT];
  float muv[16];
  float inv_sigma, sigma2, Lc, Ec, Cc, Rc, ncmax;
  uint32_t mult_c;   // fp8 16, 1, 1/16, 1/256: row-side multipliers of the centroid norm pieces
};

template <int NB, int NT>
__device__ __forceinline__ void load_sub_ops8(SubOps8<NT>& o, const i32x8* __restrict__ aop,
                                              const float* __restrict__ stats, int sub, int lane) {
#pragma unroll
  for (int t = 0; t < NT; ++t) o.A[t] = aop[(size_t)(sub * NT + t) * 64 + lane];
  const float* st = stats + (size_t)sub * kFp8Stats;
  auto uni = [](float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); };
#pragma unroll
  for (int e = 0; e < NB * 8; ++e) o.muv[e] = uni(st[e]);
  o.inv_sigma = uni(st[16]);
  o.sigma2 = uni(st[17]);
  o.Lc = uni(st[18]);
  o.Ec = uni(st[19]);
  o.Cc = uni(st[20]);
  o.Rc = uni(st[21]);
  o.ncmax = uni(st[22]);
  o.mult_c = (uint32_t)__builtin_amdgcn_readfirstlane((int)(pk8(16.0f, 1.0f) | (pk8(0.0625f, 0.00390625f) << 16)));
}

// FP8 decision for the row held by lanes l and l^32; estimates and the bound
// are in units of sigma^2.
template <int NB, int NT>
__device__ __forceinline__ int decide_tile_fp8(const float (&xraw)[NB * 8], const SubOps8<NT>& o, int half, int ks,
                                               float g_exact, bool& amb) {
  constexpr int DW = NB * 8;
  float xv[DW];   // x~ = (x - mu) / sigma, clamped to the fp8 range
  float nx = 0.0f;
#pragma unroll
  for (int e = 0; e < DW; ++e) {
    const float v = (xraw[e] - o.muv[e]) * o.inv_sigma;
    nx = __builtin_fmaf(v, v, nx);
    xv[e] = v;
  }
  const Split8 sx = split8<DW>(xv);
  float rx;
  const uint32_t q = pieces8(nx, 1.0f / 256.0f, rx);
  const uint32_t mult_c = o.mult_c;
  i32x8 B;
  if (DW == 8) {
    if (half == 0) {
      B = i32x8{(int)sx.h[0], (int)sx.h[1], (int)sx.h[0], (int)sx.h[1], (int)sx.l[0], (int)sx.l[1], (int)mult_c,
                (int)q};
    } else {
      B = i32x8{0, 0, 0, 0, 0, 0, 0, 0};
    }
  } else {
    if (half == 0) {
      B = i32x8{(int)sx.h[0], (int)sx.h[1], (int)sx.h[2], (int)sx.h[3],
                (int)sx.h[0], (int)sx.h[1], (int)sx.h[2], (int)sx.h[3]};
    } else {
      B = i32x8{(int)sx.l[0], (int)sx.l[1], (int)sx.l[2], (int)sx.l[3], (int)mult_c, (int)q, 0, 0};
    }
  }
  auto tile = [&](int t) {
    f32x16 acc = {};
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(o.A[t], B, acc, 0, 0, 0, 0, 0, 0);
  };
  float f1, f2;
  const int code = reduce_scores<NT>(tile, f1, f2);
  // bound on |estimate - ||x~ - c~||^2| (see the section comment)
  const float xnorm = sqrtf(nx) * 1.0001f;
  const float xh_norm = xnorm + sx.ne;
  const float beta = (sx.nl * o.Lc + xh_norm * o.Ec + sx.ne * o.Cc + o.Rc + rx +
                      7.7e-6f * (nx + o.ncmax + 3.0f * xh_norm * o.Cc) + 1.9e-6f * (nx + o.ncmax)) * 1.001f;
  amb = not_separated(f1, f2, beta, g_exact, nx) || code >= ks;
  return code;
}

// FP8 operands of one subspace (block = subspace, thread = centroid; ks <= 256).
template <int NB>
__global__ __launch_bounds__(256) void k_pack_fp8(const float* __restrict__ c32, int ks, int ds, int nt,
                                                  i32x8* __restrict__ aop, float* __restrict__ stats) {
  constexpr int DW = NB * 8;
  __shared__ float red[4][2 * DW];
  __shared__ float mu_s[DW];
  __shared__ float mx[4][6];
  __shared__ float sig_s;
  const int sub = blockIdx.x;
  const int k = threadIdx.x;
  const int lane = k & 63, w = k >> 6;
  const bool real = k < ks;
  const float* c = c32 + ((size_t)sub * ks + (real ? k : 0)) * ds;
  float cv[DW];
#pragma unroll
  for (int e = 0; e < DW; ++e) cv[e] = e < ds ? c[e < ds ? e : 0] : 0.0f;
  // centre: midpoint of the coordinate range of the centroids
#pragma unroll
  for (int e = 0; e < DW; ++e) {
    float lo = real ? cv[e] : INFINITY, hi = real ? cv[e] : -INFINITY;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      lo = fminf(lo, __shfl_xor(lo, off, 64));
      hi = fmaxf(hi, __shfl_xor(hi, off, 64));
    }
    if (lane == 0) {
      red[w][e] = lo;
      red[w][DW + e] = hi;
    }
  }
  __syncthreads();
  if (k < DW) {
    float lo = red[0][k], hi = red[0][DW + k];
    for (int i = 1; i < 4; ++i) {
      lo = fminf(lo, red[i][k]);
      hi = fmaxf(hi, red[i][DW + k]);
    }
    mu_s[k] = (k < ds && lo <= hi) ? 0.5f * lo + 0.5f * hi : 0.0f;
  }
  __syncthreads();
  // sigma: power of two with max |c - mu| / sigma <= 16
  float a = 0.0f;
#pragma unroll
  for (int e = 0; e < DW; ++e) a = fmaxf(a, real ? fabsf(cv[e] - mu_s[e]) : 0.0f);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) a = fmaxf(a, __shfl_xor(a, off, 64));
  if (lane == 0) mx[w][0] = a;
  __syncthreads();
  if (k == 0) {
    const float am = fmaxf(fmaxf(mx[0][0], mx[1][0]), fmaxf(mx[2][0], mx[3][0]));
    int ex = 0;
    (void)frexpf(am * 0.0625f, &ex);
    sig_s = am > 0.0f && am < INFINITY ? ldexpf(1.0f, ex) : 1.0f;
  }
  __syncthreads();
  const float sigma = sig_s;
  const float inv = 1.0f / sigma;   // exact: a power of two
  float ch[DW];
  float nc = 0.0f, cn2 = 0.0f;
#pragma unroll
  for (int e = 0; e < DW; ++e) {
    const float ct = (cv[e] - mu_s[e]) * inv;
    nc = __builtin_fmaf(ct, ct, nc);
    ch[e] = -2.0f * ct;
    cn2 = __builtin_fmaf(ch[e], ch[e], cn2);
  }
  Split8 sc = split8<DW>(ch);
  float rc;
  uint32_t pc = pieces8(nc, 0.0625f, rc);
  // bounds over the real centroids
  float v[5] = {real ? sc.nl : 0.0f, real ? sc.ne : 0.0f, real ? sqrtf(cn2) * 1.0001f : 0.0f, real ? rc : 0.0f,
                real ? nc : 0.0f};
#pragma unroll
  for (int i = 0; i < 5; ++i) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[i] = fmaxf(v[i], __shfl_xor(v[i], off, 64));
    if (lane == 0) mx[w][i] = v[i];
  }
  __syncthreads();
  float* st = stats + (size_t)sub * kFp8Stats;
  if (k < 5) {
    const float r = fmaxf(fmaxf(mx[0][k], mx[1][k]), fmaxf(mx[2][k], mx[3][k]));
    st[18 + k] = r;
  }
  if (k < 16) st[k] = k < DW ? mu_s[k] : 0.0f;
  if (k == 0) {
    st[16] = inv;
    st[17] = sigma * sigma;
    st[23] = 0.0f;
  }
  if (k < nt * 32) {
    if (!real) {   // padded candidate: zero parts, large norm
      for (int i = 0; i < 4; ++i) sc.h[i] = sc.l[i] = 0u;
      pc = pk8(kFp8Max, kFp8Max) | (pk8(kFp8Max, kFp8Max) << 16);
    }
    const uint32_t mult_x = pk8(256.0f, 16.0f) | (pk8(1.0f, 0.0625f) << 16);
    i32x8 a0, a1;
    if (DW == 8) {
      a0 = i32x8{(int)sc.h[0], (int)sc.h[1], (int)sc.l[0], (int)sc.l[1], (int)sc.h[0], (int)sc.h[1], (int)pc,
                 (int)mult_x};
      a1 = i32x8{0, 0, 0, 0, 0, 0, 0, 0};
    } else {
      a0 = i32x8{(int)sc.h[0], (int)sc.h[1], (int)sc.h[2], (int)sc.h[3],
                 (int)sc.l[0], (int)sc.l[1], (int)sc.l[2], (int)sc.l[3]};
      a1 = i32x8{(int)sc.h[0], (int)sc.h[1], (int)sc.h[2], (int)sc.h[3], (int)pc, (int)mult_x, 0, 0};
    }
    const int t = k >> 5, i = k & 31;
    aop[((size_t)sub * nt + t) * 64 + i] = a0;
    aop[((size_t)sub * nt + t) * 64 + 32 + i] = a1;
  }
}

// One problem, FP8 operands; same geometry and exact re-decision as the BF16 kernel.
template <int NB, int NT, bool FULL>
__global__ __launch_bounds__(kThreads) void k_assign_fp8(
    const float* __restrict__ x, int64_t n, int d, int m, int ks, int ds, const i32x8* __restrict__ aop,
    const float* __restrict__ stats, const float* __restrict__ c32, uint8_t* __restrict__ codes,
    unsigned long long* __restrict__ rescored, int groups, int rpb, float g_exact) {
  const XcdMap bm = xcd_map(blockIdx.x, groups);
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int sub = bm.group * 4 + w;
  const int64_t rbeg = (int64_t)bm.rowblk * rpb;
  if (sub >= m || rbeg >= n) return;
  const int64_t rend = min(n, rbeg + rpb);
  SubOps8<NT> o;
  load_sub_ops8<NB, NT>(o, aop, stats, sub, lane);
  extern __shared__ uint32_t pend_all[];
  auto decide = [&](const float (&xv)[NB * 8], int half, bool& amb) {
    return decide_tile_fp8<NB, NT>(xv, o, half, ks, g_exact, amb);
  };
  const uint32_t nres = assign_rows<NB * 8, FULL, false, true>(x, d, ds, m, ks, sub, rbeg, rend, decide,
                                                         c32 + (int64_t)sub * ks * ds, codes, pend_all + w * rpb,
                                                         0, lane);
  if (rescored && lane == 0 && nres) atomicAdd(rescored, (unsigned long long)nres);
}

}  // namespace

size_t bf16_operand_count(int m, int ks, int ds) {
  const int nb = (ds + 7) / 8;
  return (size_t)m * tiles_for(ks) * bf16_nmfma(nb) * 64;
}

Bf16Geom bf16_geometry(int64_t n, int m, int max_tiles) {
  Bf16Geom g;
  g.groups = ceil_div(m, 4);
  // one round of resident blocks (three per CU: the assignment kernels' register
  // use allows three waves per SIMD), so no partly filled last round; at most
  // 64 row tiles per block, an even number (the single-problem kernel steps
  // 64 rows at a time).  (On 100k-row fit launches: 61 us against 65 us
  // with ~8 blocks per CU.)
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                              hipSuccess || cus < 1)
    cus = 256;
  const int64_t resident = 3 * (int64_t)cus;
  const int64_t row_tiles = (n + 31) / 32;
  // beyond max_tiles per block: as many rounds as needed, the tiles spread
  // evenly over them (a last round nearly as full as the others, rather than
  // a few max_tiles blocks running alone at the end)
  const int64_t work = row_tiles * g.groups;
  int64_t rounds = (work + resident * max_tiles - 1) / (resident * max_tiles);
  if (rounds < 1) rounds = 1;
  int64_t tpb = (work + resident * rounds - 1) / (resident * rounds);
  if (tpb < 1) tpb = 1;
  if (tpb > max_tiles) tpb = max_tiles;
  tpb = (tpb + 1) & ~int64_t(1);   // whole 64-row steps
  g.rpb = int(tpb * 32);
  g.rowblks = n > 0 ? ceil_div(n, g.rpb) : 0;
  g.blocks = ceil_div(g.rowblks, 8) * 8 * g.groups;
  return g;
}

namespace {
// error-bound constants: split products 3.1 u^2 per term (u = 2^-8), twice
// for the -2 factor, plus float32 accumulation over K = 16*NMF terms at
// 2^-23 each, plus the rounding of the centring (2^-22 of the squared
// norms); g_exact bounds the relative error of the exact float32 rule
Band band_for(int ds) {
  const int nb = (ds + 7) / 8;
  const int nmf = bf16_nmfma(nb);
  Band b;
  b.e_cross = 1.25e-4f * (nb == 1 ? 1.0f : 1.05f);
  b.e_norm = 2.4e-6f * nmf + 2.4e-7f;
  b.g_exact = (float)((ds + 2) * 1.01 / 16777216.0);
  return b;
}
}  // namespace

int launch_assign_bf16(const float* x, int64_t n, int d, int m, int ks, const void* aop,
                       const float* cmax, const float* mu, const float* c32, uint8_t* codes,
                       int64_t* rescored, float* min_dist, double* sse_part, hipStream_t s) {
  const int ds = d / m;
  const int nb = (ds + 7) / 8;
  const int nt = tiles_for(ks);
  const bool out = min_dist || sse_part;
  const Bf16Geom g = bf16_geometry(n, m, out ? kOutTiles : 64);
  if (g.blocks == 0) return MIPQ_OK;
  const Band bd = band_for(ds);
  ProfScope ps(MIPQ_K_ASSIGN_BF16, s);
  const bool full = (ds == nb * 8) && (d % 4 == 0) &&
                    (((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(c32)) & 15) == 0);
  unsigned long long* resc = reinterpret_cast<unsigned long long*>(rescored);
  const size_t pend_bytes = (size_t)(kThreads / 64) * g.rpb * sizeof(uint16_t) +
                            (out && nb == 1 ? (size_t)4 * ks * ds * sizeof(float) + (size_t)(kThreads / 64) * 64 * 8 * sizeof(float)
                                            : 0);
#define LAUNCH1(NB, NT, FULL, OUT)                                                                  \
  k_assign_bf16<NB, NT, FULL, OUT><<<g.blocks, kThreads, pend_bytes, s>>>(                          \
      x, n, d, m, ks, ds, (const bf16x8*)aop, cmax, mu, c32, codes, resc, g.groups, g.rpb, bd.e_cross, \
      bd.e_norm, bd.g_exact, min_dist, sse_part)
#define LAUNCH(NB, NT)                                 \
  do {                                                 \
    if (full) {                                        \
      if (out) LAUNCH1(NB, NT, true, true);            \
      else LAUNCH1(NB, NT, true, false);               \
    } else {                                           \
      if (out) LAUNCH1(NB, NT, false, true);           \
      else LAUNCH1(NB, NT, false, false);              \
    }                                                  \
  } while (0)
  if (nb == 1) {
    switch (nt) {
      case 1: LAUNCH(1, 1); break;
      case 2: LAUNCH(1, 2); break;
      case 4: LAUNCH(1, 4); break;
      default: LAUNCH(1, 8); break;
    }
  } else {
    switch (nt) {
      case 1: LAUNCH(2, 1); break;
      case 2: LAUNCH(2, 2); break;
      case 4: LAUNCH(2, 4); break;
      default: LAUNCH(2, 8); break;
    }
  }
#undef LAUNCH
#undef LAUNCH1
  MIPQ_LAUNCHED("k_assign_bf16");
  return MIPQ_OK;
}

int assign_bf16_sse_parts(int64_t n, int m) { return 4 * bf16_geometry(n, m, kOutTiles).blocks; }

namespace {
constexpr int kFitBlocks = 256;     // one block per CU on 256 CUs
constexpr int kFitRowsMax = 2048;   // rows per wave at most (as k_assign_bf16's blocks)
constexpr size_t kFitLdsMax = 65536;

size_t fit_lds_bytes(int ks, int ds, int rpw) {
  const int nb = ds <= 8 ? 1 : 2;
  const int w = fit_waves(nb);
  return fit_lds_stash_offset(ks, ds) + (size_t)w * 64 * nb * 8 * sizeof(float) +
         (((size_t)w * rpw * sizeof(uint16_t) + 3) & ~size_t(3)) + 2 * sizeof(int);
}
}  // namespace

// Chunks of the fused round: kFitBlocks / m of them (one round of blocks), or
// a whole number of such rounds when the rows per wave would pass
// kFitRowsMax or the pending lists' LDS.  rpw = 0: the sums and stashes leave
// no LDS for a list.  Depends on the shape only, so that workspace sizes need
// no device.
FitGeom fit_round_geometry(int64_t n, int m, int ks, int ds) {
  FitGeom g;
  if (n < 1 || m < 1) return g;
  const int w = fit_waves(ds <= 8 ? 1 : 2);
  int cap = kFitBlocks / m;
  if (cap < 1) cap = 1;
  int64_t rpw = ceil_div(n, (int64_t)w * cap);
  const size_t fixed = fit_lds_bytes(ks, ds, 0);
  int64_t room = fixed < kFitLdsMax ? (int64_t)((kFitLdsMax - fixed) / (w * sizeof(uint16_t))) : 0;
  if (room > kFitRowsMax) room = kFitRowsMax;
  if (room < 64) return g;
  if (rpw > room) {   // several rounds of blocks: as many equal full rounds as needed
    const int64_t rounds = ceil_div(ceil_div(n, (int64_t)w * room), cap);
    rpw = ceil_div(n, (int64_t)w * cap * rounds);
  }
  g.rpw = (int)rpw;
  g.nch = (int)ceil_div(n, (int64_t)w * rpw);
  return g;
}

int fit_round_batched_rpw(int ks, int ds, int64_t max_rpc) {
  if (max_rpc < 1 || max_rpc > 65536 || ds > kMaxDsBf16) return 0;   // pending offsets are 16-bit
  const int w = fit_waves(ds <= 8 ? 1 : 2);
  const int rpw = (int)ceil_div(max_rpc, w);
  int dev = 0, lds_max = 65536;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    lds_max = 65536;
  return fit_lds_bytes(ks, ds, rpw) <= (size_t)lds_max ? rpw : 0;
}

int launch_fit_round_bf16_batched(const BatchProb* probs, int nprob, int64_t items, int d, int m, int ks,
                                  const void* aop, size_t aop_stride, const float* cmax, const float* mu, bool full,
                                  int rpw, double* part_s, uint32_t* part_cnt, double* part_j, hipStream_t s) {
  const int ds = d / m;
  const int nb = (ds + 7) / 8;
  const int nt = tiles_for(ks);
  if (rpw < 1) return fail(MIPQ_EINVAL, "fused batched round: no pending-list room");
  const Band bd = band_for(ds);
  const size_t lds = fit_lds_bytes(ks, ds, rpw);
  const int64_t chunks = items / m;
  const unsigned grid = (unsigned)(((chunks + 7) / 8) * 8 * m);
  ProfScope ps(MIPQ_K_FIT_ROUND_BF16, s);
#define LAUNCH1(NB, NT, FULL)                                                                                  \
  k_fit_round_bf16_batched<NB, NT, FULL><<<grid, fit_waves(NB) * 64, lds, s>>>(                                \
      probs, nprob, items, d, m, ks, ds, (const bf16x8*)aop, aop_stride, cmax, mu, rpw, bd.e_cross, bd.e_norm,   \
      bd.g_exact, part_s, part_cnt, part_j)
#define LAUNCH(NB, NT)                 \
  do {                                 \
    if (full) LAUNCH1(NB, NT, true);   \
    else LAUNCH1(NB, NT, false);       \
  } while (0)
  if (nb == 1) {
    switch (nt) {
      case 1: LAUNCH(1, 1); break;
      case 2: LAUNCH(1, 2); break;
      case 4: LAUNCH(1, 4); break;
      default: LAUNCH(1, 8); break;
    }
  } else {
    switch (nt) {
      case 1: LAUNCH(2, 1); break;
      case 2: LAUNCH(2, 2); break;
      case 4: LAUNCH(2, 4); break;
      default: LAUNCH(2, 8); break;
    }
  }
#undef LAUNCH
#undef LAUNCH1
  MIPQ_LAUNCHED("k_fit_round_bf16_batched");
  return MIPQ_OK;
}

int launch_fit_round_bf16(const float* x, int64_t n, int d, int m, int ks, const void* aop, const float* cmax,
                          const float* mu, const float* c32, uint8_t* codes, int64_t* rescored, double* part_s,
                          uint32_t* part_cnt, float* cmax_zero, hipStream_t s) {
  const int ds = d / m;
  const int nb = (ds + 7) / 8;
  const int nt = tiles_for(ks);
  const FitGeom g = fit_round_geometry(n, m, ks, ds);
  if (g.rpw == 0) return fail(MIPQ_EUNSUPPORTED, "fused round: sums of ks=%d, ds=%d leave no LDS", ks, ds);
  const Band bd = band_for(ds);
  const bool full = (ds == nb * 8) && (d % 4 == 0) &&
                    (((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(c32)) & 15) == 0);
  unsigned long long* resc = reinterpret_cast<unsigned long long*>(rescored);
  const size_t lds = fit_lds_bytes(ks, ds, g.rpw);
  const unsigned grid = (unsigned)(ceil_div(g.nch, 8) * 8 * m);
  ProfScope ps(MIPQ_K_FIT_ROUND_BF16, s);
#define LAUNCH1(NB, NT, FULL)                                                                             \
  k_fit_round_bf16<NB, NT, FULL><<<grid, fit_waves(NB) * 64, lds, s>>>(                                    \
      x, n, d, m, ks, ds, (const bf16x8*)aop, cmax, mu, c32, codes, resc, g.nch, g.rpw, bd.e_cross,          \
      bd.e_norm, bd.g_exact, part_s, part_cnt, cmax_zero)
#define LAUNCH(NB, NT)                 \
  do {                                 \
    if (full) LAUNCH1(NB, NT, true);   \
    else LAUNCH1(NB, NT, false);       \
  } while (0)
  if (nb == 1) {
    switch (nt) {
      case 1: LAUNCH(1, 1); break;
      case 2: LAUNCH(1, 2); break;
      case 4: LAUNCH(1, 4); break;
      default: LAUNCH(1, 8); break;
    }
  } else {
    switch (nt) {
      case 1: LAUNCH(2, 1); break;
      case 2: LAUNCH(2, 2); break;
      case 4: LAUNCH(2, 4); break;
      default: LAUNCH(2, 8); break;
    }
  }
#undef LAUNCH
#undef LAUNCH1
  MIPQ_LAUNCHED("k_fit_round_bf16");
  return MIPQ_OK;
}

namespace {
template <int NB, int NT, bool FULL, bool REG>
const void* batched_fn() {
  return reinterpret_cast<const void*>(&k_assign_bf16_batched<NB, NT, FULL, REG>);
}
// variant 0: pending rows re-decided one at a time; variant 1: register form
template <int NB, int NT>
const void* batched_pick(bool full, int variant) {
  if (variant == 0) return full ? batched_fn<NB, NT, true, false>() : batched_fn<NB, NT, false, false>();
  return full ? batched_fn<NB, NT, true, true>() : batched_fn<NB, NT, false, true>();
}
const void* pick_batched(int ds, int ks, bool full, int variant) {
  const int nb = (ds + 7) / 8;
  const int nt = tiles_for(ks);
#define PICK(NB)                                                  \
  switch (nt) {                                                   \
    case 1: return batched_pick<NB, 1>(full, variant);            \
    case 2: return batched_pick<NB, 2>(full, variant);            \
    case 4: return batched_pick<NB, 4>(full, variant);            \
    default: return batched_pick<NB, 8>(full, variant);           \
  }
  if (nb == 1) PICK(1)
  PICK(2)
#undef PICK
}
}  // namespace

int assign_bf16_batched_resident(int ds, int ks, bool full, int variant, int* resident) {
  int per_cu = 0, dev = 0, cus = 0;
  MIPQ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, pick_batched(ds, ks, full, variant), kThreads, 0));
  MIPQ_HIP(hipGetDevice(&dev));
  MIPQ_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  *resident = per_cu * cus;
  return MIPQ_OK;
}

int launch_assign_bf16_batched(const BatchProb* probs, int nprob, int64_t units, int d, int m, int ks,
                               const void* aop, size_t aop_stride, const float* cmax, const float* mu, bool full,
                               int variant, int grid, int64_t* rescored, hipStream_t s) {
  if (units == 0) return MIPQ_OK;
  if (grid < 8 || grid % 8) return fail(MIPQ_EINVAL, "batched assignment grid must be a positive multiple of 8");
  const int ds = d / m;
  Band bd = band_for(ds);
  unsigned long long* resc = reinterpret_cast<unsigned long long*>(rescored);
  ProfScope ps(MIPQ_K_ASSIGN_BF16_BATCHED, s);
  void* args[] = {(void*)&probs, (void*)&nprob, (void*)&units, (void*)&d, (void*)&m, (void*)&ks, (void*)&ds,
                  (void*)&aop, (void*)&aop_stride, (void*)&cmax, (void*)&mu, (void*)&resc,
                  (void*)&bd.e_cross, (void*)&bd.e_norm, (void*)&bd.g_exact};
  MIPQ_HIP(hipLaunchKernel(pick_batched(ds, ks, full, variant), dim3(grid), dim3(kThreads), args, 0, s));
  return MIPQ_OK;
}

size_t fp8_operand_count(int m, int ks) { return (size_t)m * tiles_for(ks) * 64; }
size_t fp8_stats_count(int m) { return (size_t)m * kFp8Stats; }

int launch_pack_fp8(const float* c32, int m, int ks, int ds, void* aop, float* stats, hipStream_t s) {
  const int nt = tiles_for(ks);
  ProfScope ps(MIPQ_K_PACK_FP8, s);
  if (ds <= 8)
    k_pack_fp8<1><<<m, 256, 0, s>>>(c32, ks, ds, nt, (i32x8*)aop, stats);
  else
    k_pack_fp8<2><<<m, 256, 0, s>>>(c32, ks, ds, nt, (i32x8*)aop, stats);
  MIPQ_LAUNCHED("k_pack_fp8");
  return MIPQ_OK;
}

int launch_assign_fp8(const float* x, int64_t n, int d, int m, int ks, const void* aop, const float* stats,
                      const float* c32, uint8_t* codes, int64_t* rescored, hipStream_t s) {
  const int ds = d / m;
  const int nb = (ds + 7) / 8;
  const int nt = tiles_for(ks);
  const Bf16Geom g = bf16_geometry(n, m, 64);
  if (g.blocks == 0) return MIPQ_OK;
  const float g_exact = band_for(ds).g_exact;
  ProfScope ps(MIPQ_K_ASSIGN_FP8, s);
  const bool full = (ds == nb * 8) && (d % 4 == 0) && ((reinterpret_cast<uintptr_t>(x) & 15) == 0);
  unsigned long long* resc = reinterpret_cast<unsigned long long*>(rescored);
  const size_t pend_bytes = (size_t)(kThreads / 64) * g.rpb * sizeof(uint32_t);
#define LAUNCH(NB, NT)                                                                                         \
  do {                                                                                                         \
    if (full)                                                                                                  \
      k_assign_fp8<NB, NT, true><<<g.blocks, kThreads, pend_bytes, s>>>(x, n, d, m, ks, ds, (const i32x8*)aop, \
                                                                        stats, c32, codes, resc, g.groups,     \
                                                                        g.rpb, g_exact);                       \
    else                                                                                                       \
      k_assign_fp8<NB, NT, false><<<g.blocks, kThreads, pend_bytes, s>>>(x, n, d, m, ks, ds,                   \
                                                                         (const i32x8*)aop, stats, c32, codes, \
                                                                         resc, g.groups, g.rpb, g_exact);      \
  } while (0)
  if (nb == 1) {
    switch (nt) {
      case 1: LAUNCH(1, 1); break;
      case 2: LAUNCH(1, 2); break;
      case 4: LAUNCH(1, 4); break;
      default: LAUNCH(1, 8); break;
    }
  } else {
    switch (nt) {
      case 1: LAUNCH(2, 1); break;
      case 2: LAUNCH(2, 2); break;
      case 4: LAUNCH(2, 4); break;
      default: LAUNCH(2, 8); break;
    }
  }
#undef LAUNCH
  MIPQ_LAUNCHED("k_assign_fp8");
  return MIPQ_OK;
}

}  // namespace mipq
