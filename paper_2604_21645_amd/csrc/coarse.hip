// Coarse k-means quantiser (paper Section 2.2: rows are bucketed for the
// inverted file; the buckets here are coarse k-means lists, see the
// inverted-index reading): the centre and operand packing of the Kc
// centroids and the assignment of rows to their nearest centroid.
//
// Exact rule: label = argmin_l ||x - c_l||^2 over Kc full-dimension
// centroids, float32 differences squared and summed in float64 in ascending
// dimension order, lowest index on ties.  Ranked on matrix cores (32x32x16
// bfloat16 MFMA, centred operands, squared norms folded into the
// contraction); rows whose best two estimates are not separated by the proven
// error bound are re-decided with the exact rule.
//
// Compiled without NaN semantics (like the PQ matrix-core kernels): minima of
// matrix-core estimates need no quieting of signalling NaNs.
#include <math.h>

#include <type_traits>

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
// 32-centroid tile the block stages the tile's S+1 operands in LDS once for its
// four waves; each wave runs S+1 MFMAs per row group and lane l receives 16
// distance estimates of its row (centroids 8(r/4) + 4h + r%4 of the tile).
//
// First launch (k_coarse_assign_mfma): the best two estimates of every row.
// A row they separate by the proven error bound gets its label; any other row
// (ambiguous) keeps its best estimate f1 in its label slot, encoded as a
// negative integer.  Second launch (k_coarse_resolve_mfma): the ambiguous rows,
// gathered into full waves, recompute their estimates, collect every (row,
// centroid) whose estimate is within the bound of f1 (the exact winner is
// always among them) in an LDS list and are decided by the exact rule over
// their candidates only.  A row whose candidates do not fit the list is
// decided by the exact rule over all centroids.

// candidate pairs per wave of the resolve launch
constexpr int kCandCap = 640;

// bits of a tile index (nt tiles), at least 1
__device__ __forceinline__ int coarse_tile_bits(int nt) { return nt > 1 ? 32 - __clz(nt - 1) : 1; }

// f1 of an ambiguous row in its label slot: the float's bits shifted right by
// one under a set sign bit (the float's sign moves to bit 30; the dropped bit
// 0 is one unit in the last place, inside the key quantisation the bound
// already allows).  Decided labels are in [0, kc).
__device__ __forceinline__ int32_t coarse_encode_f1(float f) {
  return (int32_t)(0x80000000u | ((uint32_t)__float_as_int(f) >> 1));
}
__device__ __forceinline__ float coarse_decode_f1(int32_t v) { return __int_as_float((int)((uint32_t)v << 1)); }

// relative quantisation of estimates read back from keys that drop the low tb
// (tile) or 4 (register) mantissa bits: 2^(max(tb, 4) + 1 - 23)
__device__ __forceinline__ float coarse_key_quant(int tb) {
  return __int_as_float((127 - 23 + (tb > 4 ? tb : 4) + 1) << 23);
}

// Row operands (centred, bfloat16) of the wave's row groups and the rows'
// ||x - mu||^2 (float32), with its three bfloat16 pieces in K-step S.
// row_at(i) is the row of local index i = 32 g + row-in-group, or -1 (a
// missing row reads row n - 1 and is never written).
template <int S, int RG, typename RowAt>
__device__ __forceinline__ void coarse_row_operands(const float* __restrict__ x, int64_t n, int d,
                                                    const float* __restrict__ mu, RowAt row_at,
                                                    bf16x8 (&B)[RG][S + 1], float (&xn)[RG]) {
  const int lane = threadIdx.x & 63;
  const int h = lane >> 5;
  // every row slice is whole and 16-byte aligned (mu is a workspace buffer)
  const bool vec = d == 16 * S && (reinterpret_cast<uintptr_t>(x) & 15) == 0 &&
                   (reinterpret_cast<uintptr_t>(mu) & 15) == 0;
#pragma unroll
  for (int g = 0; g < RG; ++g) {
    const int64_t row = row_at(32 * g + (lane & 31));
    const float* xr = x + (row >= 0 ? row : n - 1) * d;
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
}

// s_waitcnt operand: at most n vector memory operations of the wave
// outstanding, no LDS operation (expcnt left alone)
constexpr int waitcnt_vm_lgkm0(int n) { return (n & 15) | (7 << 4) | ((n >> 4) << 14); }

// The estimates of one tile for the wave's row groups, from its staged
// operands.  They are read through a restrict pointer, so the LDS reads carry
// an alias scope while the loads into the ring carry none (the operand
// pointer of coarse_sweep and its callers are not restrict): the compiler's
// wait insertion then leaves the loads in flight alone, and the waits of the
// ring are the explicit ones at the end of each tile.
template <int NK, int RG>
__device__ __forceinline__ void coarse_tile_mfma(const bf16x8* __restrict__ a, int lane, const bf16x8 (&B)[RG][NK],
                                                 f32x16 (&acc)[RG]) {
#pragma unroll
  for (int g = 0; g < RG; ++g) acc[g] = f32x16{};
#pragma unroll
  for (int s = 0; s < NK; ++s) {
    const bf16x8 av = a[s * 64 + lane];
#pragma unroll
    for (int g = 0; g < RG; ++g) acc[g] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, B[g][s], acc[g], 0, 0, 0);
  }
}

// The tile loop of both launches.  Tile t's operands are staged in LDS once for
// the block's four waves, in a ring of P buffers: at the start of tile t the
// chunks of tile t + P - 1 go from memory straight to the buffer tile t - 1
// used (global_load_lds, no registers held), so each tile's operands are
// requested P - 1 tiles before they are read.  The barrier that ends tile t
// waits only for the wave's loads of tile t + 1 (its vector memory counter
// may keep the younger tiles' loads outstanding: every wave issues at least
// cnt_min chunks per tile) and for its LDS reads, so the buffer refilled next
// is free.  (A release fence would also wait for the loads in flight, as they
// write LDS.)  epi(t, g, acc)
// receives the 16 estimates of row group g.  Every wave of the block runs
// every tile.
template <int S, int RG, int P, typename Epi>
__device__ __forceinline__ void coarse_sweep(const bf16x8* aop, bf16x8* ring, int nt, const bf16x8 (&B)[RG][S + 1],
                                             Epi&& epi) {
  static_assert(P >= 2, "at least two operand buffers");
  constexpr int NK = S + 1;
  constexpr int CH = NK * 64;               // 16-byte operand chunks per tile
  constexpr int PT = (CH + kT - 1) / kT;    // chunks per thread
  // chunks per tile of the wave that issues the fewest (the last one)
  constexpr int cnt_min = CH > kT - 64 ? (CH - (kT - 64) + kT - 1) / kT : 0;
  constexpr int keep = (P - 2) * cnt_min;   // loads that may stay in flight at a tile's end
  static_assert(keep < 64, "vector memory counter range");
  const int lane = threadIdx.x & 63;
  const int wbase = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) * 64;
  auto fetch = [&](int t, int buf) {
#pragma unroll
    for (int i = 0; i < PT; ++i) {
      const int c = threadIdx.x + i * kT;   // lane l of wave w lands in slot wbase + i kT + l (wave-uniform test)
      if (c < CH)
        __builtin_amdgcn_global_load_lds(static_cast<const void*>(aop + (size_t)t * CH + c),
                                         (__attribute__((address_space(3))) void*)(ring + buf * CH + wbase + i * kT),
                                         16, 0, 0);
    }
  };
  // the end of a tile: wait until at most n loads of the wave are in flight
  // and its LDS reads are done, then the block's barrier
  auto tile_end = [&](auto n) {
    __builtin_amdgcn_s_waitcnt(waitcnt_vm_lgkm0(decltype(n)::value));
    __builtin_amdgcn_s_barrier();
  };
  auto score = [&](int t, int cur) {
    f32x16 acc[RG];
    coarse_tile_mfma<NK, RG>(ring + cur * CH, lane, B, acc);
#pragma unroll
    for (int g = 0; g < RG; ++g) epi(t, g, acc[g]);
  };
  using keep_c = std::integral_constant<int, keep>;
  using none_c = std::integral_constant<int, 0>;
#pragma unroll
  for (int i = 0; i < P - 1; ++i)
    if (i < nt) fetch(i, i);
  if (P - 2 < nt) tile_end(keep_c{});   // tile 0 loaded, tiles 1 .. P - 2 may be in flight
  else tile_end(none_c{});
  int cur = 0;
  int t = 0;
  // tiles whose successor's loads are followed by P - 2 younger tiles' loads
  for (; t + P - 1 < nt; ++t) {
    fetch(t + P - 1, cur == 0 ? P - 1 : cur - 1);   // the buffer of tile t - 1
    score(t, cur);
    tile_end(keep_c{});
    cur = cur == P - 1 ? 0 : cur + 1;
  }
  for (; t < nt; ++t) {   // the last P - 1 tiles: nothing left to fetch
    score(t, cur);
    tile_end(none_c{});
    cur = cur == P - 1 ? 0 : cur + 1;
  }
}

// operand buffers of the first launch (three blocks per CU) and of the resolve
// launch (two blocks per CU beside the candidate lists)
constexpr int coarse_ring_assign(int S) { return S <= 12 ? 4 : 3; }
constexpr int coarse_ring_resolve(int S) { return S <= 8 ? 4 : (S <= 12 ? 3 : 2); }
// 16-byte operand chunks of one tile
constexpr int coarse_tile_chunks(int S) { return (S + 1) * 64; }

// minimum of the 16 estimates of a lane
__device__ __forceinline__ float coarse_tile_min(const f32x16& acc) {
  const float m0 = fminf(fminf(acc[0], acc[1]), acc[2]);
  const float m1 = fminf(fminf(acc[3], acc[4]), acc[5]);
  const float m2 = fminf(fminf(acc[6], acc[7]), acc[8]);
  const float m3 = fminf(fminf(acc[9], acc[10]), acc[11]);
  const float m4 = fminf(fminf(acc[12], acc[13]), acc[14]);
  return fminf(fminf(fminf(m0, m1), m2), fminf(fminf(m3, m4), acc[15]));
}

// error bound of one estimate: single bfloat16 cross products (e_cross of
// |x - mu| |c - mu|, cm bounding the centroids' centred norms) and the
// float32 norm pieces (e_norm)
__device__ __forceinline__ float coarse_beta(float xn, float cm, float e_cross, float e_norm) {
  return e_cross * sqrtf(xn) * 1.0001f * cm + e_norm * (cm * cm + xn);
}

// Rows r0 .. r0 + 32 RG - 1 of the wave (lanes l and l ^ 32 share row l % 32
// of each group): labels of the separated rows, encoded f1 of the others.
template <int S, int RG>
__global__ __launch_bounds__(kT, 3) void k_coarse_assign_mfma(
    const float* __restrict__ x, int64_t n, int d, int kc, const bf16x8* aop,
    const float* __restrict__ mu, const unsigned int* __restrict__ cmax_bits, int32_t* __restrict__ labels,
    unsigned long long* __restrict__ rescored, float e_cross, float e_norm, float g_exact) {
  constexpr int NK = S + 1;
  const int lane = threadIdx.x & 63;
  const int h = lane >> 5;
  const int w = threadIdx.x >> 6;
  const int64_t r0 = ((int64_t)blockIdx.x * (kT / 64) + w) * (32 * RG);
  auto row_at = [&](int i) -> int64_t { return r0 + i < n ? r0 + i : -1; };
  __shared__ bf16x8 ring[coarse_ring_assign(S) * coarse_tile_chunks(S)];   // the kernel's only LDS object
  const float cm = __uint_as_float(*cmax_bits);
  bf16x8 B[RG][NK];
  float xn[RG];
  coarse_row_operands<S, RG>(x, n, d, mu, row_at, B, xn);

  // Per lane and row group, two groupings of the lane's 16 candidates of every
  // tile: by accumulator register over all tiles (bmin) and by tile (the two
  // smallest tile minima, kept as integer keys: the float's bits with the tile
  // index in the low tb bits, a1 <= a2).  Two candidates of a lane differ in
  // tile or in register, so the best estimate, its tile and register, and the
  // runner-up all follow from them (one minimum per candidate and a few
  // instructions per tile, instead of a compare-and-select per candidate).
  const int nt = (kc + 31) / 32;
  const int tb = coarse_tile_bits(nt);
  const int tmask = (1 << tb) - 1;
  float bmin[RG][16];
  int a1[RG], a2[RG];
#pragma unroll
  for (int g = 0; g < RG; ++g) {
    a1[g] = INT_MAX;
    a2[g] = INT_MAX;
#pragma unroll
    for (int r = 0; r < 16; ++r) bmin[g][r] = INFINITY;
  }
  coarse_sweep<S, RG, coarse_ring_assign(S)>(aop, ring, nt, B, [&](int t, int g, const f32x16& acc) {
    const float tmin = coarse_tile_min(acc);
#pragma unroll
    for (int r = 0; r < 16; ++r) bmin[g][r] = fminf(bmin[g][r], acc[r]);
    const int key = (__float_as_int(tmin) & ~tmask) | t;
    a2[g] = min(a2[g], max(a1[g], key));
    a1[g] = min(a1[g], key);
  });

  // merge the two lanes of each row; separation test
  const float qk = coarse_key_quant(tb);
#pragma unroll
  for (int g = 0; g < RG; ++g) {
    // register grouping: the two smallest register minima as keys
    int b1 = INT_MAX, b2 = INT_MAX;
#pragma unroll
    for (int r = 0; r < 16; r += 2) {
      const int ka = (__float_as_int(bmin[g][r]) & ~15) | r;
      const int kb = (__float_as_int(bmin[g][r + 1]) & ~15) | (r + 1);
      b2 = min(b2, max(min(ka, kb), min(max(ka, kb), b1)));   // runner-up of {b1, b2, ka, kb}, b1 <= b2 (med3)
      b1 = min(b1, min(ka, kb));
    }
    const int s2 = min(a2[g], b2);
    // the two lanes of a row (l and l ^ 32): lane l % 32 holds candidates
    // 8j + 0..3 of every tile, lane 32 + l % 32 candidates 8j + 4..7
    const auto A1 = __builtin_amdgcn_permlane32_swap(a1[g], a1[g], false, false);
    const auto S2 = __builtin_amdgcn_permlane32_swap(s2, s2, false, false);
    const auto RL = __builtin_amdgcn_permlane32_swap(b1 & 15, b1 & 15, false, false);
    const int a1l = (int)A1[0], a1h = (int)A1[1];
    const bool hiw = a1h < a1l;
    const int w1 = min(a1l, a1h);
    const int sec = min(max(a1l, a1h), min((int)S2[0], (int)S2[1]));
    const int tw = (hiw ? a1h : a1l) & tmask;
    const int rw = hiw ? (int)RL[1] : (int)RL[0];
    const float f1 = __int_as_float(w1);
    const float f2 = __int_as_float(sec);
    const int code = tw * 32 + (rw >> 2) * 8 + (hiw ? 4 : 0) + (rw & 3);
    const float beta = coarse_beta(xn[g], cm, e_cross, e_norm);
    const float gap = f2 - f1;
    const float thr = 2.0f * beta + g_exact * (fabsf(f1) + fabsf(f2) + 2.0f * beta + 2.0f * xn[g] * g_exact) +
                      qk * (fabsf(f1) + fabsf(f2));
    const int64_t row = row_at(32 * g + (lane & 31));
    const bool amb = row >= 0 && (!(gap > thr) || code >= kc);
    if (h == 0 && row >= 0) labels[row] = amb ? coarse_encode_f1(f1) : code;
    const uint64_t ab = __ballot(h == 0 && amb);
    if (rescored && lane == 0 && ab) atomicAdd(rescored, (unsigned long long)__popcll(ab));
  }
}

// Decide the rows rlist[w 32 RG + i] (i < 32 RG, slots past take are empty) of
// wave w: candidates within the bound of each row's f1 (from its label slot),
// then the exact rule over them.  Every wave meets the block's barriers.
template <int S, int RG>
__device__ __forceinline__ void coarse_resolve_rows(const float* x, int64_t n, int d, int kc, const bf16x8* aop,
                                                    const float* mu, const unsigned int* cmax_bits, const float* cc,
                                                    int32_t* labels, float e_cross, float e_norm, float g_exact,
                                                    const int32_t* rlist, int take, bf16x8* ring,
                                                    uint32_t* cand_rk_all, double* cand_d_all) {
  constexpr int NK = S + 1;
  const int lane = threadIdx.x & 63;
  const int h = lane >> 5;
  const int w = threadIdx.x >> 6;
  auto row_at = [&](int i) -> int64_t {
    const int slot = w * (32 * RG) + i;
    return slot < take ? (int64_t)rlist[slot] : -1;
  };
  uint32_t* cand_rk = cand_rk_all + w * kCandCap;   // (row in wave) << 16 | centroid
  double* cand_d = cand_d_all + w * kCandCap;
  const float cm = __uint_as_float(*cmax_bits);
  bf16x8 B[RG][NK];
  float xn[RG];
  coarse_row_operands<S, RG>(x, n, d, mu, row_at, B, xn);
  const int nt = (kc + 31) / 32;
  const float qk = coarse_key_quant(coarse_tile_bits(nt));
  // Candidate test: est - f1 <= c0 + c1 |est| (the separation bound, the
  // row's terms gathered in c0).  Every estimate that passes it is at most
  // T = f1 + c0 + 2 c1 (|f1| + c0) (c1 < 1/2), so the pass keeps the
  // estimates up to T: a superset by at most c1 |est|, decided exactly all
  // the same, for one compare per estimate.
  const float c1 = g_exact + qk;
  float thr[RG];
  bool valid[RG];
#pragma unroll
  for (int g = 0; g < RG; ++g) {
    const int64_t row = row_at(32 * g + (lane & 31));
    valid[g] = row >= 0;
    const float f1 = valid[g] ? coarse_decode_f1(labels[row]) : 0.0f;
    const float beta = coarse_beta(xn[g], cm, e_cross, e_norm);
    const float c0 = 2.0f * beta + g_exact * (fabsf(f1) + 2.0f * beta + 2.0f * xn[g] * g_exact) + qk * fabsf(f1);
    const float tt = f1 + c0 + 2.0f * c1 * (fabsf(f1) + c0);
    thr[g] = valid[g] ? tt + fabsf(tt) * 0x1p-20f : -INFINITY;   // and the rounding of T
  }
  int nc = 0;
  bool ovf[RG];
#pragma unroll
  for (int g = 0; g < RG; ++g) ovf[g] = false;
  coarse_sweep<S, RG, coarse_ring_resolve(S)>(aop, ring, nt, B, [&](int t, int g, const f32x16& acc) {
    // no candidate of the wave in this tile unless some lane's smallest
    // estimate is within its threshold (padded centroids estimate +inf)
    if (!__ballot(coarse_tile_min(acc) <= thr[g])) return;   // wave-uniform
    const uint32_t rl = (uint32_t)(32 * g + (lane & 31)) << 16;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const bool cand = acc[r] <= thr[g];
      const uint64_t m = __ballot(cand);
      if (!m) continue;   // wave-uniform
      if (cand) {
        const int pos =
            nc + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        const int k = t * 32 + (r >> 2) * 8 + h * 4 + (r & 3);
        if (pos >= kCandCap) ovf[g] = true;
        else if (k < kc) cand_rk[pos] = rl | (uint32_t)k;
        else cand_rk[pos] = rl | (uint32_t)(kc - 1);   // never: a padded centroid estimates +inf
      }
      nc += __popcll(m);
    }
  });
  const int ncl = nc < kCandCap ? nc : kCandCap;
  __builtin_amdgcn_wave_barrier();
  for (int i = lane; i < ncl; i += 64) {
    const uint32_t rk = cand_rk[i];
    const int64_t row = row_at((int)(rk >> 16));
    cand_d[i] = coarse_exact_dist(x + row * d, cc + (int64_t)(rk & 0xFFFFu) * d, d);
  }
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int g = 0; g < RG; ++g) {
    // a row overflowed when either of its two lanes dropped a candidate
    const uint64_t ob = __ballot(ovf[g]);
    const uint32_t rows_full = (uint32_t)(ob | (ob >> 32));
    const int64_t row = row_at(32 * g + (lane & 31));
    if (h == 0 && valid[g] && !((rows_full >> (lane & 31)) & 1u)) {
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
    uint32_t fm = rows_full & (uint32_t)__ballot(h == 0 && valid[g]);
    while (fm) {   // wave-uniform
      const int l = __ffs(fm) - 1;
      fm &= fm - 1;
      const int64_t frow = row_at(32 * g + l);
      const int ec = coarse_exact_wave(x + frow * d, cc, kc, d, lane);
      if (lane == 0) labels[frow] = ec;
    }
  }
}

// The rows that k_coarse_assign_mfma left ambiguous (negative label), gathered:
// block b scans rows [b span, (b + 1) span) kPer kT at a time, collects them in
// LDS and decides them kT / 64 * 32 RG at a time (full waves of such rows).
template <int S, int RG>
__global__ __launch_bounds__(kT, 2) void k_coarse_resolve_mfma(
    const float* __restrict__ x, int64_t n, int d, int kc, const bf16x8* aop,
    const float* __restrict__ mu, const unsigned int* __restrict__ cmax_bits, const float* __restrict__ cc,
    int32_t* __restrict__ labels, float e_cross, float e_norm, float g_exact, int64_t span) {
  constexpr int kRows = kT / 64 * 32 * RG;   // rows decided per pass of the block
  constexpr int kPer = 4;                     // labels scanned per thread and step
  // the kernel's only LDS object (separate objects would give the LDS reads
  // of the ring alias scopes that make the compiler wait for its loads):
  // operand ring, candidate lists, row list and its count
  constexpr size_t kRing = (size_t)coarse_ring_resolve(S) * coarse_tile_chunks(S) * 16;
  constexpr size_t kCand = (size_t)(kT / 64) * kCandCap;
  __shared__ __attribute__((aligned(16))) unsigned char lds[kRing + kCand * 12 + (kRows + kPer * kT + 1) * 4];
  bf16x8* ring = reinterpret_cast<bf16x8*>(lds);
  double* cand_d_all = reinterpret_cast<double*>(lds + kRing);
  uint32_t* cand_rk_all = reinterpret_cast<uint32_t*>(lds + kRing + kCand * 8);
  int32_t* rlist = reinterpret_cast<int32_t*>(lds + kRing + kCand * 12);
  int& rcnt = rlist[kRows + kPer * kT];
  int64_t pos = (int64_t)blockIdx.x * span;
  const int64_t end = min(n, pos + span);
  if (threadIdx.x == 0) rcnt = 0;
  __syncthreads();
  while (true) {
    while (pos < end && rcnt < kRows) {   // rcnt is read after a barrier: block-uniform
      const int64_t r = pos + (int64_t)kPer * threadIdx.x;
      int v[kPer];
#pragma unroll
      for (int u = 0; u < kPer; ++u) v[u] = r + u < end ? labels[r + u] : 0;
#pragma unroll
      for (int u = 0; u < kPer; ++u)
        if (v[u] < 0) rlist[atomicAdd(&rcnt, 1)] = (int32_t)(r + u);
      pos += (int64_t)kPer * kT;
      __syncthreads();
    }
    const int c = rcnt;
    if (c == 0) break;   // block-uniform; pos == end
    const int take = c < kRows ? c : kRows;
    coarse_resolve_rows<S, RG>(x, n, d, kc, aop, mu, cmax_bits, cc, labels, e_cross, e_norm, g_exact, rlist, take,
                               ring, cand_rk_all, cand_d_all);
    __syncthreads();
    // the rows not yet taken (fewer than kPer * kT) move to the front
    const int rest = c - take;
    int32_t keep[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int i = (int)threadIdx.x + j * kT;
      keep[j] = i < rest ? rlist[take + i] : 0;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int i = (int)threadIdx.x + j * kT;
      if (i < rest) rlist[i] = keep[j];
    }
    if (threadIdx.x == 0) rcnt = rest;
    __syncthreads();
    if (pos >= end && rest == 0) break;
  }
}

// the resolve launch: up to two blocks per CU on 256 CUs (its registers allow
// two waves per SIMD; fewer where the LDS of the operand buffers, the
// candidate lists and the row list does not fit two), each scanning at least
// kResolveMinSpan rows
constexpr int64_t kResolveMinSpan = 1024;
// up to this many rows the resolve launch is one pass per block, bound by the
// latency of the tile loop rather than by throughput: one row group per wave
// (S + 1 instead of 2 (S + 1) MFMAs per tile and wave) and spans of at least
// kResolveMinSpanSmall rows (more, smaller blocks)
constexpr int64_t kResolveSmallN = int64_t(1) << 20;
constexpr int64_t kResolveMinSpanSmall = 256;

int resolve_blocks(int S, int RG) {
  const size_t lds = (size_t)coarse_ring_resolve(S) * coarse_tile_chunks(S) * 16 + (size_t)(kT / 64) * kCandCap * 12 +
                     ((size_t)(kT / 64) * 32 * RG + 4 * kT + 1) * 4;
  size_t per_cu = (size_t)160 * 1024 / lds;
  if (per_cu > 2) per_cu = 2;
  if (per_cu < 1) per_cu = 1;
  return int(256 * per_cu);
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
  // the row operands fit the registers; then the ambiguous rows, gathered by
  // a second launch so that the candidate pass runs for full waves of them
#define CA(SV)                                                                                                  \
  do {                                                                                                          \
    constexpr int RGV = SV <= 8 ? 2 : 1;                                                                        \
    const int blocks = ceil_div((n + 32 * RGV - 1) / (32 * RGV), kT / 64);                                      \
    k_coarse_assign_mfma<SV, RGV><<<blocks, kT, 0, s>>>(x, n, d, kc, (const bf16x8*)aop, mu, cmax_bits, labels, \
                                                        resc, e_cross, e_norm, g_exact);                        \
    MIPQ_LAUNCHED("k_coarse_assign_mfma");                                                                      \
    if (n <= kResolveSmallN) { /* one pass per block: one row group per wave halves the tile latency */        \
      const int64_t rb = resolve_blocks(SV, 1);                                                                 \
      int64_t span = (n + rb - 1) / rb;                                                                         \
      if (span < kResolveMinSpanSmall) span = kResolveMinSpanSmall;                                             \
      k_coarse_resolve_mfma<SV, 1><<<ceil_div(n, span), kT, 0, s>>>(x, n, d, kc, (const bf16x8*)aop, mu,        \
                                                                    cmax_bits, cc, labels, e_cross, e_norm,     \
                                                                    g_exact, span);                             \
    } else {                                                                                                    \
      const int64_t rb = resolve_blocks(SV, RGV);                                                               \
      int64_t span = (n + rb - 1) / rb;                                                                         \
      if (span < kResolveMinSpan) span = kResolveMinSpan;                                                       \
      k_coarse_resolve_mfma<SV, RGV><<<ceil_div(n, span), kT, 0, s>>>(x, n, d, kc, (const bf16x8*)aop, mu,      \
                                                                      cmax_bits, cc, labels, e_cross, e_norm,   \
                                                                      g_exact, span);                           \
    }                                                                                                           \
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
  MIPQ_LAUNCHED("k_coarse_resolve_mfma");
  return MIPQ_OK;
}

}  // namespace mipq
