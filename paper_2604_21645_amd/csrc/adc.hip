// Asymmetric-distance (ADC) search over the inverted file (paper Section 2.2:
// a query returns its first to k-th nearest neighbours).
//
// 1. k_adc_dist: distance estimates of every (query, coarse centroid) pair on
//    matrix cores (queries as the A operand, the packed coarse operands as B).
// 2. k_adc_probe: per query, the nprobe lists with the smallest exact coarse
//    distance (float32 differences, float64 squares and sums), ties to the
//    lower list.  The estimate's error is at most beta, so every exact
//    top-nprobe list has an estimate <= T + 2 beta, T the nprobe-th smallest
//    estimate; exactly those candidates are re-scored with the exact rule and
//    sorted.
// 3. k_adc_scan: one block per (query, probed list l): the table
//    LUT[j][k] = subspace-j distance of (q - c_l) to C_j[k] (float32 rule),
//    then s = sum over j ascending of LUT[j][code_j] (float32) for every row
//    of the list; the list's topk smallest (s, id) pairs, kept with a
//    threshold and an LDS buffer.  The per-query threshold is shared through
//    global memory, so lists scanned later prune against earlier ones.
// 4. k_adc_merge: per query, the topk smallest of its lists' candidates.
#include <math.h>

#include <type_traits>

#include "bf16_pack.h"
#include "dist32.h"
#include "mipq_internal.h"

namespace mipq {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kT = 256;
constexpr int kTilesPerWave = 16;

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

// Wave (query group g of 32, tile range): A = centred queries (lane l: query
// l%32, dimensions 16s + 8h .. +7), B = packed coarse operands.  Output row
// q of est holds the kc estimates of query q.
template <int S>
__global__ __launch_bounds__(kT) void k_adc_dist(const float* __restrict__ q, int nq, int d, int kc,
                                                 const bf16x8* __restrict__ aop, const float* __restrict__ mu,
                                                 float* __restrict__ est) {
  constexpr int NK = S + 1;
  const int lane = threadIdx.x & 63;
  const int h = lane >> 5;
  const int nt = (kc + 31) / 32;
  const int tgroups = (nt + kTilesPerWave - 1) / kTilesPerWave;
  const int wid = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int g = wid / tgroups;
  const int tg = wid - g * tgroups;
  const int q0 = g * 32;
  if (q0 >= nq) return;
  const int qi = q0 + (lane & 31);
  const float* qr = q + (int64_t)(qi < nq ? qi : q0) * d;
  bf16x8 A[NK];
  float xn_part = 0.0f;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    float v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int dim = 16 * s + 8 * h + e;
      const float xv = qr[dim < d ? dim : d - 1];
      v[e] = dim < d ? xv - mu[dim] : 0.0f;
      xn_part = xn_part + v[e] * v[e];
    }
    A[s] = to_bf16x8(v);
  }
  const auto sw = __builtin_amdgcn_permlane32_swap(__float_as_int(xn_part), __float_as_int(xn_part), false, false);
  const float xn = __int_as_float((int)sw[0]) + __int_as_float((int)sw[1]);
  {
    bf16x8 nb = {};
    if (h == 0) {
      const __bf16 hb = (__bf16)xn;
      const float r1 = xn - (float)hb;
      const __bf16 mb = (__bf16)r1;
      nb[0] = nb[1] = nb[2] = (__bf16)1.0f;
      nb[3] = hb;
      nb[4] = mb;
      nb[5] = (__bf16)(r1 - (float)mb);
    }
    A[S] = nb;
  }
  const int t0 = tg * kTilesPerWave;
  const int t1 = min(nt, t0 + kTilesPerWave);
  for (int t = t0; t < t1; ++t) {
    f32x16 acc = {};
#pragma unroll
    for (int s = 0; s < NK; ++s)
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[s], aop[((size_t)t * NK + s) * 64 + lane], acc, 0, 0, 0);
    const int k = t * 32 + (lane & 31);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int qq = q0 + (r >> 2) * 8 + h * 4 + (r & 3);
      if (qq < nq && k < kc) est[(int64_t)qq * kc + k] = acc[r];
    }
  }
}

// qs: the query row in LDS.  vec (c 16-byte aligned, d % 16 == 0): the row
// of c is read 16 floats at a time, the next 16 in flight while the current
// ones are summed; the sum itself runs over t ascending either way.
__device__ __forceinline__ double coarse_exact(const float* qs, const float* __restrict__ c, int d, bool vec) {
  double acc = 0.0;
  if (vec) {
    const float4* c4 = reinterpret_cast<const float4*>(c);
    const int nch = d >> 4;
    float4 cur[4], nxt[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) cur[k] = c4[k];
    for (int ch = 0; ch < nch; ++ch) {
      if (ch + 1 < nch) {
#pragma unroll
        for (int k = 0; k < 4; ++k) nxt[k] = c4[(ch + 1) * 4 + k];
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float cv[4] = {cur[k].x, cur[k].y, cur[k].z, cur[k].w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const double df = (double)(qs[ch * 16 + k * 4 + i] - cv[i]);
          acc = acc + df * df;
        }
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) cur[k] = nxt[k];
    }
    return acc;
  }
  for (int t = 0; t < d; ++t) {
    const double df = (double)(qs[t] - c[t]);
    acc = acc + df * df;
  }
  return acc;
}

// order-preserving uint of a float (negatives below positives)
__device__ __forceinline__ uint32_t fkey(float f) {
  const uint32_t b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

struct DK {   // (distance, list) ordered lexicographically
  double d;
  int l;
};
__device__ __forceinline__ bool dk_less(const DK& a, const DK& b) { return a.d < b.d || (a.d == b.d && a.l < b.l); }

constexpr int kBandMax = 512;
constexpr int kMaxCoarseD = 256;   // the search's coarse matrix-core path takes d <= 256

// One block per query: select the nprobe lists (exact rule, ties to the lower
// list) from the estimates; see the file comment for the band argument.
__global__ __launch_bounds__(kT) void k_adc_probe(const float* __restrict__ q, int d, const float* __restrict__ cc,
                                                  int kc, const float* __restrict__ est, const float* __restrict__ mu,
                                                  const unsigned int* __restrict__ cmax_bits, int nprobe,
                                                  float e_cross, float e_norm, float g_exact,
                                                  int32_t* __restrict__ probes, unsigned long long* __restrict__ wide) {
  __shared__ uint32_t hist[256];
  __shared__ uint32_t sel_prefix, sel_need;
  __shared__ DK band[kBandMax];
  __shared__ int nband;
  __shared__ float red[kT / 64];
  __shared__ float qs[kMaxCoarseD];
  const int qi = blockIdx.x;
  const float* qr = q + (int64_t)qi * d;
  const float* er = est + (int64_t)qi * kc;
  const bool vec = ((reinterpret_cast<uintptr_t>(cc) & 15) == 0) && (d % 16 == 0);
  for (int t = threadIdx.x; t < d; t += blockDim.x) qs[t] = qr[t];
  // ||q - mu|| for the error bound
  float xn = 0.0f;
  for (int t = threadIdx.x; t < d; t += blockDim.x) {
    const float v = qr[t] - mu[t];
    xn += v * v;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) xn += __shfl_xor(xn, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = xn;
  // radix select of the nprobe-th smallest estimate (order-preserving keys)
  if (threadIdx.x == 0) {
    sel_prefix = 0u;
    sel_need = (uint32_t)nprobe;
    nband = 0;
  }
  __syncthreads();
  float xs = 0.0f;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) xs += red[i];
  // the thread's estimates l = tid + i * kT, held in registers when Kc fits
  constexpr int kEstRegs = 16;
  const bool in_regs = kc <= kEstRegs * kT;   // block-uniform
  uint32_t ek[kEstRegs];
  if (in_regs) {
#pragma unroll
    for (int i = 0; i < kEstRegs; ++i) {
      const int l = threadIdx.x + i * kT;
      ek[i] = l < kc ? fkey(er[l]) : 0xFFFFFFFFu;
    }
  }
  for (int shift = 24; shift >= 0; shift -= 8) {
    hist[threadIdx.x] = 0u;
    __syncthreads();
    const uint32_t pmask = shift == 24 ? 0u : (0xFFFFFFFFu << (shift + 8));
    const uint32_t pre = sel_prefix;
    if (in_regs) {
#pragma unroll
      for (int i = 0; i < kEstRegs; ++i)
        if (threadIdx.x + i * kT < kc && (ek[i] & pmask) == pre) atomicAdd(&hist[(ek[i] >> shift) & 255u], 1u);
    } else {
      for (int l = threadIdx.x; l < kc; l += blockDim.x) {
        const uint32_t k = fkey(er[l]);
        if ((k & pmask) == pre) atomicAdd(&hist[(k >> shift) & 255u], 1u);
      }
    }
    __syncthreads();
    // the digit: the first bin whose running count reaches sel_need (the
    // last bin at most); lane i of wave 0 holds bins 4i .. 4i + 3
    if (threadIdx.x < 64) {
      const int ln = threadIdx.x;
      uint32_t hh[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) hh[k] = hist[4 * ln + k];
      const uint32_t tot = hh[0] + hh[1] + hh[2] + hh[3];
      uint32_t inc = tot;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t v = __shfl_up(inc, o, 64);
        if (ln >= o) inc += v;
      }
      const uint32_t exc = inc - tot, need = sel_need;
      if ((exc < need && need <= inc) || (ln == 63 && inc < need)) {
        uint32_t nd = need - exc, b = 4 * ln;
        for (int k = 0; k < 3 && hh[k] < nd; ++k) {
          nd -= hh[k];
          ++b;
        }
        sel_prefix |= b << shift;
        sel_need = nd;
      }
    }
    __syncthreads();
  }
  const uint32_t tk = sel_prefix;
  const float T = __uint_as_float((tk & 0x80000000u) ? (tk & 0x7FFFFFFFu) : ~tk);
  const float cm = __uint_as_float(*cmax_bits);
  const float beta = e_cross * sqrtf(xs) * 1.0001f * cm + e_norm * (cm * cm + xs);
  const float lim = T + 2.0f * beta + g_exact * (2.0f * fabsf(T) + 4.0f * beta + 2.0f * xs * g_exact);
  // band members: listed first, then re-scored with the exact rule one per
  // thread, so that the lanes of a wave run their exact sums together
  bool overflow = false;
  auto add_member = [&](int l) {
    const int p = atomicAdd(&nband, 1);
    if (p < kBandMax) band[p].l = l;
  };
  if (in_regs) {
#pragma unroll
    for (int i = 0; i < kEstRegs; ++i) {
      const int l = threadIdx.x + i * kT;
      if (l < kc && er[l] <= lim) add_member(l);
    }
  } else {
    for (int l = threadIdx.x; l < kc; l += blockDim.x)
      if (er[l] <= lim) add_member(l);
  }
  __syncthreads();
  {
    const int nm = nband < kBandMax ? nband : kBandMax;
    for (int i = threadIdx.x; i < nm; i += blockDim.x) band[i].d = coarse_exact(qs, cc + (int64_t)band[i].l * d, d, vec);
  }
  __syncthreads();
  int nb = nband;
  if (nb > kBandMax) {
    overflow = true;
    nb = kBandMax;
  }
  if (overflow) {   // too many near the boundary: rank every list exactly, keep the nprobe best
    if (threadIdx.x == 0 && wide) atomicAdd(wide, 1ull);
    __syncthreads();
    if (threadIdx.x == 0) nband = 0;
    __syncthreads();
    // exact distances in chunks, merged with the best nprobe kept in front
    for (int next = 0; next < kc;) {
      const int keep = next == 0 ? 0 : nprobe;
      for (int i = threadIdx.x; i < kBandMax - keep; i += blockDim.x) {
        const int l = next + i;
        band[keep + i] = l < kc ? DK{coarse_exact(qs, cc + (int64_t)l * d, d, vec), l} : DK{INFINITY, 0x7FFFFFFF};
      }
      next += kBandMax - keep;
      __syncthreads();
      for (int kk = 2; kk <= kBandMax; kk <<= 1)
        for (int j = kk >> 1; j > 0; j >>= 1) {
          for (int i = threadIdx.x; i < kBandMax; i += blockDim.x) {
            const int ij = i ^ j;
            if (ij > i) {
              const bool up = (i & kk) == 0;
              const DK a = band[i], b = band[ij];
              if (up ? dk_less(b, a) : dk_less(a, b)) {
                band[i] = b;
                band[ij] = a;
              }
            }
          }
          __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < nprobe; i += blockDim.x) probes[(int64_t)qi * nprobe + i] = band[i].l;
    return;
  }
  // sort the band (padded to a power of two) and keep the first nprobe
  int p2 = 1;
  while (p2 < nb) p2 <<= 1;
  for (int i = nb + threadIdx.x; i < p2; i += blockDim.x) band[i] = DK{INFINITY, 0x7FFFFFFF};
  __syncthreads();
  for (int kk = 2; kk <= p2; kk <<= 1)
    for (int j = kk >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < p2; i += blockDim.x) {
        const int ij = i ^ j;
        if (ij > i) {
          const bool up = (i & kk) == 0;
          const DK a = band[i], b = band[ij];
          if (up ? dk_less(b, a) : dk_less(a, b)) {
            band[i] = b;
            band[ij] = a;
          }
        }
      }
      __syncthreads();
    }
  for (int i = threadIdx.x; i < nprobe; i += blockDim.x) probes[(int64_t)qi * nprobe + i] = i < nb ? band[i].l : -1;
}

constexpr int kBatch = kT;   // keys inserted per merge step (one per thread)
constexpr int kScanRows = 2;  // rows per thread per scan step
constexpr int kScanBatch = kScanRows * kT;
// M = 16 rows are first summed over their first kScanPre subspaces; table
// entries are non-negative and the float32 sum runs in a fixed order, so it
// never decreases, and a row whose partial sum is already above the bound
// cannot be inserted.  The other rows are finished from a per-wave queue.
constexpr int kScanPre = 4;
// table rows built before the scan (M = 16): they also give the list's lower bound
constexpr int kLutPre = 8;
static_assert(kScanPre <= kLutPre && kLutPre <= 16, "partial sums use built table rows");

// Ascending sort of buf[0, n), any n: a bitonic network in the form where
// every comparator is ascending (each merge first compares mirrored
// positions), so positions n and beyond act as +infinity and are never read.
__device__ void sort_keys(uint64_t* buf, int n) {
  int n2 = 1;
  while (n2 < n) n2 <<= 1;
  auto cswap = [&](int lo, int hi) {
    if (hi < n) {
      const uint64_t a = buf[lo], b = buf[hi];
      if (b < a) {
        buf[lo] = b;
        buf[hi] = a;
      }
    }
  };
  for (int kk = 2; kk <= n2; kk <<= 1) {
    const int h = kk >> 1;
    for (int i = threadIdx.x; i < (n2 >> 1); i += blockDim.x) {
      const int base = (i / h) * kk, off = i % h;
      cswap(base + off, base + kk - 1 - off);
    }
    __syncthreads();
    for (int j = kk >> 2; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < (n2 >> 1); i += blockDim.x) {
        const int lo = (i / j) * 2 * j + i % j;
        cswap(lo, lo + j);
      }
      __syncthreads();
    }
  }
}

__device__ __forceinline__ uint64_t load_relaxed(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Block-wide top-k collection of unique uint64 keys: a key is kept while it is
// <= *thr; once the LDS buffer (cap, a power of two) could not take another
// batch of `batch` keys, it is sorted, cut to the best topk and *thr lowered
// to the topk-th key (and to *ext, a bound shared with other blocks, when
// given).  Call after a barrier that follows the batch's insertions.
__device__ __forceinline__ void topk_compact(uint64_t* buf, int cap, int topk, int* cnt, uint64_t* thr,
                                             const unsigned long long* ext, int batch) {
  if (*cnt <= cap - batch) return;   // block-uniform
  const int c = *cnt < cap ? *cnt : cap;
  __syncthreads();
  sort_keys(buf, c);
  if (threadIdx.x == 0) {
    const int keep = c < topk ? c : topk;
    *cnt = keep;
    uint64_t t = *thr;
    if (keep == topk && buf[topk - 1] < t) t = buf[topk - 1];
    if (ext) {
      const uint64_t e = load_relaxed(ext);
      if (e < t) t = e;
    }
    *thr = t;
  }
  __syncthreads();
}

// final sort of the first c keys of buf
__device__ __forceinline__ void topk_finish(uint64_t* buf, int c) {
  __syncthreads();
  sort_keys(buf, c);
}

// Scan order of the (query, probe slot) pairs: probe rank major, so every
// query's nearest lists are scanned first and its bound tightens early; within
// a rank the pairs are bucketed by list, so the blocks that read one list run
// close together.  (Bucketing several ranks together shares a list among more
// queries but scans more candidates before the bounds tighten: on 10M rows,
// Kc = 4096, nprobe 32, one rank per bucketing is fastest.)  The order within
// a list does not change the search results.
constexpr int kXcdRun = 16;        // consecutive logical blocks given to one XCD
constexpr int kOrderT = 1024;
constexpr int kOrderMaxBins = 8192;   // LDS counters of k_pair_order

// one block per probe rank pi: pair ids pi * nq + qi bucketed by probed list
// (kc: no list), written to order[pi * nq, (pi + 1) * nq)
__global__ __launch_bounds__(kOrderT) void k_pair_order(const int32_t* __restrict__ probes, int nq, int nprobe,
                                                        int kc, int32_t* __restrict__ order) {
  extern __shared__ uint32_t cnt[];   // kc + 1
  __shared__ uint32_t part[kOrderT / 64];
  const int pi = blockIdx.x, nb = kc + 1;
  auto bin = [&](int qi) {
    const int l = probes[(int64_t)qi * nprobe + pi];
    return (l < 0 || l >= kc) ? kc : l;
  };
  for (int i = threadIdx.x; i < nb; i += kOrderT) cnt[i] = 0u;
  __syncthreads();
  for (int qi = threadIdx.x; qi < nq; qi += kOrderT) atomicAdd(&cnt[bin(qi)], 1u);
  __syncthreads();
  // exclusive prefix of the counts: thread t owns bins [t * per, (t + 1) * per)
  const int per = (nb + kOrderT - 1) / kOrderT;
  const int b0 = threadIdx.x * per;
  uint32_t tot = 0u;
  for (int i = 0; i < per; ++i)
    if (b0 + i < nb) tot += cnt[b0 + i];
  uint32_t inc = tot;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t v = __shfl_up(inc, o, 64);
    if ((threadIdx.x & 63) >= o) inc += v;
  }
  if ((threadIdx.x & 63) == 63) part[threadIdx.x >> 6] = inc;
  __syncthreads();
  uint32_t run = inc - tot;
  for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) run += part[w];
  for (int i = 0; i < per; ++i)
    if (b0 + i < nb) {
      const uint32_t c = cnt[b0 + i];
      cnt[b0 + i] = run;
      run += c;
    }
  __syncthreads();
  int32_t* out = order + (int64_t)pi * nq;
  for (int qi = threadIdx.x; qi < nq; qi += kOrderT) out[atomicAdd(&cnt[bin(qi)], 1u)] = pi * nq + qi;
}

// larger kc: the same order by the stable radix sort of the index build on
// the key pi * (kc + 1) + list
inline int order_labels(int nprobe, int kc) { return nprobe * (kc + 1); }

__global__ void k_pair_lists(const int32_t* __restrict__ probes, int nq, int nprobe, int kc,
                             int32_t* __restrict__ plab) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (int64_t)nq * nprobe) return;
  const int pi = (int)(p / nq);
  const int qi = (int)(p - (int64_t)pi * nq);
  const int l = probes[(int64_t)qi * nprobe + pi];
  plab[p] = pi * (kc + 1) + ((l < 0 || l >= kc) ? kc : l);
}

__global__ void k_fill_u64(unsigned long long* p, int n, unsigned long long v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Block = (probe slot pi, query qi), probe-major so that every query's nearest
// lists are scanned first.  LDS: the table (m*ks floats), the query residual
// (d floats) and the key buffer.  Keys: (score bits << 32 | id); scores are
// non-negative floats, so integer order is (score, id) order.  The block
// writes its list's best topk keys (~0 padded) and lowers the query's shared
// bound qthr to its topk-th key: a row above the topk-th key of any single
// list cannot be in the query's top topk.
template <int DS, bool V16, bool WORK>
__global__ __launch_bounds__(kT) void k_adc_scan(const float* __restrict__ q, int d, const float* __restrict__ cc,
                                                 const float* __restrict__ pq, int m, int ks,
                                                 const int64_t* __restrict__ offsets, const int32_t* __restrict__ ids,
                                                 const uint8_t* __restrict__ codes, const int32_t* __restrict__ probes,
                                                 int nq, int nprobe, int topk, int cap,
                                                 unsigned long long* __restrict__ qthr,
                                                 uint64_t* __restrict__ pair_out,
                                                 const int32_t* __restrict__ order, int npairs,
                                                 unsigned long long* __restrict__ work) {
  extern __shared__ float sm[];
  float* lut = sm;                                   // m*ks
  float* rq = lut + m * ks;                          // d
  uint64_t* buf = reinterpret_cast<uint64_t*>(rq + ((d + 1) & ~1));   // cap
  __shared__ int cnt;
  __shared__ uint64_t thr;
  __shared__ uint16_t wq[kScanBatch];   // per wave: its rows left after the partial sums
  __shared__ int need;                  // 1 + the last step at which a row needed the full table
  // logical block: runs of kXcdRun consecutive ones on one XCD (hardware
  // block id mod 8), so the pairs of one list, adjacent in `order`, read it
  // through that XCD's L2; the runs advance through `order` together
  const int xcd = (int)(blockIdx.x & 7), t = (int)(blockIdx.x >> 3);
  const int lbk = (t / kXcdRun) * (8 * kXcdRun) + xcd * kXcdRun + t % kXcdRun;
  if (lbk >= npairs) return;   // block-uniform
  const int pair = order[lbk];
  const int pi = pair / nq;
  const int qi = pair - pi * nq;
  uint64_t* outp = pair_out + ((size_t)qi * nprobe + pi) * topk;
  const int l = probes[(int64_t)qi * nprobe + pi];
  if (l < 0) {   // block-uniform
    for (int i = threadIdx.x; i < topk; i += blockDim.x) outp[i] = ~0ull;
    return;
  }
  const float* qr = q + (int64_t)qi * d;
  const int64_t a = offsets[l], b = offsets[l + 1];
  // executed work (WORK, when `work` is given): table entries built, rows
  // given the partial sum over the first kScanPre subspaces, rows summed over
  // all subspaces (a row that passes the partial sum is summed again in
  // full).  A separate instantiation: the counters cost registers and
  // occupancy that the plain search keeps.
  uint32_t w_lut = 0, w_part = 0, w_full = 0;
  auto report = [&](bool entered) {
    if (!WORK || !work) return;
    unsigned long long v[3] = {w_lut, w_part, w_full};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v[i] += __shfl_xor(v[i], off, 64);
      if ((threadIdx.x & 63) == 0 && v[i]) atomicAdd(work + i, v[i]);
    }
    if (threadIdx.x == 0 && entered) atomicAdd(work + 3, 1ull);
  };
  const bool m16 = V16 && m == 16;
  const uint4* c4 = reinterpret_cast<const uint4*>(codes);
  // M = 16: the code rows of the first two steps, in flight while the table
  // is built; each step then loads the rows two steps ahead
  uint4 cv[kScanRows], n1[kScanRows];
  if (m16) {
#pragma unroll
    for (int r = 0; r < kScanRows; ++r) {
      const int64_t p = a + r * kT + threadIdx.x;
      if (p < b) cv[r] = c4[p];
      if (p + kScanBatch < b) n1[r] = c4[p + kScanBatch];
    }
  }
  if (threadIdx.x == 0) {
    cnt = 0;
    need = 0;
    thr = load_relaxed(qthr + qi);
  }
  for (int t = threadIdx.x; t < d; t += blockDim.x) rq[t] = qr[t] - cc[(int64_t)l * d + t];
  __syncthreads();
  // table rows of subspaces [j0, j1)
  auto build_lut = [&](int j0, int j1) {
    for (int j = j0; j < j1; ++j)
      for (int k = threadIdx.x; k < ks; k += blockDim.x) {
        lut[j * ks + k] = sqdist_fixed<DS>(rq + j * DS, pq + ((int64_t)j * ks + k) * DS);
        if (WORK) ++w_lut;
      }
  };
  // M = 16 rows: the table of the first kLutPre subspaces now, the rest once
  // a row needs it (the rows of distant lists mostly never do).
  // A lower bound of every row's running sum over those subspaces: the
  // smallest entry of each table row, summed in the same order (float
  // addition is monotone).  Once the score of the query's bound is below it,
  // no row of the list can be inserted and the list is left.  The bound over
  // the first half of the rows is checked before the second half is built.
  __shared__ float lb_w[kLutPre][kT / 64];
  __shared__ float lb_run;
  __shared__ uint32_t lb_bits;
  auto bound_rows = [&](int j0, int j1) {   // lb_run += the minima of rows [j0, j1), in order
    for (int u = j0; u < j1; ++u) {
      float v = (int)threadIdx.x < ks ? lut[u * ks + threadIdx.x] : INFINITY;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v = fminf(v, __shfl_xor(v, off, 64));
      if ((threadIdx.x & 63) == 0) lb_w[u][threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      float lb = lb_run;
      for (int u = j0; u < j1; ++u) {
        float mu = lb_w[u][0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) mu = fminf(mu, lb_w[u][w]);
        lb = (u == 0) ? mu : lb + mu;
      }
      lb_run = lb;
      lb_bits = __float_as_uint(lb);
    }
    __syncthreads();
  };
  if (m16) {
    constexpr int kHalf = kLutPre / 2;
    build_lut(0, kHalf);
    __syncthreads();
    bound_rows(0, kHalf);
    const uint32_t tb0 = (uint32_t)(thr >> 32);
    if (tb0 != 0xFFFFFFFFu && lb_bits > tb0) {   // block-uniform: the list is left
      for (int i = threadIdx.x; i < topk; i += blockDim.x) outp[i] = ~0ull;
      report(false);
      return;
    }
    build_lut(kHalf, kLutPre);
    __syncthreads();
    bound_rows(kHalf, kLutPre);
  } else {
    build_lut(0, m);
    __syncthreads();
  }
  // each step takes kScanRows rows per thread (rows p0 + r * kT + thread), so
  // that their loads are in flight together; room for a whole step of keys is
  // kept free in the buffer
  auto insert = [&](float s, int32_t id, uint64_t tl) {
    const uint64_t key = ((uint64_t)__float_as_uint(s) << 32) | (uint32_t)id;
    if (key <= tl) {
      const int slot = atomicAdd(&cnt, 1);
      buf[slot] = key;
    }
  };
  // sum of the first U table entries of a 16-code row, subspaces ascending
  auto sum16 = [&](const uint4 v, auto U) {
    const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
    float s = 0.0f;
#pragma unroll
    for (int u = 0; u < decltype(U)::value; ++u) {
      const float e = lut[u * ks + ((w4[u >> 2] >> (8 * (u & 3))) & 0xFFu)];
      s = (u == 0) ? e : s + e;
    }
    return s;
  };
  // end of a step: compaction when the buffer may not hold another step,
  // else the query's bound as other lists of the query may have lowered it
  // (ext: its value loaded by thread 0 at the start of the step)
  auto step_end = [&](uint64_t ext) {
    __syncthreads();
    if (cnt > cap - kScanBatch) {   // block-uniform
      topk_compact(buf, cap, topk, &cnt, &thr, qthr + qi, kScanBatch);
    } else {
      if (threadIdx.x == 0 && ext < thr) thr = ext;
      __syncthreads();
    }
  };
  auto ext_load = [&]() { return threadIdx.x == 0 ? load_relaxed(qthr + qi) : ~0ull; };
  if (m16) {   // one 16-byte code row per row
    const int lane = threadIdx.x & 63;
    uint16_t* wql = wq + (threadIdx.x >> 6) * (64 * kScanRows);
    bool full = false;   // table of all subspaces built (block-uniform)
    int step = 0;
    for (int64_t p0 = a; p0 < b; p0 += kScanBatch, ++step) {
      const uint64_t tl = thr;
      const uint32_t tb = (uint32_t)(tl >> 32);   // score bits of the bound
      if (tb != 0xFFFFFFFFu && lb_bits > tb) break;   // block-uniform: no row can be inserted
      const uint64_t ext = ext_load();
      // the code rows two steps ahead, in flight while this step is scored
      uint4 nx[kScanRows];
#pragma unroll
      for (int r = 0; r < kScanRows; ++r) {
        const int64_t p = p0 + 2 * kScanBatch + r * kT + threadIdx.x;
        if (p < b) nx[r] = c4[p];
      }
      if (tb != 0xFFFFFFFFu) {
        // partial sums over the first kScanPre subspaces; the rows that may
        // still be inserted, compacted per wave, are finished by all lanes
        int nq_w = 0;
#pragma unroll
        for (int r = 0; r < kScanRows; ++r) {
          const int64_t p = p0 + r * kT + threadIdx.x;
          bool keep = false;
          if (p < b) {
            keep = __float_as_uint(sum16(cv[r], std::integral_constant<int, kScanPre>{})) <= tb;
            if (WORK) ++w_part;
          }
          const unsigned long long bal = __ballot(keep);
          if (keep) wql[nq_w + __popcll(bal & __lanemask_lt())] = (uint16_t)(r * kT + threadIdx.x);
          nq_w += __popcll(bal);
        }
        if (!full) {
          if (lane == 0 && nq_w > 0) need = step + 1;
          __syncthreads();
          if (need == step + 1) {
            build_lut(kLutPre, m);
            __syncthreads();
            full = true;
          }
        } else {
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        }
        for (int i = lane; i < nq_w; i += 64) {
          const int64_t p = p0 + wql[i];
          insert(sum16(c4[p], std::integral_constant<int, 16>{}), ids[p], tl);
          if (WORK) ++w_full;
        }
      } else {   // no bound yet: every row is summed in full
        if (!full) {
          build_lut(kLutPre, m);
          __syncthreads();
          full = true;
        }
#pragma unroll
        for (int r = 0; r < kScanRows; ++r) {
          const int64_t p = p0 + r * kT + threadIdx.x;
          if (p < b) {
            insert(sum16(cv[r], std::integral_constant<int, 16>{}), ids[p], tl);
            if (WORK) ++w_full;
          }
        }
      }
      step_end(ext);
#pragma unroll
      for (int r = 0; r < kScanRows; ++r) {
        cv[r] = n1[r];
        n1[r] = nx[r];
      }
    }
  } else {
    for (int64_t p0 = a; p0 < b; p0 += kScanBatch) {
      const uint64_t tl = thr;
      const uint64_t ext = ext_load();
      for (int r = 0; r < kScanRows; ++r) {
        const int64_t p = p0 + r * kT + threadIdx.x;
        if (p >= b) break;
        float s;
        if (V16) {   // m % 16 == 0 and aligned rows: 16 codes per load
          const uint4* cr = reinterpret_cast<const uint4*>(codes + p * m);
          s = 0.0f;
          for (int j0 = 0; j0 < m; j0 += 16) {
            const uint4 v = cr[j0 >> 4];
            const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int u = 0; u < 16; ++u) {
              const int j = j0 + u;
              const float e = lut[j * ks + ((w4[u >> 2] >> (8 * (u & 3))) & 0xFFu)];
              s = (j == 0) ? e : s + e;
            }
          }
        } else {
          const uint8_t* cr = codes + p * m;
          s = lut[cr[0]];
          for (int j = 1; j < m; ++j) s = s + lut[j * ks + cr[j]];
        }
        insert(s, ids[p], tl);
        if (WORK) ++w_full;
      }
      step_end(ext);
    }
  }
  report(true);
  const int c = cnt;
  topk_finish(buf, c);
  const int keep = c < topk ? c : topk;
  for (int i = threadIdx.x; i < topk; i += blockDim.x) outp[i] = i < keep ? buf[i] : ~0ull;
  if (threadIdx.x == 0 && keep == topk) atomicMin(qthr + qi, (unsigned long long)buf[topk - 1]);
}

// One block per query: the best topk of its lists' candidates (keys <= the
// query's final bound), ascending; ids -1 and distance +inf past the end.
__global__ __launch_bounds__(kT) void k_adc_merge(const uint64_t* __restrict__ pair_out, int nprobe, int topk,
                                                  int cap, const unsigned long long* __restrict__ qthr,
                                                  int32_t* __restrict__ out_ids, float* __restrict__ out_dist) {
  extern __shared__ uint64_t mbuf[];
  __shared__ int cnt;
  __shared__ uint64_t thr;
  const int qi = blockIdx.x;
  if (threadIdx.x == 0) {
    cnt = 0;
    thr = qthr[qi];
  }
  __syncthreads();
  const int total = nprobe * topk;
  const uint64_t* src = pair_out + (size_t)qi * total;
  for (int i0 = 0; i0 < total; i0 += kBatch) {
    const int i = i0 + threadIdx.x;
    const uint64_t tl = thr;
    const uint64_t key = i < total ? src[i] : ~0ull;
    if (key != ~0ull && key <= tl) {
      const int slot = atomicAdd(&cnt, 1);
      mbuf[slot] = key;
    }
    __syncthreads();
    topk_compact(mbuf, cap, topk, &cnt, &thr, nullptr, kBatch);
  }
  const int c = cnt;
  topk_finish(mbuf, c);
  for (int i = threadIdx.x; i < topk; i += blockDim.x) {
    const bool real = i < c;
    out_ids[(int64_t)qi * topk + i] = real ? (int32_t)(uint32_t)(mbuf[i] & 0xFFFFFFFFull) : -1;
    out_dist[(int64_t)qi * topk + i] = real ? __uint_as_float((uint32_t)(mbuf[i] >> 32)) : INFINITY;
  }
}

}  // namespace

// key buffer of a scan block / the merge block: room for topk kept keys plus
// one full batch, rounded up to 64 keys
int adc_key_cap(int topk, int batch) { return ((topk + batch + 63) / 64) * 64; }

int adc_scan_smem(int d, int m, int ks, int topk) {
  return (int)((size_t)m * ks * sizeof(float) + (size_t)((d + 1) & ~1) * sizeof(float) +
               (size_t)adc_key_cap(topk, kScanBatch) * sizeof(uint64_t));
}

bool adc_fits_lds(int d, int m, int ks, int topk) {
  // dynamic part + the survivor queues and counters of the scan block
  return (size_t)adc_scan_smem(d, m, ks, topk) + kScanBatch * sizeof(uint16_t) + 64 <= kAdcMaxLds;
}

namespace {
struct OrderWs {
  int32_t *plab, *vals_a, *vals_b, *order;
  uint32_t *keys_a, *keys_b, *keys_sorted, *hist;
  int64_t* poff;
  size_t bytes;
};
OrderWs carve_order(void* ws, int64_t pairs, int nlabels) {
  Carver c(ws);
  OrderWs o;
  o.plab = c.take<int32_t>(pairs);
  o.keys_a = c.take<uint32_t>(pairs);
  o.keys_b = c.take<uint32_t>(pairs);
  o.keys_sorted = c.take<uint32_t>(pairs);
  o.hist = c.take<uint32_t>(sort_hist_entries(pairs));
  o.vals_a = c.take<int32_t>(pairs);
  o.vals_b = c.take<int32_t>(pairs);
  o.order = c.take<int32_t>(pairs);
  o.poff = c.take<int64_t>((size_t)nlabels + 1);
  o.bytes = c.bytes();
  return o;
}
}  // namespace

size_t adc_order_bytes(int64_t pairs, int nprobe, int kc) {
  return carve_order(nullptr, pairs > 0 ? pairs : 1, order_labels(nprobe, kc)).bytes;
}

int launch_adc(const float* q, int nq, int d, const float* cc, int kc, const void* aop, const float* mu,
               const unsigned int* cmax_bits, const float* pq, int m, int ks, const int64_t* offsets,
               const int32_t* ids, const uint8_t* codes, int nprobe, int topk, float* est, int32_t* probes,
               unsigned long long* qthr, uint64_t* pair_out, void* order_ws, int64_t* wide, int32_t* out_ids,
               float* out_dist, int64_t* work_out, hipStream_t s) {
  if (nq == 0) return MIPQ_OK;
  unsigned long long* work = reinterpret_cast<unsigned long long*>(work_out);
  ProfScope ps(MIPQ_K_ADC, s);
  const int S = coarse_ksteps(d);
  const int nt = (kc + 31) / 32;
  const int tgroups = (nt + kTilesPerWave - 1) / kTilesPerWave;
  const int waves = ceil_div(nq, 32) * tgroups;
  const int blocks = ceil_div(waves, kT / 64);
#define AD(SV) k_adc_dist<SV><<<blocks, kT, 0, s>>>(q, nq, d, kc, (const bf16x8*)aop, mu, est)
  switch (S) {
    case 1: AD(1); break;
    case 2: AD(2); break;
    case 4: AD(4); break;
    case 6: AD(6); break;
    case 8: AD(8); break;
    case 12: AD(12); break;
    case 16: AD(16); break;
    default: return fail(MIPQ_EUNSUPPORTED, "ADC needs d <= 16 or d in {32, 64, 96, 128, 192, 256}");
  }
#undef AD
  MIPQ_LAUNCHED("k_adc_dist");
  const float e_cross = 0.0165f;
  const float e_norm = 16.0f * (S + 1) * 1.2e-7f + 2.4e-7f;
  const float g_exact = 1.3e-7f;
  k_adc_probe<<<nq, kT, 0, s>>>(q, d, cc, kc, est, mu, cmax_bits, nprobe, e_cross, e_norm, g_exact, probes,
                                reinterpret_cast<unsigned long long*>(wide));
  MIPQ_LAUNCHED("k_adc_probe");
  k_fill_u64<<<ceil_div(nq, kT), kT, 0, s>>>(qthr, nq, ~0ull);
  MIPQ_LAUNCHED("k_fill_u64");
  // the scan blocks' order (see k_pair_order)
  const int64_t npairs = (int64_t)nq * nprobe;
  const int nlabels = order_labels(nprobe, kc);
  const OrderWs ow = carve_order(order_ws, npairs, nlabels);
  if (kc + 1 <= kOrderMaxBins) {
    k_pair_order<<<nprobe, kOrderT, (size_t)(kc + 1) * sizeof(uint32_t), s>>>(probes, nq, nprobe, kc, ow.order);
    MIPQ_LAUNCHED("k_pair_order");
  } else {
    k_pair_lists<<<(unsigned)((npairs + kT - 1) / kT), kT, 0, s>>>(probes, nq, nprobe, kc, ow.plab);
    MIPQ_LAUNCHED("k_pair_lists");
    const int rc = launch_sort_by_label(ow.plab, npairs, nlabels, ow.keys_a, ow.keys_b, ow.vals_a, ow.vals_b,
                                        ow.hist, ow.order, ow.keys_sorted, ow.poff, s);
    if (rc) return rc;
  }
  const int ds = d / m;
  const int cap = adc_key_cap(topk, kScanBatch);
  const int mcap = adc_key_cap(topk, kBatch);
  const size_t shm = adc_scan_smem(d, m, ks, topk);
  const bool v16 = (m % 16 == 0) && ((reinterpret_cast<uintptr_t>(codes) & 15) == 0);
  const unsigned sblocks = (unsigned)(((npairs + 8 * kXcdRun - 1) / (8 * kXcdRun)) * (8 * kXcdRun));
#define SC1(DSV, V, W)                                                                                  \
  k_adc_scan<DSV, V, W><<<sblocks, kT, shm, s>>>(q, d, cc, pq, m, ks, offsets, ids, codes, probes, nq, nprobe, \
                                                 topk, cap, qthr, pair_out, ow.order, (int)npairs, work)
#define SC(DSV)                               \
  do {                                        \
    if (work) {                               \
      if (v16) SC1(DSV, true, true);          \
      else SC1(DSV, false, true);             \
    } else {                                  \
      if (v16) SC1(DSV, true, false);         \
      else SC1(DSV, false, false);            \
    }                                         \
  } while (0)
  {
    ProfScope pscan(MIPQ_K_ADC_SCAN, s);
    switch (ds) {
      case 1: SC(1); break;
      case 2: SC(2); break;
      case 4: SC(4); break;
      case 8: SC(8); break;
      case 16: SC(16); break;
      default: return fail(MIPQ_EUNSUPPORTED, "ADC supports d/m in {1, 2, 4, 8, 16} (got %d)", ds);
    }
  }
#undef SC
#undef SC1
  MIPQ_LAUNCHED("k_adc_scan");
  k_adc_merge<<<nq, kT, (size_t)mcap * sizeof(uint64_t), s>>>(pair_out, nprobe, topk, mcap, qthr, out_ids,
                                                               out_dist);
  MIPQ_LAUNCHED("k_adc_merge");
  return MIPQ_OK;
}

}  // namespace mipq
