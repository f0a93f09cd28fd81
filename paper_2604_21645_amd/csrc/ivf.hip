// Inverted file (paper Section 2.2: row ids stored per bucket for fast lookup;
// buckets here are coarse k-means lists, see the inverted-index reading).
//
//  * coarse assignment: coarse.hip;
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

// ---------------------------------------------------------------- radix sort
// Stable LSD radix sort of (key, value) by key, 6-bit digits.  Tile = `tile`
// consecutive elements per block (a multiple of kT, chosen so that the sort
// runs on up to kRsMaxBlocks blocks); a round = 64 elements per wave, waves
// in element order.
constexpr int kRsBits = 6;
constexpr int kRsBuckets = 1 << kRsBits;
constexpr int kRsMaxBlocks = 1024;
static_assert(kRsBuckets == 64, "one bucket per lane of a wave");

__global__ __launch_bounds__(kT) void k_rs_hist(const uint32_t* __restrict__ keys, int64_t n, int shift,
                                                uint32_t* __restrict__ hist, int nblk, int64_t tile) {
  __shared__ uint32_t cnt[kRsBuckets];
  if (threadIdx.x < kRsBuckets) cnt[threadIdx.x] = 0u;
  __syncthreads();
  const int64_t b0 = (int64_t)blockIdx.x * tile;
  const int64_t b1 = min(n, b0 + tile);
  for (int64_t i = b0 + threadIdx.x; i < b1; i += blockDim.x)
    atomicAdd(&cnt[(keys[i] >> shift) & (kRsBuckets - 1)], 1u);
  __syncthreads();
  if (threadIdx.x < kRsBuckets) hist[(size_t)threadIdx.x * nblk + blockIdx.x] = cnt[threadIdx.x];
}

// exclusive scan of each bucket's row of hist (bucket-major: row b holds the
// nblk <= kRsMaxBlocks block counts of digit b) in place, one block per
// bucket, one entry per thread; the row totals go to tot[b] (the scatter adds
// their exclusive prefix)
constexpr int kScanT = kRsMaxBlocks;
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, int lane) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t u = __shfl_up(v, off, 64);
    if (lane >= off) v += u;
  }
  return v;
}
__global__ __launch_bounds__(kScanT) void k_rs_scan(uint32_t* __restrict__ hist, int nblk, uint32_t* __restrict__ tot) {
  __shared__ uint32_t wsum[kScanT / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t* row = hist + (size_t)blockIdx.x * nblk;
  const bool in = (int)threadIdx.x < nblk;
  const uint32_t v = in ? row[threadIdx.x] : 0u;
  const uint32_t incl = wave_incl_scan(v, lane);
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  if (w == 0) {
    const uint32_t ws = lane < kScanT / 64 ? wsum[lane] : 0u;
    const uint32_t wi = wave_incl_scan(ws, lane);
    if (lane < kScanT / 64) wsum[lane] = wi - ws;   // exclusive prefix of the waves
    if (lane == kScanT / 64 - 1) tot[blockIdx.x] = wi;
  }
  __syncthreads();
  if (in) row[threadIdx.x] = wsum[w] + incl - v;
}

// scatter in element order; vals_in == NULL means value = element index.  A
// lane's rank among the wave's lanes with the same digit comes from one ballot
// per digit bit (the lanes that agree with it on every bit).
__global__ __launch_bounds__(kT) void k_rs_scatter(const uint32_t* __restrict__ keys_in,
                                                   const int32_t* __restrict__ vals_in, int64_t n, int shift,
                                                   const uint32_t* __restrict__ offs, int nblk, int64_t tile,
                                                   const uint32_t* __restrict__ tot,
                                                   uint32_t* __restrict__ keys_out, int32_t* __restrict__ vals_out) {
  __shared__ uint32_t base[kRsBuckets];
  __shared__ uint32_t wcnt[kT / 64][kRsBuckets];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  if (threadIdx.x < kRsBuckets) {   // wave 0: the digit's start = earlier digits' totals + earlier blocks' counts
    const uint32_t t = tot[threadIdx.x];
    base[threadIdx.x] = wave_incl_scan(t, lane) - t + offs[(size_t)threadIdx.x * nblk + blockIdx.x];
  }
  const int64_t b0 = (int64_t)blockIdx.x * tile;
  const int64_t b1 = min(n, b0 + tile);
  const uint64_t below = (1ull << lane) - 1ull;
  for (int64_t r0 = b0; r0 < b1; r0 += (int64_t)nw * 64) {
    const int64_t i = r0 + (int64_t)w * 64 + lane;
    const bool ok = i < b1;
    const uint32_t key = ok ? keys_in[i] : 0u;
    const int32_t val = ok ? (vals_in ? vals_in[i] : (int32_t)i) : 0;
    const int dig = ok ? (int)((key >> shift) & (kRsBuckets - 1)) : 0;
    uint64_t peers = __ballot(ok);   // valid lanes with this lane's digit
#pragma unroll
    for (int b = 0; b < kRsBits; ++b) {
      const bool bit = (dig >> b) & 1;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const int rank = __popcll(peers & below);
    wcnt[w][lane] = 0u;   // lane b clears bucket b (kRsBuckets == 64), then the first lane of each digit counts it
    if (ok && rank == 0) wcnt[w][dig] = (uint32_t)__popcll(peers);
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
// value); also the list's objective sum of (x - c_old)^2 in float64.  The
// rows are loaded kU at a time (their loads in flight together) and then
// added in id order, so the sums are those of the plain loop.
__global__ __launch_bounds__(kT) void k_coarse_update(const float* __restrict__ x, int d,
                                                      const int32_t* __restrict__ ids,
                                                      const int64_t* __restrict__ offsets,
                                                      float* __restrict__ cc, double* __restrict__ cc64,
                                                      double* __restrict__ obj_list) {
  __shared__ double red[kT / 64];
  const int l = blockIdx.x;
  const int64_t a = offsets[l], b = offsets[l + 1];
  double jl = 0.0;
  constexpr int kU = 32;
  const int lane = threadIdx.x & 63;
  // every lane runs every pass (the ids are read back from lanes 0 .. kU - 1,
  // which must all have loaded them); lanes past d load dimension d - 1 and
  // keep nothing
  for (int t0 = 0; t0 < d; t0 += blockDim.x) {
    const int t = t0 + (int)threadIdx.x;
    const bool act = t < d;
    const int tc = act ? t : d - 1;
    const float cold = cc[(int64_t)l * d + tc];
    double s = 0.0;
    for (int64_t p0 = a; p0 < b; p0 += kU) {
      const int cnt = b - p0 < kU ? (int)(b - p0) : kU;
      // lane u holds the id of row p0 + u (one vector load), read back per row
      const int myid = ids[p0 + (lane < cnt ? lane : cnt - 1)];
      float xv[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int r = __builtin_amdgcn_readlane(myid, u < cnt ? u : cnt - 1);
        xv[u] = x[(int64_t)r * d + tc];   // all kU loads in flight
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        if (act && u < cnt) {
          s += (double)xv[u];
          const double df = (double)xv[u] - (double)cold;
          jl += df * df;
        }
      }
    }
    if (act && b > a) {
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
// elements per block of the sort: a multiple of kT, at most kRsMaxBlocks blocks
int64_t sort_tile(int64_t n) {
  int64_t t = (n + kRsMaxBlocks - 1) / kRsMaxBlocks;
  t = (t + kT - 1) / kT * kT;
  return t < kT ? kT : t;
}
int sort_blocks(int64_t n) { return n > 0 ? ceil_div(n, sort_tile(n)) : 1; }
// (enough for every sort of up to n elements: sort_blocks(m) <= min(ceil(m / kT), kRsMaxBlocks), which
// grows with m although sort_blocks itself does not)
size_t sort_hist_entries(int64_t n) {
  const int64_t b = (n + kT - 1) / kT;
  return (size_t)kRsBuckets * (size_t)(b < 1 ? 1 : (b > kRsMaxBlocks ? kRsMaxBlocks : b)) + kRsBuckets;
}

int launch_sort_by_label(const int32_t* labels, int64_t n, int kc, uint32_t* keys_a, uint32_t* keys_b,
                         int32_t* vals_a, int32_t* vals_b, uint32_t* hist, int32_t* ids_out,
                         uint32_t* keys_out_sorted, int64_t* offsets, hipStream_t s) {
  ProfScope ps(MIPQ_K_SORT, s);
  const int nblk = sort_blocks(n);
  const int64_t tile = sort_tile(n);
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
      k_rs_hist<<<nblk, kT, 0, s>>>(kin, n, p * kRsBits, hist, nblk, tile);
      MIPQ_LAUNCHED("k_rs_hist");
      k_rs_scan<<<kRsBuckets, kScanT, 0, s>>>(hist, nblk, hist + (size_t)kRsBuckets * nblk);
      MIPQ_LAUNCHED("k_rs_scan");
      k_rs_scatter<<<nblk, kT, 0, s>>>(kin, vin, n, p * kRsBits, hist, nblk, tile, hist + (size_t)kRsBuckets * nblk,
                                       kout, vout);
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
