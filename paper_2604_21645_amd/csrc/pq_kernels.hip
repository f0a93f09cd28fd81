// Plain float32 assignment, centroid-update reductions, decode and SSE.
//
// Paper Section 2.1 (fit: per-subspace k-means; encode: nearest subspace
// centroid) and Section 3 (encode + decode to measure the RMSE).
#include <math.h>

#include "dist32.h"
#include "mipq_internal.h"

namespace mipq {

namespace {

constexpr int kThreads = 256;

// Block index -> (row block, subspace group) so that all subspace groups of a
// row block sit on the same XCD (consecutive block ids go to consecutive XCDs)
// and are dispatched next to each other: the rows they share stay in that
// XCD's L2.
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

__global__ void k_zero_u32(uint32_t* p, size_t count) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0u;
}

__global__ void k_gather_rows(const float* __restrict__ x, int64_t n, int d,
                              const int64_t* __restrict__ rows, int64_t n_rows,
                              float* __restrict__ out, uint32_t* bad) {
  const int64_t total = n_rows * d;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / d;
    const int t = int(i - r * d);
    const int64_t src = rows[r];
    if (src < 0 || src >= n) {
      out[i] = NAN;
      if (t == 0) atomicOr(bad, 1u);
    } else {
      out[i] = x[src * d + t];
    }
  }
}

__global__ void k_init_codebook(const float* __restrict__ train, int64_t n_train, int d, int m,
                                int ks, const int64_t* __restrict__ init_rows,
                                const float* __restrict__ init_cb, double* __restrict__ c64,
                                float* __restrict__ c32, uint32_t* bad) {
  const int ds = d / m;
  const int64_t total = (int64_t)m * ks * ds;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    float v;
    if (init_cb) {
      v = init_cb[i];
    } else {
      const int64_t jk = i / ds;            // j * ks + k
      const int t = int(i - jk * ds);
      const int j = int(jk / ks);
      const int64_t r = init_rows[jk];
      if (r < 0 || r >= n_train) {
        v = NAN;
        if (t == 0) atomicOr(bad, 1u);
      } else {
        v = train[r * d + (int64_t)j * ds + t];
      }
    }
    c64[i] = (double)v;
    c32[i] = v;
  }
}

// One lane per row, one wave per subspace: candidate centroids are wave-uniform
// and come through the scalar cache.
template <int DS>
__global__ __launch_bounds__(kThreads) void k_assign_fp32(const float* __restrict__ x, int64_t n,
                                                          int d, int m, int ks, int ds_rt,
                                                          const float* __restrict__ c32,
                                                          uint8_t* __restrict__ codes, int groups) {
  const XcdMap bm = xcd_map(blockIdx.x, groups);
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int sub = bm.group * 4 + w;
  const int64_t row0 = (int64_t)bm.rowblk * 64;
  if (sub >= m || row0 >= n) return;
  const int64_t row = row0 + lane;
  const bool valid = row < n;
  const int ds = DS ? DS : ds_rt;
  constexpr int CAP = DS ? DS : kMaxDsFp32;
  float xv[CAP];
  const float* xr = x + (valid ? row : row0) * d + (int64_t)sub * ds;
#pragma unroll
  for (int t = 0; t < CAP; ++t) xv[t] = (t < ds) ? xr[t] : 0.0f;
  const float* cb = c32 + (int64_t)sub * ks * ds;
  float best = INFINITY;
  int bi = 0;
  for (int k = 0; k < ks; ++k) {
    const float dk = DS ? sqdist_fixed<DS>(xv, cb + (int64_t)k * DS) : sqdist_rt(xv, cb + (int64_t)k * ds, ds);
    if (dk < best) {   // strict: the lowest index wins ties
      best = dk;
      bi = k;
    }
  }
  if (valid) codes[row * m + sub] = (uint8_t)bi;
}

__device__ __forceinline__ double block_sum_f64(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
  return s;   // valid on thread 0
}

// Float64 centroid sums and counts of one subspace over one row chunk, in LDS;
// the chunk partials are summed in a fixed order by k_finalize.  Also the
// objective: the float32 distance of each row to its assigned centroid.
template <int DS>
__global__ __launch_bounds__(kThreads) void k_accumulate(const float* __restrict__ x, int64_t n,
                                                         int d, int m, int ks, int ds_rt,
                                                         const uint8_t* __restrict__ codes,
                                                         const float* __restrict__ c32, int64_t rpc,
                                                         double* __restrict__ part_s,
                                                         uint32_t* __restrict__ part_cnt,
                                                         double* __restrict__ part_j) {
  extern __shared__ double smem[];
  const int ds = DS ? DS : ds_rt;
  constexpr int CAP = DS ? DS : kMaxDsFit;
  double* S = smem;
  uint32_t* cnt = reinterpret_cast<uint32_t*>(S + (size_t)ks * ds);
  double* red = S + (size_t)ks * ds + (ks + 1) / 2;
  const int c = blockIdx.x, sub = blockIdx.y;
  for (int i = threadIdx.x; i < ks * ds; i += blockDim.x) S[i] = 0.0;
  for (int i = threadIdx.x; i < ks; i += blockDim.x) cnt[i] = 0u;
  __syncthreads();
  const int64_t r0 = (int64_t)c * rpc;
  const int64_t r1 = min(n, r0 + rpc);
  const float* cb = c32 + (int64_t)sub * ks * ds;
  double jl = 0.0;
  for (int64_t row = r0 + threadIdx.x; row < r1; row += blockDim.x) {
    const int code = codes[row * m + sub];
    const float* xr = x + row * d + (int64_t)sub * ds;
    float xv[CAP];
#pragma unroll
    for (int t = 0; t < CAP; ++t) xv[t] = (t < ds) ? xr[t] : 0.0f;
    if (code >= ks) {       // corrupt code: poison the objective, touch nothing
      jl += NAN;
      continue;
    }
    const float dd = DS ? sqdist_fixed<DS>(xv, cb + code * DS) : sqdist_rt(xv, cb + code * ds, ds);
    jl += (double)dd;
#pragma unroll
    for (int t = 0; t < CAP; ++t)
      if (t < ds) atomicAdd(&S[code * ds + t], (double)xv[t]);
    atomicAdd(&cnt[code], 1u);
  }
  const double js = block_sum_f64(jl, red);
  __syncthreads();
  const size_t base = ((size_t)c * m + sub);
  for (int i = threadIdx.x; i < ks * ds; i += blockDim.x) part_s[base * ks * ds + i] = S[i];
  for (int i = threadIdx.x; i < ks; i += blockDim.x) part_cnt[base * ks + i] = cnt[i];
  if (threadIdx.x == 0) part_j[base] = js;
}

// Lloyd update of one subspace: centroid = float64 sum / count over all chunks
// (fixed chunk order), an empty centroid keeps its value; float32 copy by
// round-to-nearest.  Also the subspace's objective for this round.
__global__ __launch_bounds__(kThreads) void k_finalize(int m, int ks, int ds, int nch,
                                                       const double* __restrict__ part_s,
                                                       const uint32_t* __restrict__ part_cnt,
                                                       const double* __restrict__ part_j,
                                                       double* __restrict__ c64,
                                                       float* __restrict__ c32,
                                                       double* __restrict__ j_sub) {
  const int sub = blockIdx.x;
  const size_t per = (size_t)ks * ds;
  for (int i = threadIdx.x; i < ks * ds; i += blockDim.x) {
    const int k = i / ds;
    double s = 0.0;
    uint64_t cn = 0;
    for (int c = 0; c < nch; ++c) {
      const size_t base = (size_t)c * m + sub;
      s += part_s[base * per + i];
      cn += part_cnt[base * ks + k];
    }
    const size_t o = (size_t)sub * per + i;
    const double v = cn ? s / (double)cn : c64[o];
    c64[o] = v;
    c32[o] = (float)v;
  }
  if (threadIdx.x == 0) {
    double j = 0.0;
    for (int c = 0; c < nch; ++c) j += part_j[(size_t)c * m + sub];
    j_sub[sub] = j;
  }
}

__global__ void k_objective(const double* __restrict__ j_sub, int iters, int m, double* objective) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= iters) return;
  double s = 0.0;
  for (int j = 0; j < m; ++j) s += j_sub[(size_t)t * m + j];
  objective[t] = s;
}

__global__ void k_copy_f64(const double* __restrict__ src, double* __restrict__ dst, size_t count) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// Decode (concatenate coded centroids) and the float64 squared error, one
// thread per (row, subspace); per-block partial sums, reduced in block order.
__global__ __launch_bounds__(kThreads) void k_decode_sse(const uint8_t* __restrict__ codes,
                                                         int64_t n, int d, int m, int ks, int ds,
                                                         const float* __restrict__ c32,
                                                         const float* __restrict__ x,
                                                         float* __restrict__ x_hat,
                                                         double* __restrict__ partials) {
  __shared__ double red[kThreads / 64];
  double acc = 0.0;
  const int64_t pairs = n * m;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < pairs;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = p / m;
    const int sub = int(p - row * m);
    const int code = codes[p];
    const int64_t off = row * d + (int64_t)sub * ds;
    if (code >= ks) {
      if (x_hat)
        for (int t = 0; t < ds; ++t) x_hat[off + t] = NAN;
      acc += NAN;
      continue;
    }
    const float* c = c32 + ((int64_t)sub * ks + code) * ds;
    for (int t = 0; t < ds; ++t) {
      const float cv = c[t];
      if (x_hat) x_hat[off + t] = cv;
      if (x) {
        const double df = (double)x[off + t] - (double)cv;
        acc += df * df;
      }
    }
  }
  const double s = block_sum_f64(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ void k_sse_final(const double* __restrict__ partials, int nblk, int64_t n, int d,
                            double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < nblk; ++i) s += partials[i];
  out[0] = s;
  const double cnt = (double)n * (double)d;
  out[1] = cnt > 0 ? sqrt(s / cnt) : 0.0;
}

int grid_for(int64_t work, int per_block, int cap) {
  int64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return int(g);
}

}  // namespace

int launch_zero_u32(uint32_t* p, size_t count, hipStream_t s) {
  if (!count) return MIPQ_OK;
  k_zero_u32<<<grid_for((int64_t)count, kThreads, 1 << 30), kThreads, 0, s>>>(p, count);
  MIPQ_LAUNCHED("k_zero_u32");
  return MIPQ_OK;
}

int launch_gather_rows(const float* x, int64_t n, int d, const int64_t* rows, int64_t n_rows,
                       float* out, uint32_t* bad, hipStream_t s) {
  k_gather_rows<<<grid_for(n_rows * d, kThreads, 8192), kThreads, 0, s>>>(x, n, d, rows, n_rows, out, bad);
  MIPQ_LAUNCHED("k_gather_rows");
  return MIPQ_OK;
}

int launch_init_codebook(const float* train, int64_t n_train, int d, int m, int ks,
                         const int64_t* init_rows, const float* init_cb, double* c64, float* c32,
                         uint32_t* bad, hipStream_t s) {
  const int64_t total = (int64_t)d * ks;   // m * ks * ds
  k_init_codebook<<<grid_for(total, kThreads, 4096), kThreads, 0, s>>>(train, n_train, d, m, ks, init_rows,
                                                                       init_cb, c64, c32, bad);
  MIPQ_LAUNCHED("k_init_codebook");
  return MIPQ_OK;
}

#define MIPQ_DS_SWITCH(ds, CALL)  \
  switch (ds) {                   \
    case 1: CALL(1); break;       \
    case 2: CALL(2); break;       \
    case 3: CALL(3); break;       \
    case 4: CALL(4); break;       \
    case 6: CALL(6); break;       \
    case 8: CALL(8); break;       \
    case 12: CALL(12); break;     \
    case 16: CALL(16); break;     \
    case 32: CALL(32); break;     \
    default: CALL(0); break;      \
  }

int launch_assign_fp32(const float* x, int64_t n, int d, int m, int ks, const float* c32,
                       uint8_t* codes, hipStream_t s) {
  const int ds = d / m;
  const int groups = ceil_div(m, 4);
  const int rowblks = ceil_div(n, 64);
  const int blocks = ceil_div(rowblks, 8) * 8 * groups;
#define CALL(DSV) \
  k_assign_fp32<DSV><<<blocks, kThreads, 0, s>>>(x, n, d, m, ks, ds, c32, codes, groups)
  MIPQ_DS_SWITCH(ds, CALL)
#undef CALL
  MIPQ_LAUNCHED("k_assign_fp32");
  return MIPQ_OK;
}

int accumulate_chunks(int64_t n, int m) {
  int nch = ceil_div(n, 2048);
  if (nch < 1) nch = 1;
  const int cap = m >= 16 ? 64 : 128;
  return nch > cap ? cap : nch;
}

int launch_accumulate(const float* x, int64_t n, int d, int m, int ks, const uint8_t* codes,
                      const float* c32, int nch, double* part_s, uint32_t* part_cnt,
                      double* part_j, hipStream_t s) {
  const int ds = d / m;
  const int64_t rpc = (n + nch - 1) / nch;
  const size_t shm = (size_t)ks * ds * sizeof(double) + ((ks + 1) / 2) * sizeof(double) +
                     (kThreads / 64) * sizeof(double);
  dim3 grid(nch, m);
#define CALL(DSV)                                                                              \
  k_accumulate<DSV><<<grid, kThreads, shm, s>>>(x, n, d, m, ks, ds, codes, c32, rpc, part_s, \
                                                part_cnt, part_j)
  MIPQ_DS_SWITCH(ds, CALL)
#undef CALL
  MIPQ_LAUNCHED("k_accumulate");
  return MIPQ_OK;
}

int launch_finalize(int m, int ks, int ds, int nch, const double* part_s, const uint32_t* part_cnt,
                    const double* part_j, double* c64, float* c32, double* j_sub, hipStream_t s) {
  k_finalize<<<m, kThreads, 0, s>>>(m, ks, ds, nch, part_s, part_cnt, part_j, c64, c32, j_sub);
  MIPQ_LAUNCHED("k_finalize");
  return MIPQ_OK;
}

int launch_objective(const double* j_sub, int iters, int m, double* objective, hipStream_t s) {
  if (iters <= 0) return MIPQ_OK;
  k_objective<<<ceil_div(iters, 64), 64, 0, s>>>(j_sub, iters, m, objective);
  MIPQ_LAUNCHED("k_objective");
  return MIPQ_OK;
}

int launch_copy_f64(const double* src, double* dst, size_t count, hipStream_t s) {
  if (!count) return MIPQ_OK;
  k_copy_f64<<<grid_for((int64_t)count, kThreads, 4096), kThreads, 0, s>>>(src, dst, count);
  MIPQ_LAUNCHED("k_copy_f64");
  return MIPQ_OK;
}

int decode_blocks(int64_t n, int m) { return grid_for(n * m, kThreads, 2048); }

int launch_decode_sse(const uint8_t* codes, int64_t n, int d, int m, int ks, const float* c32,
                      const float* x, float* x_hat, double* partials, int nblk, hipStream_t s) {
  k_decode_sse<<<nblk, kThreads, 0, s>>>(codes, n, d, m, ks, d / m, c32, x, x_hat, partials);
  MIPQ_LAUNCHED("k_decode_sse");
  return MIPQ_OK;
}

int launch_sse_final(const double* partials, int nblk, int64_t n, int d, double* out, hipStream_t s) {
  k_sse_final<<<1, 64, 0, s>>>(partials, nblk, n, d, out);
  MIPQ_LAUNCHED("k_sse_final");
  return MIPQ_OK;
}

}  // namespace mipq
