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

// out[r] = x[rows[r]]; block-stride over output rows, threads over the row
// (16-byte accesses when d % 4 == 0).  Out-of-range indices give NaN rows.
__global__ void k_gather_rows(const float* __restrict__ x, int64_t n, int d,
                              const int64_t* __restrict__ rows, int64_t n_rows,
                              float* __restrict__ out, uint32_t* bad, int vec4) {
  const int per = vec4 ? d / 4 : d;
  const int rpb = blockDim.x / per > 0 ? blockDim.x / per : 1;
  const int lr = threadIdx.x / per;
  for (int64_t r0 = (int64_t)blockIdx.x * rpb; r0 < n_rows; r0 += (int64_t)gridDim.x * rpb) {
    const int64_t r = r0 + lr;
    if (lr >= rpb || r >= n_rows) continue;
    const int64_t src = rows[r];
    const bool ok = src >= 0 && src < n;
    for (int e = threadIdx.x - lr * per; e < per; e += (per > (int)blockDim.x ? blockDim.x : per)) {
      if (vec4) {
        reinterpret_cast<float4*>(out + r * d)[e] =
            ok ? reinterpret_cast<const float4*>(x + src * d)[e] : make_float4(NAN, NAN, NAN, NAN);
      } else {
        out[r * d + e] = ok ? x[src * d + e] : NAN;
      }
      if (!ok && e == 0) atomicOr(bad, 1u);
    }
  }
}

__global__ void k_init_codebook(const float* __restrict__ train, int64_t n_train, int d, int m,
                                int ks, const int64_t* __restrict__ init_rows,
                                const float* __restrict__ init_cb, double* __restrict__ c64,
                                float* __restrict__ c32, uint32_t* bad, uint32_t* done) {
  const int ds = d / m;
  const int64_t total = (int64_t)m * ks * ds;
  if (done && blockIdx.x == 0)
    for (int j = threadIdx.x; j < m; j += blockDim.x) done[j] = 0u;
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

// Decode (concatenate coded centroids) and the float64 squared error.  VEC:
// one thread per 4 consecutive elements of a row (ds % 4 == 0, so the four lie
// in one subspace): 16-byte loads and stores.  Otherwise one thread per
// element.  Block blk of nblk takes items blk*256 + tid, stepping by
// nblk*256; per-block partial sums are reduced in a fixed order.
template <int VEC>
__device__ __forceinline__ double decode_sse_part(const uint8_t* __restrict__ codes, int64_t n, int d, int m,
                                                  int ks, int ds, const float* __restrict__ c32,
                                                  const float* __restrict__ x, float* __restrict__ x_hat,
                                                  int64_t blk, int64_t nblk) {
  double acc = 0.0;
  const int per_row = d / VEC;
  const int64_t items = n * per_row;
  const int64_t stride = nblk * blockDim.x;
  // item p: VEC consecutive elements of one row, all in one subspace
  // item (row, col4) advanced incrementally: no division in the loop
  auto one = [&](int64_t row, int c4, float (&cv)[VEC], float (&xv)[VEC], int64_t& off) {
    const int col = c4 * VEC;
    const int sub = col / ds;
    const int t = col - sub * ds;
    const int code = codes[row * m + sub];
    off = row * d + col;
    const bool ok = code < ks;
    const float* c = c32 + ((int64_t)sub * ks + (ok ? code : 0)) * ds + t;
    if (VEC == 4) {
      const float4 q = *reinterpret_cast<const float4*>(c);
      cv[0] = q.x; cv[VEC > 1 ? 1 : 0] = q.y; cv[VEC > 2 ? 2 : 0] = q.z; cv[VEC > 3 ? 3 : 0] = q.w;
    } else {
      cv[0] = c[0];
    }
    if (!ok)
#pragma unroll
      for (int i = 0; i < VEC; ++i) cv[i] = NAN;
    if (x) {
      if (VEC == 4) {
        const float4 q = *reinterpret_cast<const float4*>(x + off);
        xv[0] = q.x; xv[VEC > 1 ? 1 : 0] = q.y; xv[VEC > 2 ? 2 : 0] = q.z; xv[VEC > 3 ? 3 : 0] = q.w;
      } else {
        xv[0] = x[off];
      }
    }
  };
  auto finish = [&](const float (&cv)[VEC], const float (&xv)[VEC], int64_t off) {
    if (x_hat) {
      if (VEC == 4) *reinterpret_cast<float4*>(x_hat + off) = make_float4(cv[0], cv[VEC > 1 ? 1 : 0], cv[VEC > 2 ? 2 : 0], cv[VEC > 3 ? 3 : 0]);
      else x_hat[off] = cv[0];
    }
    if (x) {
#pragma unroll
      for (int i = 0; i < VEC; ++i) {
        const double df = (double)xv[i] - (double)cv[i];
        acc += df * df;
      }
    }
  };
  const int64_t p0 = blk * blockDim.x + threadIdx.x;
  int64_t row = p0 / per_row;
  int c4 = int(p0 - row * per_row);
  const int64_t srow = stride / per_row;
  const int scol = int(stride - srow * per_row);
  auto advance = [&](int64_t& r, int& c) {
    r += srow;
    c += scol;
    if (c >= per_row) {
      c -= per_row;
      ++r;
    }
  };
  // two items in flight per iteration; the sum order per thread is item order
  while (row < n) {
    int64_t row1 = row;
    int c41 = c4;
    advance(row1, c41);
    float c0[VEC], x0[VEC], c1[VEC], x1[VEC];
    int64_t o0, o1;
    one(row, c4, c0, x0, o0);
    if (row1 < n) {
      one(row1, c41, c1, x1, o1);
      finish(c0, x0, o0);
      finish(c1, x1, o1);
      advance(row1, c41);
    } else {
      finish(c0, x0, o0);
    }
    row = row1;
    c4 = c41;
  }
  (void)items;
  return acc;
}

template <int VEC>
__global__ __launch_bounds__(kThreads) void k_decode_sse(const uint8_t* __restrict__ codes,
                                                         int64_t n, int d, int m, int ks, int ds,
                                                         const float* __restrict__ c32,
                                                         const float* __restrict__ x,
                                                         float* __restrict__ x_hat,
                                                         double* __restrict__ partials) {
  __shared__ double red[kThreads / 64];
  const double acc = decode_sse_part<VEC>(codes, n, d, m, ks, ds, c32, x, x_hat, blockIdx.x, gridDim.x);
  const double s = block_sum_f64(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}


// Distance of every (row, subspace) to its coded centroid: the float32 rule
// (min_dist, optional) and the float64 squared error of the decode (sum of
// ((double)x - (double)c)^2 over the subspace's dimensions, ascending), one
// thread per (row, subspace) pair in pair order; per-block partial sums are
// reduced in a fixed order by k_sse_final.  Codes >= ks give NaN.
template <int DS>
__global__ __launch_bounds__(kThreads) void k_code_dist(const float* __restrict__ x, int64_t n, int d, int m,
                                                        int ks, int ds_rt, const float* __restrict__ c32,
                                                        const uint8_t* __restrict__ codes,
                                                        float* __restrict__ min_dist,
                                                        double* __restrict__ partials) {
  __shared__ double red[kThreads / 64];
  const int ds = DS ? DS : ds_rt;
  const int64_t items = n * m;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t row = i / m;
  int sub = int(i - row * m);
  const int64_t srow = stride / m;
  const int ssub = int(stride - srow * m);
  double acc = 0.0;
  for (; i < items; i += stride) {
    const int code = codes[i];
    const bool ok = code < ks;
    const float* c = c32 + ((int64_t)sub * ks + (ok ? code : 0)) * ds;
    const float* xr = x + row * d + (int64_t)sub * ds;
    float dist = 0.0f;
    double sq = 0.0;
    for (int t = 0; t < ds; ++t) {
      const float xv = xr[t], cv = c[t];
      const float df = xv - cv;
      const float s2 = df * df;
      dist = dist + s2;
      const double dd = (double)xv - (double)cv;
      sq = sq + dd * dd;
    }
    if (!ok) {
      dist = NAN;
      sq = NAN;
    }
    if (min_dist) min_dist[i] = dist;
    acc += sq;
    row += srow;
    sub += ssub;
    if (sub >= m) {
      sub -= m;
      ++row;
    }
  }
  const double s = block_sum_f64(acc, red);
  if (threadIdx.x == 0 && partials) partials[blockIdx.x] = s;
}

// flag[0] = 1 when any of the count floats at p is NaN or infinite
__global__ __launch_bounds__(kThreads) void k_nonfinite(const float* __restrict__ p, size_t count,
                                                        uint32_t* __restrict__ flag) {
  bool bad = false;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
    bad |= !isfinite(p[i]);
  if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1u);
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

// Many problems: block i is decode block i - dblk0 of problem p, with the
// single-problem partition of that problem's rows (same partial sums).
template <int VEC>
__global__ __launch_bounds__(kThreads) void k_decode_sse_batched(const BatchProb* __restrict__ probs, int nprob,
                                                                 int d, int m, int ks, int ds,
                                                                 double* __restrict__ partials) {
  __shared__ double red[kThreads / 64];
  const int64_t i = blockIdx.x;
  const int p = find_problem(probs, nprob, i, [](const BatchProb& b) { return b.dblk0; });
  const double acc = decode_sse_part<VEC>(probs[p].codes, probs[p].n, d, m, ks, ds, probs[p].c32, probs[p].x,
                                          nullptr, i - probs[p].dblk0, probs[p].nblk);
  const double s = block_sum_f64(acc, red);
  if (threadIdx.x == 0) partials[i] = s;
}

// Sum of the block partials: thread i adds partials i, i+256, ... in order,
// then a fixed pairwise tree over the threads; out = {SSE, RMSE}.
__device__ __forceinline__ void sse_final_body(const double* __restrict__ partials, int nblk, int64_t n, int d,
                                               double* out, double* red) {
  // thread t adds partials t, t + blockDim, ... in that order, with eight
  // loads in flight (one at a time would chain their latencies)
  double s = 0.0;
  constexpr int V = 8;
  const int step = blockDim.x;
  int i = threadIdx.x;
  for (; i + (V - 1) * step < nblk; i += V * step) {
    double v[V];
#pragma unroll
    for (int u = 0; u < V; ++u) v[u] = partials[i + u * step];
#pragma unroll
    for (int u = 0; u < V; ++u) s += v[u];
  }
  for (; i < nblk; i += step) s += partials[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0 && out) {
    const double tot = red[0];
    out[0] = tot;
    const double cnt = (double)n * (double)d;
    out[1] = cnt > 0 ? sqrt(tot / cnt) : 0.0;
  }
}

__global__ __launch_bounds__(kThreads) void k_sse_final(const double* __restrict__ partials, int nblk,
                                                        int64_t n, int d, double* out) {
  __shared__ double red[kThreads];
  sse_final_body(partials, nblk, n, d, out, red);
}

// block p: problem p's SSE and RMSE
__global__ __launch_bounds__(kThreads) void k_sse_final_batched(const BatchProb* __restrict__ probs, int d,
                                                                const double* __restrict__ partials) {
  __shared__ double red[kThreads];
  const BatchProb& P = probs[blockIdx.x];
  sse_final_body(partials + P.dblk0, P.nblk, P.n, d, P.sse_rmse, red);
}

// Many problems: the starting codebook of problem p from its own rows
// (c64 of problem p at c64_all + p * m*ks*ds).
__global__ void k_init_batched(const BatchProb* __restrict__ probs, int nprob, int d, int m, int ks,
                               double* __restrict__ c64_all, uint32_t* bad) {
  const int ds = d / m;
  const int64_t per = (int64_t)m * ks * ds;
  const int64_t total = per * nprob;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int p = (int)(i / per);
    const int64_t e = i - p * per;
    const int64_t jk = e / ds;   // j * ks + k
    const int t = int(e - jk * ds);
    const int j = int(jk / ks);
    const int64_t r = probs[p].init_rows[jk];
    float v;
    if (r < 0 || r >= probs[p].n) {
      v = NAN;
      if (t == 0) atomicOr(bad, 1u);
    } else {
      v = probs[p].x[r * d + (int64_t)j * ds + t];
    }
    c64_all[i] = (double)v;
    probs[p].c32[e] = v;
  }
}

// Many problems: objective[r] of problem p = sum over subspaces j ascending of
// j_all[(r * nprob + p) * m + j].
__global__ void k_objective_batched(const BatchProb* __restrict__ probs, int nprob, int iters, int m,
                                    const double* __restrict__ j_all) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nprob * iters) return;
  const int p = t / iters, r = t - (t / iters) * iters;
  double* out = probs[p].objective;
  if (!out) return;
  double s = 0.0;
  for (int j = 0; j < m; ++j) s += j_all[((size_t)r * nprob + p) * m + j];
  out[r] = s;
}

// Decoded centroids of many codebooks: out[(b*ks + k)*d + j*ds + t] =
// cb[((b*m + j)*ks + k)*ds + t], i.e. row k of book b is the decode of the code
// row (k, k, ..., k).
__global__ void k_decode_centroids(const float* __restrict__ cb, int64_t nbooks, int m, int ks, int ds,
                                   float* __restrict__ out) {
  const int d = m * ds;
  const int64_t total = nbooks * ks * d;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t bk = i / d;   // b * ks + k
    const int col = int(i - bk * d);
    const int j = col / ds, t = col - j * ds;
    const int64_t b = bk / ks;
    const int k = int(bk - b * ks);
    out[i] = cb[((b * m + j) * ks + k) * ds + t];
  }
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
  const int vec4 = (d % 4 == 0) && (((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(out)) & 15) == 0);
  const int per = vec4 ? d / 4 : d;
  const int rpb = kThreads / per > 0 ? kThreads / per : 1;   // rows per block step
  k_gather_rows<<<grid_for(n_rows, rpb, 8192), kThreads, 0, s>>>(x, n, d, rows, n_rows, out, bad, vec4);
  MIPQ_LAUNCHED("k_gather_rows");
  return MIPQ_OK;
}

int launch_init_codebook(const float* train, int64_t n_train, int d, int m, int ks,
                         const int64_t* init_rows, const float* init_cb, double* c64, float* c32,
                         uint32_t* bad, uint32_t* done, hipStream_t s) {
  const int64_t total = (int64_t)d * ks;   // m * ks * ds
  k_init_codebook<<<grid_for(total, kThreads, 4096), kThreads, 0, s>>>(train, n_train, d, m, ks, init_rows,
                                                                       init_cb, c64, c32, bad, done);
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
  ProfScope ps(MIPQ_K_ASSIGN_FP32, s);
#define CALL(DSV) \
  k_assign_fp32<DSV><<<blocks, kThreads, 0, s>>>(x, n, d, m, ks, ds, c32, codes, groups)
  MIPQ_DS_SWITCH(ds, CALL)
#undef CALL
  MIPQ_LAUNCHED("k_assign_fp32");
  return MIPQ_OK;
}

int launch_code_dist(const float* x, int64_t n, int d, int m, int ks, const float* c32, const uint8_t* codes,
                     float* min_dist, double* partials, int nblk, hipStream_t s) {
  if (n == 0) return MIPQ_OK;
  const int ds = d / m;
#define CALL(DSV) \
  k_code_dist<DSV><<<nblk, kThreads, 0, s>>>(x, n, d, m, ks, ds, c32, codes, min_dist, partials)
  MIPQ_DS_SWITCH(ds, CALL)
#undef CALL
  MIPQ_LAUNCHED("k_code_dist");
  return MIPQ_OK;
}

int launch_nonfinite(const float* p, size_t count, uint32_t* flag, hipStream_t s) {
  if (!count) return MIPQ_OK;
  k_nonfinite<<<grid_for((int64_t)count, kThreads, 4096), kThreads, 0, s>>>(p, count, flag);
  MIPQ_LAUNCHED("k_nonfinite");
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
  ProfScope ps(MIPQ_K_DECODE, s);
  const int ds = d / m;
  const bool vec = (ds % 4 == 0) && ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(x_hat) |
                                      reinterpret_cast<uintptr_t>(c32)) & 15) == 0;
  if (vec)
    k_decode_sse<4><<<nblk, kThreads, 0, s>>>(codes, n, d, m, ks, ds, c32, x, x_hat, partials);
  else
    k_decode_sse<1><<<nblk, kThreads, 0, s>>>(codes, n, d, m, ks, ds, c32, x, x_hat, partials);
  MIPQ_LAUNCHED("k_decode_sse");
  return MIPQ_OK;
}

int launch_sse_final(const double* partials, int nblk, int64_t n, int d, double* out, hipStream_t s) {
  k_sse_final<<<1, kThreads, 0, s>>>(partials, nblk, n, d, out);
  MIPQ_LAUNCHED("k_sse_final");
  return MIPQ_OK;
}

int launch_init_batched(const BatchProb* probs, int nprob, int d, int m, int ks, double* c64_all, uint32_t* bad,
                        hipStream_t s) {
  const int64_t total = (int64_t)nprob * d * ks;
  k_init_batched<<<grid_for(total, kThreads, 8192), kThreads, 0, s>>>(probs, nprob, d, m, ks, c64_all, bad);
  MIPQ_LAUNCHED("k_init_batched");
  return MIPQ_OK;
}

int launch_decode_sse_batched(const BatchProb* probs, int nprob, int64_t blocks, int d, int m, int ks, bool vec,
                              double* partials, hipStream_t s) {
  const int ds = d / m;
  {
    ProfScope ps(MIPQ_K_DECODE, s);
    if (vec)
      k_decode_sse_batched<4><<<(unsigned)blocks, kThreads, 0, s>>>(probs, nprob, d, m, ks, ds, partials);
    else
      k_decode_sse_batched<1><<<(unsigned)blocks, kThreads, 0, s>>>(probs, nprob, d, m, ks, ds, partials);
    MIPQ_LAUNCHED("k_decode_sse_batched");
  }
  k_sse_final_batched<<<nprob, kThreads, 0, s>>>(probs, d, partials);
  MIPQ_LAUNCHED("k_sse_final_batched");
  return MIPQ_OK;
}

int launch_objective_batched(const BatchProb* probs, int nprob, int iters, int m, const double* j_all,
                             hipStream_t s) {
  if (iters <= 0) return MIPQ_OK;
  k_objective_batched<<<ceil_div((int64_t)nprob * iters, 64), 64, 0, s>>>(probs, nprob, iters, m, j_all);
  MIPQ_LAUNCHED("k_objective_batched");
  return MIPQ_OK;
}

int launch_decode_centroids(const float* cb, int64_t nbooks, int m, int ks, int ds, float* out, hipStream_t s) {
  const int64_t total = nbooks * ks * (int64_t)m * ds;
  if (total == 0) return MIPQ_OK;
  k_decode_centroids<<<grid_for(total, kThreads, 8192), kThreads, 0, s>>>(cb, nbooks, m, ks, ds, out);
  MIPQ_LAUNCHED("k_decode_centroids");
  return MIPQ_OK;
}

}  // namespace mipq
