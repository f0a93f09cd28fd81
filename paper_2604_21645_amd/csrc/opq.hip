// Optimized PQ (paper Section 3.1.1 names it beside PQ): rows are quantised
// after an orthogonal rotation y = x R, and R is re-fitted by the orthogonal
// Procrustes problem min ||X R - Y_hat||_F over orthogonal R, solved by
// R = U V^T from the singular value decomposition U S V^T = X^T Y_hat.
//
// Kernels:
//   k_rotate        y = x R, float64 products and sums in ascending t, unfused
//                   (the product of a float32 and a float64 is not exact), one
//                   rounding to float32 per output;
//   k_cross_partial X^T Y_hat over a chunk of rows per block, float64 (float32
//                   products are exact in float64), partials summed in chunk
//                   order by k_cross_reduce;
//   k_polar         one work-group: one-sided (Hestenes) Jacobi on the columns
//                   of M = X^T Y_hat, A = M V with orthogonal columns, U = A's
//                   normalised columns (rank-deficient columns completed to an
//                   orthonormal basis), R = U V^T.
#include <math.h>

#include "mipq_internal.h"

namespace mipq {

namespace {

constexpr int kTile = 64;      // output tile edge (rows x columns)
constexpr int kTk = 32;        // reduction depth staged per step
constexpr int kThreads = 256;  // 16 x 16 threads, 4 x 4 outputs each
typedef double XsT;            // x staged in LDS as float64: converted once per block, not per use
constexpr int kRotR = 4;       // rows per thread of the rotation (16 x kRotR rows per block; 8 measured slower)
constexpr int kRotRows = 16 * kRotR;

// Block (row tile, column tile) of y = x R.  XCD-aware: consecutive column
// tiles of one row tile go to one XCD (blocks b, b + 8, ...) so that the row
// tile is read from HBM once and then from that XCD's L2.
__global__ __launch_bounds__(kThreads) void k_rotate(const float* __restrict__ x, int64_t n, int d,
                                                     const double* __restrict__ r, float* __restrict__ y,
                                                     int ctiles, int64_t nblocks) {
  __shared__ __align__(16) XsT xs[kTk][kRotRows + 4];   // x tile, transposed: xs[t][row]
  __shared__ __align__(16) double rs[kTk][kTile + 2];  // R tile: rs[t][col]
  // logical block -> (row tile, column tile)
  const int64_t b = blockIdx.x;
  const int64_t xcd = b & 7, slot = b >> 3;
  const int64_t per_xcd = (nblocks + 7) >> 3;
  const int64_t lb = xcd * per_xcd + slot;     // logical block, contiguous per XCD
  if (lb >= nblocks) return;
  const int64_t rt = lb / ctiles;
  const int ct = (int)(lb - rt * ctiles);
  const int64_t row0 = rt * kRotRows;
  const int col0 = ct * kTile;
  const int tid = threadIdx.x;
  const int tc = tid & 15, tr = tid >> 4;
  double acc[kRotR][4];
#pragma unroll
  for (int i = 0; i < kRotR; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;

  // staging of x[row0 .. +kRotRows][t0 .. +32] (transposed) and R[t0 .. +32]
  // [col0 .. +64]: the next step's elements are loaded into registers while
  // the current step is computed
  constexpr int PX = kRotRows * kTk / kThreads;   // x elements per thread
  constexpr int PR = kTile * kTk / kThreads;      // R elements per thread
  float px[PX];
  double pr[PR];
  auto fetch = [&](int t0) {
#pragma unroll
    for (int k = 0; k < PX; ++k) {
      const int e = tid + k * kThreads;
      const int rr = e / kTk, tt = e - rr * kTk;
      const int64_t row = row0 + rr;
      const int t = t0 + tt;
      px[k] = (row < n && t < d) ? x[row * d + t] : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < PR; ++k) {
      const int e = tid + k * kThreads;
      const int t2 = t0 + e / kTile, col = col0 + (e - (e / kTile) * kTile);
      pr[k] = (t2 < d && col < d) ? r[(int64_t)t2 * d + col] : 0.0;
    }
  };
  auto put = [&]() {
#pragma unroll
    for (int k = 0; k < PX; ++k) {
      const int e = tid + k * kThreads;
      const int rr = e / kTk;
      xs[e - rr * kTk][rr] = (XsT)px[k];
    }
#pragma unroll
    for (int k = 0; k < PR; ++k) {
      const int e = tid + k * kThreads;
      rs[e / kTile][e - (e / kTile) * kTile] = pr[k];
    }
  };
  fetch(0);
  put();
  __syncthreads();
  for (int t0 = 0; t0 < d; t0 += kTk) {
    const bool more = t0 + kTk < d;
    if (more) fetch(t0 + kTk);
    const int tend = min(kTk, d - t0);
    for (int tt = 0; tt < tend; ++tt) {
      double xa[kRotR], ra[4];
#pragma unroll
      for (int i = 0; i < kRotR; ++i) xa[i] = (double)xs[tt][tr * kRotR + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) ra[j] = rs[tt][tc * 4 + j];
#pragma unroll
      for (int i = 0; i < kRotR; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = acc[i][j] + xa[i] * ra[j];   // unfused: rounded product, rounded sum
    }
    __syncthreads();
    if (more) {
      put();
      __syncthreads();
    }
  }
#pragma unroll
  for (int i = 0; i < kRotR; ++i) {
    const int64_t row = row0 + tr * kRotR + i;
    if (row >= n) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = col0 + tc * 4 + j;
      if (col < d) y[row * d + col] = (float)acc[i][j];
    }
  }
}

// Block (chunk c, tile (ti, tj)): part[c][t][j] = sum over the chunk's rows n
// of x[n][t] * yh[n][j] for t in tile ti, j in tile tj.
__global__ __launch_bounds__(kThreads) void k_cross_partial(const float* __restrict__ x,
                                                            const float* __restrict__ yh, int64_t n, int d,
                                                            int64_t rpc, int tiles, double* __restrict__ part) {
  __shared__ __align__(16) float xs[kTk][kTile + 4];   // xs[row][t]
  __shared__ __align__(16) float ys[kTk][kTile + 4];   // ys[row][j]
  const int tile = blockIdx.x % (tiles * tiles);
  const int64_t c = blockIdx.x / (tiles * tiles);
  const int ti = tile / tiles, tj = tile - ti * tiles;
  const int tbase = ti * kTile, jbase = tj * kTile;
  const int64_t r0 = c * rpc;
  const int64_t r1 = min(n, r0 + rpc);
  const int tid = threadIdx.x;
  const int tc = tid & 15, tr = tid >> 4;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  for (int64_t s0 = r0; s0 < r1; s0 += kTk) {
    for (int e = tid; e < kTk * kTile; e += kThreads) {
      const int rr = e / kTile, cc = e - rr * kTile;
      const int64_t row = s0 + rr;
      const bool okr = row < r1;
      xs[rr][cc] = (okr && tbase + cc < d) ? x[row * d + tbase + cc] : 0.0f;
      ys[rr][cc] = (okr && jbase + cc < d) ? yh[row * d + jbase + cc] : 0.0f;
    }
    __syncthreads();
    const int rend = (int)min((int64_t)kTk, r1 - s0);
    for (int rr = 0; rr < rend; ++rr) {
      const float4 xv = *reinterpret_cast<const float4*>(&xs[rr][tr * 4]);
      const float4 yv = *reinterpret_cast<const float4*>(&ys[rr][tc * 4]);
      const double xa[4] = {(double)xv.x, (double)xv.y, (double)xv.z, (double)xv.w};
      const double ya[4] = {(double)yv.x, (double)yv.y, (double)yv.z, (double)yv.w};
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(xa[i], ya[j], acc[i][j]);   // exact product
    }
    __syncthreads();
  }
  double* out = part + (size_t)c * d * d;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int t = tbase + tr * 4 + i;
    if (t >= d) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int jj = jbase + tc * 4 + j;
      if (jj < d) out[(size_t)t * d + jj] = acc[i][j];
    }
  }
}

// M[t][j] = sum over chunks in order of part[c][t][j]
__global__ void k_cross_reduce(const double* __restrict__ part, int nch, int d, double* __restrict__ m) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t dd = (int64_t)d * d;
  if (e >= dd) return;
  double s = 0.0;
  for (int c = 0; c < nch; ++c) s += part[c * dd + e];
  m[e] = s;
}

constexpr int kPolarThreads = 1024;

// dot products of columns p and q over the group's rows, reduced over the G
// lanes of the group (G a power of two within one wave)
template <int G>
__device__ __forceinline__ void group_sum3(double& a, double& b, double& c) {
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) {
    a += __shfl_xor(a, off, 64);
    b += __shfl_xor(b, off, 64);
    c += __shfl_xor(c, off, 64);
  }
}

// Column pair of slot k in round r of the round-robin schedule over de
// (even) columns: position 0 stays, the others turn by one each round.
// Returned with p < q.
__device__ __forceinline__ void round_pair(int de, int r, int k, int& p, int& q) {
  const int mm = de - 1;
  auto at = [&](int pos) {
    if (pos == 0) return 0;
    int v = pos - 1 + r;   // < 2 * mm
    if (v >= mm) v -= mm;
    return 1 + v;
  };
  const int a = at(k), b = at(de - 1 - k);
  p = a < b ? a : b;
  q = a < b ? b : a;
}

// Work-group barrier.  LOCAL: orders LDS accesses only (outstanding global
// stores, such as the rotation log, are not waited for at every barrier).
template <bool LOCAL>
__device__ __forceinline__ void block_sync() {
  if (LOCAL) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
  } else {
    __syncthreads();
  }
}

// Jacobi rotation (cos, sin) that makes columns with squared norms alpha,
// beta and inner product gamma orthogonal: tan = sign(z) / (|z| + sqrt(1 + z^2))
// with z = (beta - alpha) / (2 gamma), written with one division.
__device__ __forceinline__ void jacobi_rotation(double alpha, double beta, double gamma, double& cs, double& sn) {
  const double h = beta - alpha;
  const double g2 = 2.0 * fabs(gamma);
  double t = g2 / (fabs(h) + sqrt(h * h + g2 * g2));
  if ((h < 0.0) != (gamma < 0.0)) t = -t;   // sign of z = h / (2 gamma)
  cs = rsqrt(1.0 + t * t);
  sn = cs * t;
}

// Sweeps of one-sided Jacobi over the columns of a (column c at a + c * lda)
// until a sweep rotates no pair.  The G lanes of a pair hold its two columns
// in registers, RPL rows each (RPL * G >= d).  With v, the rotations are
// applied to v's columns (stride d) as they happen; with rlog, each pair slot
// of each round records its rotation (cos, sin) instead ((1, 0) for none), to
// be replayed onto V afterwards.
template <int G, int RPL, bool LOCAL>
__device__ void jacobi_sweeps(double* __restrict__ a, int lda, double* __restrict__ v, double2* __restrict__ rlog,
                              int d, int de, int max_sweeps, int* __restrict__ flag, int* sweeps_done) {
  const int npairs = de / 2;
  const int grp = threadIdx.x / G;
  const int lane = threadIdx.x % G;
  const double tol = 2.220446049250313e-16 * (double)d;
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    if (threadIdx.x == 0) *flag = 0;
    block_sync<LOCAL>();
    for (int rnd = 0; rnd < de - 1; ++rnd) {
      if (grp < npairs) {
        int p, q;
        round_pair(de, rnd, grp, p, q);
        double cs = 1.0, sn = 0.0;
        if (q < d) {   // a pair with the padding column (odd d) is idle
          double* ap = a + (size_t)p * lda;
          double* aq = a + (size_t)q * lda;
          // up to 8 rows per lane stay in registers from the dot products to
          // the rotation; longer columns are read again in chunks of 8
          constexpr int CH = RPL < 8 ? RPL : 8;
          double u[CH], w[CH];
          double alpha = 0.0, beta = 0.0, gamma = 0.0;
          for (int k0 = 0; k0 < RPL; k0 += CH) {
#pragma unroll
            for (int k = 0; k < CH; ++k) {
              const int i = lane + (k0 + k) * G;
              u[k] = i < d ? ap[i] : 0.0;
              w[k] = i < d ? aq[i] : 0.0;
            }
#pragma unroll
            for (int k = 0; k < CH; ++k) {
              alpha += u[k] * u[k];
              beta += w[k] * w[k];
              gamma += u[k] * w[k];
            }
          }
          group_sum3<G>(alpha, beta, gamma);
          if (fabs(gamma) > tol * sqrt(alpha * beta) && fabs(gamma) > 0.0) {
            jacobi_rotation(alpha, beta, gamma, cs, sn);
            for (int k0 = 0; k0 < RPL; k0 += CH) {
              if (RPL > CH) {
#pragma unroll
                for (int k = 0; k < CH; ++k) {
                  const int i = lane + (k0 + k) * G;
                  u[k] = i < d ? ap[i] : 0.0;
                  w[k] = i < d ? aq[i] : 0.0;
                }
              }
#pragma unroll
              for (int k = 0; k < CH; ++k) {
                const int i = lane + (k0 + k) * G;
                if (i < d) {
                  ap[i] = cs * u[k] - sn * w[k];
                  aq[i] = sn * u[k] + cs * w[k];
                }
              }
            }
            if (v) {
              double* vp = v + (size_t)p * d;
              double* vq = v + (size_t)q * d;
              for (int i = lane; i < d; i += G) {
                const double vu = vp[i], vw = vq[i];
                vp[i] = cs * vu - sn * vw;
                vq[i] = sn * vu + cs * vw;
              }
            }
            if (lane == 0) *flag = 1;
          }
        }
        if (rlog && lane == 0) rlog[((size_t)sweep * (de - 1) + rnd) * npairs + grp] = make_double2(cs, sn);
      }
      block_sync<LOCAL>();
    }
    const int any = *flag;
    block_sync<LOCAL>();
    if (!any) break;
  }
  if (threadIdx.x == 0) *sweeps_done = sweep;
}

// V = the product of the logged rotations of `sweeps` sweeps, applied to the
// identity in the order they were taken (column c at v + c * ldv)
template <int G, int RPL>
__device__ void replay_rotations(double* __restrict__ v, int ldv, const double2* __restrict__ rlog, int d, int de,
                                 int sweeps) {
  const int npairs = de / 2;
  const int grp = threadIdx.x / G;
  const int lane = threadIdx.x % G;
  for (int e = threadIdx.x; e < d * d; e += blockDim.x) {
    const int col = e / d, row = e - col * d;
    v[(size_t)col * ldv + row] = (row == col) ? 1.0 : 0.0;
  }
  block_sync<true>();
  // the log entry of the next round is loaded one round ahead
  const size_t nrounds = (size_t)sweeps * (de - 1);
  double2 nxt = make_double2(1.0, 0.0);
  if (grp < npairs && nrounds > 0) nxt = rlog[grp];
  for (int sw = 0; sw < sweeps; ++sw)
    for (int rnd = 0; rnd < de - 1; ++rnd) {
      if (grp < npairs) {
        const double2 r = nxt;
        const size_t idx = (size_t)sw * (de - 1) + rnd + 1;
        if (idx < nrounds) nxt = rlog[idx * npairs + grp];
        int p, q;
        round_pair(de, rnd, grp, p, q);
        if (q < d && r.y != 0.0) {
          double* vp = v + (size_t)p * ldv;
          double* vq = v + (size_t)q * ldv;
          constexpr int CH = RPL < 8 ? RPL : 8;
          for (int k0 = 0; k0 < RPL; k0 += CH) {
            double u[CH], w[CH];
#pragma unroll
            for (int k = 0; k < CH; ++k) {
              const int i = lane + (k0 + k) * G;
              u[k] = i < d ? vp[i] : 0.0;
              w[k] = i < d ? vq[i] : 0.0;
            }
#pragma unroll
            for (int k = 0; k < CH; ++k) {
              const int i = lane + (k0 + k) * G;
              if (i < d) {
                vp[i] = r.x * u[k] - r.y * w[k];
                vq[i] = r.y * u[k] + r.x * w[k];
              }
            }
          }
        }
      }
      block_sync<true>();
    }
}

constexpr int kPolarMaxD = 256;
constexpr int kPolarMaxDLds = 128;   // A (d x (d+1) float64) in LDS up to this d

// One work-group.  a: out M V column-major (a[col * d + row]), then U; v: out
// V column-major; r: out R = U V^T (row-major float64); sweeps: out int
// (Jacobi sweeps run; max_sweeps + 1 when not converged); v_out: optional
// row-major copy of V.
// LDSA: the Jacobi sweeps run on a copy of M in LDS (d <= 128) and log their
// rotations in rlog; V is then rebuilt in LDS from the log.  Otherwise they
// run on a and v in global memory.  Threads exchange data through global
// memory only across __syncthreads.
template <bool LDSA>
__global__ __launch_bounds__(kPolarThreads) void k_polar(const double* __restrict__ m, int d, int max_sweeps,
                                                         double* __restrict__ a, double* __restrict__ v,
                                                         double2* __restrict__ rlog, double* __restrict__ r,
                                                         double* __restrict__ v_out, int* __restrict__ sweeps) {
  __shared__ int flag;
  __shared__ int sweeps_done;
  __shared__ int best_k;
  __shared__ double sig[kPolarMaxD];    // singular values; -1 marks a column still to complete
  __shared__ double work[kPolarMaxD];   // residual norms, then projections
  __shared__ double red[kPolarThreads / 64];
  extern __shared__ double lds_mat[];   // LDSA: d x (d + 1)
  const int dd = d * d;
  const int ld = LDSA ? d + 1 : d;
  double* aw = LDSA ? lds_mat : a;
  for (int e = threadIdx.x; e < dd; e += blockDim.x) {
    const int col = e / d, row = e - col * d;
    aw[(size_t)col * ld + row] = m[(size_t)row * d + col];
    if (!LDSA) v[e] = (row == col) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int de = d + (d & 1);
  const int npairs = de / 2;
  // lanes per pair: a power of two in [1, 64] with npairs * G <= 1024
  // lanes per pair: the largest power of two <= 64 with npairs * G <= 1024
  // (a round's latency falls with more lanes per pair)
  int g = 64;
  while (g > 8 && npairs * g > kPolarThreads) g >>= 1;
  double* vv = LDSA ? nullptr : v;
  double2* lg = LDSA ? rlog : nullptr;
  // G = 64, 32, 16, 8 for d <= 32, 64, 128, 256: RPL * G >= d rows per column
  // rows per lane RPL * G >= d: d <= 32, 64, 128, 256 -> G = 64, 32, 16, 8
  // (LDSA: d <= 128)
  if (g == 64) jacobi_sweeps<64, 1, LDSA>(aw, ld, vv, lg, d, de, max_sweeps, &flag, &sweeps_done);
  else if (g == 32) jacobi_sweeps<32, 2, LDSA>(aw, ld, vv, lg, d, de, max_sweeps, &flag, &sweeps_done);
  else if (LDSA || g == 16) jacobi_sweeps<16, 8, LDSA>(aw, ld, vv, lg, d, de, max_sweeps, &flag, &sweeps_done);
  else jacobi_sweeps<8, 32, LDSA>(aw, ld, vv, lg, d, de, max_sweeps, &flag, &sweeps_done);
  if (LDSA) {
    __syncthreads();
    for (int e = threadIdx.x; e < dd; e += blockDim.x) {
      const int col = e / d, row = e - col * d;
      a[e] = lds_mat[(size_t)col * ld + row];
    }
    __syncthreads();
    const int nsw = sweeps_done;
    switch (g) {
      case 64: replay_rotations<64, 1>(lds_mat, ld, rlog, d, de, nsw); break;
      case 32: replay_rotations<32, 2>(lds_mat, ld, rlog, d, de, nsw); break;
      default: replay_rotations<16, 8>(lds_mat, ld, rlog, d, de, nsw); break;
    }
    for (int e = threadIdx.x; e < dd; e += blockDim.x) {
      const int col = e / d, row = e - col * d;
      v[e] = lds_mat[(size_t)col * ld + row];
    }
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nw = blockDim.x >> 6;
  // column norms = singular values, one wave per column
  for (int col = wave; col < d; col += nw) {
    double s = 0.0;
    for (int i = lane; i < d; i += 64) s += a[(size_t)col * d + i] * a[(size_t)col * d + i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) sig[col] = sqrt(s);
  }
  __syncthreads();
  double smax = 0.0;
  for (int i = threadIdx.x; i < d; i += blockDim.x) smax = fmax(smax, sig[i]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) smax = fmax(smax, __shfl_xor(smax, off, 64));
  if (lane == 0) red[wave] = smax;
  __syncthreads();
  smax = 0.0;
  for (int i = 0; i < nw; ++i) smax = fmax(smax, red[i]);
  // numerical rank: columns at or below d * eps * sigma_max are completed below
  const double thr = smax * (double)d * 2.220446049250313e-16;
  for (int e = threadIdx.x; e < dd; e += blockDim.x) {
    const double sc = sig[e / d];
    if (sc > thr && sc > 0.0) a[e] = a[e] / sc;
  }
  __syncthreads();
  for (int col = threadIdx.x; col < d; col += blockDim.x)
    if (!(sig[col] > thr && sig[col] > 0.0)) sig[col] = -1.0;
  __syncthreads();
  // basis completion, one missing column at a time: start from the unit
  // vector e_k with the largest residual against the accepted columns, then
  // two passes of classical Gram-Schmidt and a normalisation
  for (int col = 0; col < d; ++col) {
    if (sig[col] >= 0.0) continue;   // uniform: sig is in LDS, read after a barrier
    double* u = a + (size_t)col * d;
    for (int k = threadIdx.x; k < d; k += blockDim.x) {
      double s = 0.0;
      for (int c = 0; c < d; ++c)
        if (sig[c] >= 0.0) s += a[(size_t)c * d + k] * a[(size_t)c * d + k];
      work[k] = 1.0 - s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int bk = 0;
      for (int k = 1; k < d; ++k)
        if (work[k] > work[bk]) bk = k;
      best_k = bk;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < d; i += blockDim.x) u[i] = (i == best_k) ? 1.0 : 0.0;
    __syncthreads();
    for (int pass = 0; pass < 2; ++pass) {
      for (int c = threadIdx.x; c < d; c += blockDim.x) {
        double s = 0.0;
        if (sig[c] >= 0.0)
          for (int i = 0; i < d; ++i) s += a[(size_t)c * d + i] * u[i];
        work[c] = s;
      }
      __syncthreads();
      for (int i = threadIdx.x; i < d; i += blockDim.x) {
        double s = u[i];
        for (int c = 0; c < d; ++c)
          if (sig[c] >= 0.0) s -= work[c] * a[(size_t)c * d + i];
        u[i] = s;
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int i = 0; i < d; ++i) s += u[i] * u[i];
      work[0] = 1.0 / sqrt(s);
    }
    __syncthreads();
    const double inv = work[0];
    for (int i = threadIdx.x; i < d; i += blockDim.x) u[i] *= inv;
    __syncthreads();
    if (threadIdx.x == 0) sig[col] = 0.0;   // accepted from now on
    __syncthreads();
  }
  // R[t][j] = sum over columns c of U[t][c] V[j][c]
  for (int e = threadIdx.x; e < dd; e += blockDim.x) {
    const int t = e / d, j = e - t * d;
    double s = 0.0;
    for (int c = 0; c < d; ++c) s += a[(size_t)c * d + t] * v[(size_t)c * d + j];
    r[e] = s;
    if (v_out) v_out[e] = v[(size_t)j * d + t];   // V[t][j]
  }
  if (threadIdx.x == 0) *sweeps = sweeps_done < max_sweeps ? sweeps_done : max_sweeps + 1;
}

}  // namespace

int launch_rotate(const float* x, int64_t n, int d, const double* r, float* y, hipStream_t s) {
  if (n == 0) return MIPQ_OK;
  const int ctiles = (d + kTile - 1) / kTile;
  const int64_t rtiles = (n + kRotRows - 1) / kRotRows;
  const int64_t nblocks = rtiles * ctiles;
  const int64_t grid = ((nblocks + 7) / 8) * 8;
  if (grid > 0x7fffffff) return fail(MIPQ_EUNSUPPORTED, "too many rows for one rotation launch");
  ProfScope ps(MIPQ_K_ROTATE, s);
  k_rotate<<<(unsigned)grid, kThreads, 0, s>>>(x, n, d, r, y, ctiles, nblocks);
  MIPQ_LAUNCHED("k_rotate");
  return MIPQ_OK;
}

int cross_chunks(int64_t n, int d) {
  const int tiles = (d + kTile - 1) / kTile;
  int64_t nch = (n + 1023) / 1024;
  int64_t cap = 2048 / (tiles * tiles);
  if (cap < 1) cap = 1;
  if (nch > cap) nch = cap;
  return nch < 1 ? 1 : (int)nch;
}

int launch_cross(const float* x, const float* yh, int64_t n, int d, int nch, double* part, double* m,
                 hipStream_t s) {
  const int tiles = (d + kTile - 1) / kTile;
  const int64_t rpc = (n + nch - 1) / nch;
  ProfScope ps(MIPQ_K_CROSS, s);
  k_cross_partial<<<(unsigned)(nch * tiles * tiles), kThreads, 0, s>>>(x, yh, n, d, rpc > 0 ? rpc : 1, tiles,
                                                                       part);
  MIPQ_LAUNCHED("k_cross_partial");
  const int64_t dd = (int64_t)d * d;
  k_cross_reduce<<<(unsigned)((dd + 255) / 256), 256, 0, s>>>(part, nch, d, m);
  MIPQ_LAUNCHED("k_cross_reduce");
  return MIPQ_OK;
}

size_t polar_log_bytes(int d, int max_sweeps) {
  if (d > kPolarMaxDLds) return 0;
  const int de = d + (d & 1);
  return (size_t)max_sweeps * (de - 1) * (de / 2) * sizeof(double2);
}

// c = op(a) op(b) for d x d row-major float64 matrices (op: optional
// transpose), one thread per output, k ascending; j is the fastest index so
// that b's rows (or a^T's) are read coalesced.
__global__ void k_gemm64(const double* __restrict__ a, const double* __restrict__ b, int d, int ta, int tb,
                         double* __restrict__ c) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)d * d) return;
  const int i = (int)(e / d), j = (int)(e - (int64_t)i * d);
  double acc = 0.0;
  for (int k = 0; k < d; ++k) {
    const double av = ta ? a[(size_t)k * d + i] : a[(size_t)i * d + k];
    const double bv = tb ? b[(size_t)j * d + k] : b[(size_t)k * d + j];
    acc += av * bv;
  }
  c[e] = acc;
}

int launch_gemm64(const double* a, const double* b, int d, bool ta, bool tb, double* c, hipStream_t s) {
  const int64_t dd = (int64_t)d * d;
  k_gemm64<<<(unsigned)((dd + 255) / 256), 256, 0, s>>>(a, b, d, ta ? 1 : 0, tb ? 1 : 0, c);
  MIPQ_LAUNCHED("k_gemm64");
  return MIPQ_OK;
}

// R for M: without v0, one polar launch.  With v0 (orthogonal, row-major):
// the sweeps run on M0 = M V0 (written to m0), giving U and V_J with
// R_J = U V_J^T; then R = R_J V0^T and V = V0 V_J (to v_out).
int launch_polar(const double* m, int d, int max_sweeps, const double* v0, double* m0, double* a, double* v,
                 double* rj, double* vj, void* rlog, double* r, double* v_out, int* sweeps, hipStream_t s) {
  if (d < 1 || d > kPolarMaxD) return fail(MIPQ_EUNSUPPORTED, "the rotation fit supports 1 <= d <= %d", kPolarMaxD);
  int rc;
  const double* mm = m;
  double* r_out = r;
  double* vj_out = v_out;
  if (v0) {
    if ((rc = launch_gemm64(m, v0, d, false, false, m0, s))) return rc;
    mm = m0;
    r_out = rj;
    vj_out = vj;
  }
  {
    ProfScope ps(MIPQ_K_POLAR, s);
    if (d <= kPolarMaxDLds) {
      if (!rlog) return fail(MIPQ_EINVAL, "rotation log missing");
      const size_t shm = (size_t)d * (d + 1) * sizeof(double);
      k_polar<true><<<1, kPolarThreads, shm, s>>>(mm, d, max_sweeps, a, v, static_cast<double2*>(rlog), r_out,
                                                  vj_out, sweeps);
    } else {
      k_polar<false><<<1, kPolarThreads, 0, s>>>(mm, d, max_sweeps, a, v, nullptr, r_out, vj_out, sweeps);
    }
    MIPQ_LAUNCHED("k_polar");
  }
  if (v0) {
    if ((rc = launch_gemm64(rj, v0, d, false, true, r, s))) return rc;
    if (v_out && (rc = launch_gemm64(v0, vj, d, false, false, v_out, s))) return rc;
  }
  return MIPQ_OK;
}

}  // namespace mipq
