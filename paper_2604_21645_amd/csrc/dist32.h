// The library's decision arithmetic for one subspace distance.
//
// sum over t ascending of (x_t - c_t)^2 with every subtraction, square and
// running sum rounded to float32.  The library is compiled with
// -ffp-contract=off, so the compiler never fuses the square into the sum.
// Every kernel that turns a distance into a code (plain assignment, the
// exact re-decision of ambiguous matrix-core results, the objective) uses
// this one function, so all precisions produce the same codes.
#pragma once

#include <hip/hip_runtime.h>

namespace mipq {

template <int DS>
__device__ __forceinline__ float sqdist_fixed(const float* x, const float* c) {
  float acc = 0.0f;
#pragma unroll
  for (int t = 0; t < DS; ++t) {
    float df = x[t] - c[t];
    float sq = df * df;
    acc = acc + sq;   // 0 + first square is exact
  }
  return acc;
}

__device__ __forceinline__ float sqdist_rt(const float* x, const float* c, int ds) {
  float acc = 0.0f;
  for (int t = 0; t < ds; ++t) {
    float df = x[t] - c[t];
    float sq = df * df;
    acc = acc + sq;
  }
  return acc;
}

}  // namespace mipq
