// Fixed-order workgroup reductions (library-internal).
#pragma once

#include <hip/hip_runtime.h>

namespace chimera {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// Sum over the workgroup, fixed order; every thread gets the result.
// red must hold BS/64 + 1 doubles; leaves red reusable on return.
template <int BS>
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < BS / 64; ++i) t += red[i];
    red[BS / 64] = t;
  }
  __syncthreads();
  const double r = red[BS / 64];
  __syncthreads();
  return r;
}

template <int BS>
__device__ __forceinline__ double block_max(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = red[0];
#pragma unroll
    for (int i = 1; i < BS / 64; ++i) t = fmax(t, red[i]);
    red[BS / 64] = t;
  }
  __syncthreads();
  const double r = red[BS / 64];
  __syncthreads();
  return r;
}

}  // namespace chimera
