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

// N sums (or maxima) over the workgroup in one pass: 3 barriers instead of 3N.
template <int BS, int N, bool MAX>
__device__ __forceinline__ void block_reduce(double (&v)[N], double* red /* >= N*(BS/64+1) */) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double y = __shfl_down(v[i], o, 64);
      v[i] = MAX ? fmax(v[i], y) : v[i] + y;
    }
    if (lane == 0) red[i * (BS / 64 + 1) + w] = v[i];
  }
  __syncthreads();
  if (threadIdx.x < N) {
    const int i = threadIdx.x;
    double t = red[i * (BS / 64 + 1)];
    for (int k = 1; k < BS / 64; ++k) {
      const double y = red[i * (BS / 64 + 1) + k];
      t = MAX ? fmax(t, y) : t + y;
    }
    red[i * (BS / 64 + 1) + BS / 64] = t;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = red[i * (BS / 64 + 1) + BS / 64];
  __syncthreads();
}

// Maxima over the workgroup of N ints; every thread gets them (max is exact,
// so the order does not matter).  red must hold N*(BS/64) ints and is not
// touched again by this call after its barrier.
template <int BS, int N>
__device__ __forceinline__ void block_max_i32(int (&v)[N], int* red) {
  constexpr int NW = BS / 64;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[i] = max(v[i], __shfl_xor(v[i], o, 64));
    if (lane == 0) red[i * NW + w] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < N; ++i) {
    int t = red[i * NW];
#pragma unroll
    for (int k = 1; k < NW; ++k) t = max(t, red[i * NW + k]);
    v[i] = t;
  }
}

}  // namespace chimera
