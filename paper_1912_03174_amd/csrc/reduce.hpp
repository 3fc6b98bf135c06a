// Wave- and block-wide reductions in a fixed order (shuffle trees, no
// floating-point atomics), shared by the kernels that must give bitwise
// identical results for the same input whichever launch computes them.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace td {
namespace {

constexpr int WAVE = 64;

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}
__device__ inline double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, WAVE));
  return v;
}
__device__ inline double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, WAVE));
  return v;
}

// Block-wide sum for blockDim.x = 1024 (16 waves); result valid in all threads.
__device__ double block_sum_1024(double v, double* sh) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double t = (threadIdx.x < 16) ? sh[threadIdx.x] : 0.0;
  if (w == 0) t = wave_sum(t);
  if (threadIdx.x == 0) sh[16] = t;
  __syncthreads();
  return sh[16];
}
__device__ double block_max_1024(double v, double* sh) {
  v = wave_max(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double t = (threadIdx.x < 16) ? sh[threadIdx.x] : -INFINITY;
  if (w == 0) t = wave_max(t);
  if (threadIdx.x == 0) sh[16] = t;
  __syncthreads();
  return sh[16];
}
__device__ double block_min_1024(double v, double* sh) {
  v = wave_min(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double t = (threadIdx.x < 16) ? sh[threadIdx.x] : INFINITY;
  if (w == 0) t = wave_min(t);
  if (threadIdx.x == 0) sh[16] = t;
  __syncthreads();
  return sh[16];
}

}  // namespace
}  // namespace td
