// Shared device/host helpers of the KS library (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstdio>

#define KS_WAVE 64

namespace ks {

// Upper bounds fixed at compile time.
constexpr int MAX_NQ = 27;     // quadrature points per element
constexpr int MAX_NLOC = 10;   // nodes per element (P2)
constexpr int MAX_K = 64;      // right-hand sides / orbitals

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block-wide sum of one value per thread (blockDim.x multiple of 64, <= 1024);
// result valid on thread 0.  `sh` needs blockDim.x / 64 doubles.
__device__ __forceinline__ double block_sum(double v, double *sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    const int nw = blockDim.x >> 6;
    for (int i = 0; i < nw; ++i) r += sh[i];
  }
  __syncthreads();
  return r;
}

}  // namespace ks
