// Deterministic wavefront (64 lanes) and workgroup (256 threads) reductions.
// The combination order depends only on lane and wave indices, never on
// timing, so repeated runs give bitwise-equal results.
#pragma once
#include <hip/hip_runtime.h>

namespace mppi {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Workgroup reductions over NW wavefronts: every thread gets the result.
// `lds` holds NW doubles; a __syncthreads() separates consecutive uses.
template <int NW = kWaves>
__device__ __forceinline__ double block_min(double v, double* lds) {
  v = wave_min(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  double r = lds[0];
#pragma unroll
  for (int w = 1; w < NW; ++w) r = fmin(r, lds[w]);
  __syncthreads();
  return r;
}

template <int NW = kWaves>
__device__ __forceinline__ double block_sum(double v, double* lds) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  double r = lds[0];
#pragma unroll
  for (int w = 1; w < NW; ++w) r += lds[w];
  __syncthreads();
  return r;
}

}  // namespace mppi
