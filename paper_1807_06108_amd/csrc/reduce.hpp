// Deterministic wavefront (64 lanes) and workgroup (256 threads) reductions.
// The combination order depends only on lane and wave indices, never on
// timing, so repeated runs give bitwise-equal results.
#pragma once
#include <hip/hip_runtime.h>

namespace mppi {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

// Cross-lane moves in registers (no LDS round trip): DPP within a row of 16
// lanes, the gfx950 permlane swaps across rows.  Each stage combines a
// lane's value with its partner's, a + b with b + a (equal in IEEE
// arithmetic), so after the six stages every lane holds bitwise the same
// result, formed in an order fixed by lane positions.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

constexpr int kDppXor1 = 0xB1;        // quad_perm [1, 0, 3, 2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2, 3, 0, 1]
constexpr int kDppHalfMirror = 0x141; // lane i <-> 7 - i within each 8
constexpr int kDppMirror = 0x140;     // lane i <-> 15 - i within each 16

// (a, b): this lane's row-pair halves (rows 2j and 2j + 1) or wave halves.
template <bool ROWS>
__device__ __forceinline__ void swap_f64(double v, double& a, double& b) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  if constexpr (ROWS) {
    const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    a = __hiloint2double(h[0], l[0]);
    b = __hiloint2double(h[1], l[1]);
  } else {
    const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    a = __hiloint2double(h[0], l[0]);
    b = __hiloint2double(h[1], l[1]);
  }
}

template <typename Op>
__device__ __forceinline__ double wave_reduce(double v, Op op) {
  // after the quad stages every lane of a quad holds the same value, so the
  // mirrors act as exchanges between quads and between half-rows
  v = op(v, dpp_f64<kDppXor1>(v));
  v = op(v, dpp_f64<kDppXor2>(v));
  v = op(v, dpp_f64<kDppHalfMirror>(v));
  v = op(v, dpp_f64<kDppMirror>(v));
  double a, b;
  swap_f64<true>(v, a, b);
  v = op(a, b);
  swap_f64<false>(v, a, b);
  return op(a, b);
}

__device__ __forceinline__ double wave_min(double v) {
  return wave_reduce(v, [](double x, double y) { return fmin(x, y); });
}

__device__ __forceinline__ double wave_sum(double v) {
  return wave_reduce(v, [](double x, double y) { return x + y; });
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
