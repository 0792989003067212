// Counter-based noise for the rollout: Philox4x32-10 blocks in registers,
// 24-bit uniforms, Box-Muller normals and jump counts by integer inversion.
//
// Generator: Philox4x32-10 of Salmon, Moraes, Dror, Shaw, "Parallel random
// numbers: as easy as 1, 2, 3" (SC'11): per round one 32x32->64 multiply of
// words 0 and 2 by the two Philox constants, XOR of the high halves with the
// other words and the round key, then the fixed permutation; the key is
// bumped by the golden-ratio and sqrt(3) Weyl constants between rounds.
//
// Stream layout (the library's own definition; the paper fixes no
// generator):  key = (seed lo, seed hi),
//   counter = (t, k, iteration, block | controller_id << 8).
// Word 1 carries the per-lane sample index so that every multiply of round 1
// and one of rounds 2 and 3 see wavefront-uniform operands and run on the
// scalar unit.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mppi {

struct Words4 {
  uint32_t w0, w1, w2, w3;
};

__device__ __forceinline__ Words4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n1 = (uint32_t)p1;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    const uint32_t n3 = (uint32_t)p0;
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
  }
  return Words4{c0, c1, c2, c3};
}

// Two standard normals from two words (Box & Muller 1958), fp32:
// u = ((wr >> 8) + 1) / 2^24 in (0, 1] and v = (wa >> 8) / 2^24 in [0, 1) are
// exact in fp32; radius sqrt(-2 ln u); the hardware sine/cosine take their
// argument in revolutions, so the angle 2 pi v is v itself.
__device__ __forceinline__ void box_muller(uint32_t wr, uint32_t wa, float& z0, float& z1) {
  const float u = (float)((wr >> 8) + 1u) * 0x1p-24f;
  const float v = (float)(wa >> 8) * 0x1p-24f;
  // -2 ln u = -2 ln(2) log2(u)
  const float r = __builtin_amdgcn_sqrtf(-1.38629436111989061883f * __builtin_amdgcn_logf(u));
  z0 = r * __builtin_amdgcn_cosf(v);
  z1 = r * __builtin_amdgcn_sinf(v);
}

__device__ __forceinline__ float box_muller_cos(uint32_t wr, uint32_t wa) {
  const float u = (float)((wr >> 8) + 1u) * 0x1p-24f;
  const float v = (float)(wa >> 8) * 0x1p-24f;
  const float r = __builtin_amdgcn_sqrtf(-1.38629436111989061883f * __builtin_amdgcn_logf(u));
  return r * __builtin_amdgcn_cosf(v);
}

// Jump count by inversion: the number of thresholds the word reaches.  The
// first eight thresholds come from th8 (kept in vector registers by the
// callers), longer tables continue from th_all in a loop.
__device__ __forceinline__ int jump_count(uint32_t w, const uint32_t* th8,
                                          const uint32_t* th_all, int n_th) {
  int n = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) n += (j < n_th && w >= th8[j]) ? 1 : 0;
  for (int j = 8; j < n_th; ++j) n += (w >= th_all[j]) ? 1 : 0;
  return n;
}

}  // namespace mppi
