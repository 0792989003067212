// Wave placement probe: which SIMD of its compute unit each wavefront of a
// workgroup runs on, read from the HW_ID hardware register (SIMD_ID, bits
// 5:4).  Launches the workgroup shapes of the rollout kernels (8 waves = 512
// threads, 4 waves = 256 threads) and reports, per wave index, how often it
// shared a SIMD with each other wave of its workgroup.  One store per wave,
// in bounds of the blocks x waves output buffer.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>

#define CHECK(x)                                                          \
  do {                                                                    \
    hipError_t e_ = (x);                                                  \
    if (e_ != hipSuccess) {                                               \
      fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));            \
      exit(1);                                                            \
    }                                                                     \
  } while (0)

template <int W>
__global__ __launch_bounds__(64 * W) void placement(unsigned* out) {
  // s_getreg_b32 HW_REG_HW_ID: size 32, offset 0, register id 4
  const unsigned hw = __builtin_amdgcn_s_getreg((31 << 11) | (0 << 6) | 4);
  if ((threadIdx.x & 63) == 0) out[blockIdx.x * W + (threadIdx.x >> 6)] = hw;
}

template <int W>
void run(int blocks) {
  unsigned* d;
  const size_t n = (size_t)blocks * W;
  unsigned* h = (unsigned*)malloc(n * sizeof(unsigned));
  CHECK(hipMalloc(&d, n * sizeof(unsigned)));
  placement<W><<<blocks, 64 * W>>>(d);
  CHECK(hipGetLastError());
  CHECK(hipDeviceSynchronize());
  CHECK(hipMemcpy(h, d, n * sizeof(unsigned), hipMemcpyDeviceToHost));
  printf("%d waves per workgroup, %d workgroups: fraction of workgroups in which wave i "
         "shares wave j's SIMD\n      ", W, blocks);
  for (int j = 0; j < W; ++j) printf("  w%d  ", j);
  printf("\n");
  for (int i = 0; i < W; ++i) {
    printf("  w%d  ", i);
    for (int j = 0; j < W; ++j) {
      int same = 0;
      for (int b = 0; b < blocks; ++b)
        same += ((h[b * W + i] >> 4) & 3) == ((h[b * W + j] >> 4) & 3);
      printf(" %4.2f ", (double)same / blocks);
    }
    printf("\n");
  }
  CHECK(hipFree(d));
  free(h);
}

int main() {
  run<8>(256);
  run<4>(256);
  return 0;
}
