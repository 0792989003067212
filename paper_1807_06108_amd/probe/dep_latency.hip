// Dependent-issue latency probe: one wavefront runs one dependency chain of
// a single instruction class and times it with the shader clock (s_memtime);
// the constant 100 MHz clock (s_memrealtime) over the same span gives the
// shader clock rate.  Cycles per dependent operation bound the state
// recursion of a rollout, which is one such chain per sample.  One store
// per thread, in bounds of the 64-element output buffer.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdint.h>
#include <stdlib.h>

#define CHECK(x)                                                          \
  do {                                                                    \
    hipError_t e_ = (x);                                                  \
    if (e_ != hipSuccess) {                                               \
      fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));            \
      exit(1);                                                            \
    }                                                                     \
  } while (0)

constexpr int N = 4096;

#define CHAIN(name, T, init, body)                                                   \
  __global__ __launch_bounds__(64) void name(T* out, T seed, long long* clk) {        \
    T x = init;                                                                      \
    const long long r0 = wall_clock64();                                             \
    const long long t0 = clock64();                                                  \
    _Pragma("unroll 16") for (int i = 0; i < N; ++i) { body; }                       \
    asm volatile("" ::"v"(x));                                                       \
    const long long t1 = clock64();                                                  \
    const long long r1 = wall_clock64();                                             \
    out[threadIdx.x] = x;                                                            \
    if (threadIdx.x == 0) {                                                          \
      clk[0] = t1 - t0;                                                              \
      clk[1] = r1 - r0;                                                              \
    }                                                                                \
  }

CHAIN(c_fma, float, seed + threadIdx.x, x = __builtin_fmaf(x, 0.999f, 0.001f))
CHAIN(c_add, float, seed + threadIdx.x, x = x + 0.001f)
CHAIN(c_sin, float, 0.01f * threadIdx.x, x = __builtin_amdgcn_sinf(x))
CHAIN(c_rcp, float, 2.0f + threadIdx.x, x = __builtin_amdgcn_rcpf(x) + 1.0f)
CHAIN(c_fma64, double, seed + threadIdx.x, x = __builtin_fma(x, 0.999, 0.001))
CHAIN(c_mad64, uint32_t, seed + threadIdx.x,
      { const uint64_t p = (uint64_t)0xD2511F53u * x; x = (uint32_t)(p >> 32) ^ (uint32_t)p; })

template <typename T, typename K>
void run(const char* name, K kern, T seed, int ops, const char* what) {
  T* out;
  long long* clk;
  long long h[2] = {0, 0};
  CHECK(hipMalloc(&out, 64 * sizeof(T)));
  CHECK(hipMalloc(&clk, 2 * sizeof(long long)));
  for (int rep = 0; rep < 3; ++rep) kern<<<1, 64>>>(out, seed, clk);
  CHECK(hipGetLastError());
  CHECK(hipDeviceSynchronize());
  CHECK(hipMemcpy(h, clk, sizeof(h), hipMemcpyDeviceToHost));
  const double cyc = (double)h[0] / ((double)N * ops);
  const double ghz = (double)h[0] / ((double)h[1] * 10.0);
  printf("%-10s %6.2f cycles per dependent operation (shader clock %.2f GHz)  %s\n", name, cyc,
         ghz, what);
  CHECK(hipFree(out));
  CHECK(hipFree(clk));
}

int main() {
  run("fma32", c_fma, 1.0f, 1, "v_fma_f32");
  run("add32", c_add, 1.0f, 1, "v_add_f32");
  run("sin", c_sin, 0.0f, 1, "v_sin_f32");
  run("rcp+add", c_rcp, 0.0f, 2, "v_rcp_f32 then v_add_f32 (average of the two)");
  run("fma64", c_fma64, 1.0, 1, "v_fma_f64");
  run("mad64+xor", c_mad64, 1u, 2, "v_mad_u64_u32 then v_xor_b32 (average of the two)");
  return 0;
}
