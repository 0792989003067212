// Issue-rate probe: lane-operations per CU per clock of the instruction
// classes the rollout is made of (fp32 FMA, 32x32->64 multiply, XOR,
// transcendentals, fp64 FMA, conversions), on a grid large enough to fill
// every SIMD.  Each thread runs CH independent dependency chains for ITER
// iterations and stores one value (one store per thread, in bounds of the
// blocks * threads output buffer).  The results weight the algorithmic
// operation counts of the rollout roofline.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdint.h>
#include <math.h>

constexpr int ITER = 2048, CH = 8;

#define KERN(name, T, init, body)                                          \
  __global__ __launch_bounds__(256) void name(T* out, T seed) {             \
    T v[CH];                                                               \
    _Pragma("unroll") for (int c = 0; c < CH; ++c) v[c] = init;             \
    for (int i = 0; i < ITER; ++i) {                                       \
      _Pragma("unroll") for (int c = 0; c < CH; ++c) { T x = v[c]; body; v[c] = x; } \
    }                                                                      \
    T s = v[0];                                                            \
    _Pragma("unroll") for (int c = 1; c < CH; ++c) s = s + v[c];            \
    out[blockIdx.x * 256 + threadIdx.x] = s;                                \
  }

KERN(k_fma, float, seed + c + threadIdx.x, x = __builtin_fmaf(x, 0.999f, 0.001f))
KERN(k_mad64, uint32_t, seed + c + threadIdx.x, { uint64_t p = (uint64_t)0xD2511F53u * x; x = (uint32_t)(p >> 32) + (uint32_t)p; })
KERN(k_mulhi, uint32_t, seed + c + threadIdx.x, x = __umulhi(x, 0xD2511F53u) + 7u)
KERN(k_mullo, uint32_t, seed + c + threadIdx.x, x = x * 0xD2511F53u + 7u)
KERN(k_xor3, uint32_t, seed + c + threadIdx.x, x = x ^ (x >> 3) ^ seed)
KERN(k_log, float, 1.5f + c + threadIdx.x, x = __builtin_amdgcn_logf(x) + 2.0f)
KERN(k_sin, float, 0.1f * c + threadIdx.x * 1e-3f, x = __builtin_amdgcn_sinf(x))
KERN(k_sqrt, float, 2.0f + c + threadIdx.x, x = __builtin_amdgcn_sqrtf(x) + 1.0f)
KERN(k_rcp, float, 2.0f + c + threadIdx.x, x = __builtin_amdgcn_rcpf(x) + 1.0f)
KERN(k_fma64, double, seed + c + threadIdx.x, x = __builtin_fma(x, 0.999, 0.001))
KERN(k_cvt, float, 1.0f + c, x = (float)(((uint32_t)__float_as_uint(x)) >> 9) * 1e-3f)

template <typename T, typename K>
double run(const char* name, K kern, T seed, int ops_per_body) {
  const int blocks = 256 * 16, threads = 256;
  T* out = nullptr;
  if (hipMalloc(&out, sizeof(T) * (size_t)blocks * threads) != hipSuccess) return -1;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -1;
  kern<<<blocks, threads>>>(out, seed);
  if (hipEventRecord(a) != hipSuccess) return -1;
  for (int r = 0; r < 5; ++r) kern<<<blocks, threads>>>(out, seed);
  if (hipEventRecord(b) != hipSuccess || hipEventSynchronize(b) != hipSuccess) return -1;
  float ms = 0;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return -1;
  const double lane_ops = 5.0 * blocks * threads * (double)ITER * CH * ops_per_body;
  const double per_cu_clk = lane_ops / (ms * 1e-3) / 256.0 / 2.4e9;
  printf("%-8s %8.3f ms  %8.2f Tlane-op/s  %6.1f lane-op/CU/clk (at 2.4 GHz)\n", name, ms,
         lane_ops / (ms * 1e-3) / 1e12, per_cu_clk);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  (void)hipFree(out);
  return per_cu_clk;
}

int main() {
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, 0) != hipSuccess) return 1;
  printf("device %s, %d CUs, clock %d kHz, arch %s\n", p.name, p.multiProcessorCount,
         p.clockRate, p.gcnArchName);
  run<float>("fma", k_fma, 1.0f, 1);
  run<uint32_t>("mad64+add", k_mad64, 3u, 1);
  run<uint32_t>("mulhi+add", k_mulhi, 3u, 1);
  run<uint32_t>("mullo", k_mullo, 3u, 1);
  run<uint32_t>("xor3/shr", k_xor3, 3u, 1);
  run<float>("log+add", k_log, 1.0f, 1);
  run<float>("sin", k_sin, 1.0f, 1);
  run<float>("sqrt+add", k_sqrt, 1.0f, 1);
  run<float>("rcp+add", k_rcp, 1.0f, 1);
  run<double>("fma64", k_fma64, 1.0, 1);
  run<float>("cvt", k_cvt, 1.0f, 1);
  return 0;
}
