// Kernels of one MPPI iteration on a jump-diffusion process (gfx950).
//
//   rollout_kernel  sampling + propagation + path cost, one sample per lane
//                   (Algorithm 1 inner loops; eqs. (34)-(35)); its epilogue
//                   forms per-workgroup min / normaliser partials of eq. (37)
//                   and the last workgroup to finish combines them.
//   update_kernel   U += alpha * sum_k w_k eps_k (eqs. (36)/(49)): a
//                   (T*m) x K matrix-vector product, each eps row read once,
//                   coalesced along k; the last workgroup sums the chunk
//                   partials in a fixed order and writes U.
//   shift_kernel    execute u_0, shift left, append u_init (Algorithm 1).
//   restats_kernel  the rollout epilogue alone, for costs set by the caller.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "../../include/mppi_jump.h"
#include "models.hpp"
#include "reduce.hpp"
#include "rng.hpp"

namespace mppi {

// Per-workgroup partial of the rollout epilogue; one per 128-byte line so that
// workgroups on different XCDs never share a cache line.
struct alignas(128) WgPartial {
  double rho;    // min of the finite S_k of the workgroup (+inf if none)
  double eta;    // sum exp(-(S_k - rho)/lambda) over them
  int32_t nfin;  // number of finite S_k
};

struct DevParams {
  int K, T, Ks, n_th;
  uint32_t key0, key1, ctr3;  // ctr3 = controller_id << 8
  int cost_form;
  float dt, lam, alpha, pen;
  double lam_d;
  float sigma[4], sigJ[4];
  float isc[4];   // lambda c / sigma^2   (0 where sigma = 0)
  float isv[4];   // 0.5 lambda (c - 1) / sigma^2
  float halfR[4];
  float Q[12], Qf[12], goal[12];
  ModelConsts mc;
  uint32_t th[MPPI_JUMP_MAX_LEVELS];
};

struct Buffers {
  float* U;           // [T][m]
  float* eps;         // [T][m][Ks]
  double* S;          // [K]
  double* E;          // [K] exp(-(S_k - rho_wg)/lambda)
  WgPartial* part;    // [ceil(K/256)]
  double* scale;      // [ceil(K/256)] exp(-(rho_wg - rho)/lambda)
  double* upart;      // [T*m][nch]
  mppi_jump_stats* stats;
  uint32_t* counters; // [0] rollout, [1] update
  float* dbg_zD;      // [K][T][m]
  int32_t* dbg_N;     // [K][T]
  float* dbg_zJ;      // [K][T][q]
};

// ------------------------------------------------------------------ epilogue
// Per-workgroup statistics of eq. (37) for the 256 samples of this
// workgroup, then the combine by the last workgroup to arrive.
__device__ __forceinline__ void stats_epilogue(const DevParams& p, const Buffers& b, double Sd,
                                               bool active) {
  __shared__ double lds[kWaves];
  __shared__ int is_last;
  const bool fin = active && isfinite(Sd);
  const double s = fin ? Sd : INFINITY;
  const double rho_wg = block_min(s, lds);
  const double e = fin ? exp(-(Sd - rho_wg) / p.lam_d) : 0.0;
  const int k = blockIdx.x * kBlock + threadIdx.x;
  if (active) b.E[k] = e;
  const double eta_wg = block_sum(e, lds);
  const double nfin = block_sum(fin ? 1.0 : 0.0, lds);
  if (threadIdx.x == 0) {
    b.part[blockIdx.x].rho = rho_wg;
    b.part[blockIdx.x].eta = eta_wg;
    b.part[blockIdx.x].nfin = (int32_t)nfin;
    __threadfence();
    const uint32_t prev = atomicAdd(&b.counters[0], 1u);
    is_last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  const int nwg = gridDim.x;
  double m = INFINITY;
  for (int j = threadIdx.x; j < nwg; j += kBlock)
    if (b.part[j].nfin > 0) m = fmin(m, b.part[j].rho);
  const double rho = block_min(m, lds);
  double eta = 0.0, cnt = 0.0;
  for (int j = threadIdx.x; j < nwg; j += kBlock) {
    const WgPartial q = b.part[j];
    const double sc = (q.nfin > 0) ? exp(-(q.rho - rho) / p.lam_d) : 0.0;
    b.scale[j] = sc;
    eta += q.eta * sc;
    cnt += q.nfin;
  }
  eta = block_sum(eta, lds);
  cnt = block_sum(cnt, lds);
  if (threadIdx.x == 0) {
    b.stats->rho = rho;
    b.stats->eta = eta;
    b.stats->n_finite = (int32_t)cnt;
    b.stats->status = cnt > 0 ? MPPI_OK : MPPI_ENONFINITE;
    b.counters[0] = 0u;
  }
}

// ------------------------------------------------------------------ rollout
template <int DYN, bool JUMPS>
struct Draws {
  using Md = Model<DYN>;
  static constexpr int NN = JUMPS ? Md::M + Md::Q : Md::M;   // normals needed
  static constexpr int NW = JUMPS ? Md::COUNT_WORD + 1 : 2 * ((Md::M + 1) / 2);
  static constexpr int NB = (NW + 3) / 4;                     // Philox blocks
};

__device__ __forceinline__ void kahan_add(float& s, float& comp, float term) {
  const float y = term - comp;
  const float t = s + y;
  comp = (t - s) - y;
  s = t;
}

template <int DYN, bool JUMPS, bool DEBUG>
__global__ __launch_bounds__(256) void rollout_kernel(const DevParams p, const Buffers b,
                                                      const float* __restrict__ x0,
                                                      const float* __restrict__ U) {
  using Md = Model<DYN>;
  using D = Draws<DYN, JUMPS>;
  constexpr int N = Md::N, M = Md::M, Q = Md::Q;
  const int k = blockIdx.x * kBlock + threadIdx.x;
  const bool active = k < p.K;
  const uint32_t it = (uint32_t)b.stats->iteration;

  float x[N];
#pragma unroll
  for (int i = 0; i < N; ++i) x[i] = x0[i];
  bool crashed = Md::CAN_CRASH ? Md::crashed(x, p.mc) : false;
  float S = 0.f, comp = 0.f;

  for (int t = 0; t < p.T; ++t) {
    uint32_t w[4 * D::NB];
#pragma unroll
    for (int blk = 0; blk < D::NB; ++blk) {
      const Words4 r = philox4x32_10((uint32_t)t, (uint32_t)k, it, p.ctr3 | (uint32_t)blk,
                                     p.key0, p.key1);
      w[4 * blk + 0] = r.w0;
      w[4 * blk + 1] = r.w1;
      w[4 * blk + 2] = r.w2;
      w[4 * blk + 3] = r.w3;
    }
    float z[D::NN + 1];
#pragma unroll
    for (int i = 0; i < D::NN; i += 2) {
      if (i + 1 < D::NN)
        box_muller(w[i], w[i + 1], z[i], z[i + 1]);
      else
        z[i] = box_muller_cos(w[i], w[i + 1]);
    }
    float eps[M], gust[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < M; ++j) eps[j] = p.sigma[j] * z[j];
    int ncount = 0;
    if constexpr (JUMPS) {
      ncount = jump_count(w[Md::COUNT_WORD], p.th, p.n_th);
      if (ncount > 0) {
        float sq = 1.f;
        if (ncount > 1) sq = __builtin_amdgcn_sqrtf((float)ncount);
        if constexpr (Md::JUMP_IN_CONTROL) {
#pragma unroll
          for (int j = 0; j < M; ++j) eps[j] += p.sigJ[j] * sq * z[M + j];
        } else {
#pragma unroll
          for (int i = 0; i < Q; ++i) gust[i] = p.sigJ[i] * sq * z[M + i];
        }
      }
    }

    // modified path cost, eqs. (34)-(35), on the pre-step state
    float u[M];
#pragma unroll
    for (int j = 0; j < M; ++j) u[j] = U[t * M + j];
    float qx = 0.f;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const float d = x[i] - p.goal[i];
      qx += p.Q[i] * d * d;
    }
    if (Md::CAN_CRASH && crashed) qx += p.pen;
    float term;
    if (p.cost_form == MPPI_COST_IT) {
      float ctrl = 0.f, is = 0.f;
#pragma unroll
      for (int j = 0; j < M; ++j) {
        ctrl += p.halfR[j] * u[j] * u[j];
        is += (p.isc[j] * u[j] + p.isv[j] * eps[j]) * eps[j];
      }
      term = (qx + ctrl) * p.dt + is;
    } else {
      float ctrl = 0.f;
#pragma unroll
      for (int j = 0; j < M; ++j) {
        const float v = u[j] + eps[j];
        ctrl += p.halfR[j] * v * v;
      }
      term = (qx + ctrl) * p.dt;
    }
    kahan_add(S, comp, term);

    float v[M];
#pragma unroll
    for (int j = 0; j < M; ++j) v[j] = u[j] + eps[j];
    if (!crashed) {
      Md::step(x, v, gust, p.dt, p.mc);
      if (Md::CAN_CRASH) crashed = Md::crashed(x, p.mc);
    }

    if (active) {
#pragma unroll
      for (int j = 0; j < M; ++j) b.eps[(size_t)(t * M + j) * p.Ks + k] = eps[j];
      if constexpr (DEBUG) {
        const size_t kt = (size_t)k * p.T + t;
#pragma unroll
        for (int j = 0; j < M; ++j) b.dbg_zD[kt * M + j] = z[j];
        b.dbg_N[kt] = ncount;
        if constexpr (JUMPS) {
#pragma unroll
          for (int i = 0; i < Q; ++i) b.dbg_zJ[kt * Q + i] = z[M + i];
        } else {
#pragma unroll
          for (int i = 0; i < Q; ++i) b.dbg_zJ[kt * Q + i] = 0.f;
        }
      }
    }
  }
  float qf = 0.f;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const float d = x[i] - p.goal[i];
    qf += p.Qf[i] * d * d;
  }
  if (Md::CAN_CRASH && crashed) qf += p.pen;
  kahan_add(S, comp, qf);
  const double Sd = (double)S - (double)comp;
  if (active) b.S[k] = Sd;
  stats_epilogue(p, b, Sd, active);
}

// Statistics of caller-provided costs (mppi_jump_set of S).
__global__ __launch_bounds__(256) void restats_kernel(const DevParams p, const Buffers b) {
  const int k = blockIdx.x * kBlock + threadIdx.x;
  const bool active = k < p.K;
  const double Sd = active ? b.S[k] : 0.0;
  stats_epilogue(p, b, Sd, active);
}

// ------------------------------------------------------------------ update
constexpr int kRowsPerWg = 8;

__global__ __launch_bounds__(256) void update_kernel(const DevParams p, const Buffers b, int R,
                                                     int nch, int chunk) {
  __shared__ double lds[kWaves];
  __shared__ int is_last;
  const mppi_jump_stats st = *b.stats;
  const int r0 = blockIdx.x * kRowsPerWg;
  const int c = blockIdx.y;
  if (st.status == MPPI_OK) {
    double acc[kRowsPerWg];
#pragma unroll
    for (int rr = 0; rr < kRowsPerWg; ++rr) acc[rr] = 0.0;
    const int kend = min(p.K, (c + 1) * chunk);
    for (int k = c * chunk + threadIdx.x; k < kend; k += kBlock) {
      const double e = b.E[k] * b.scale[k >> 8];
#pragma unroll
      for (int rr = 0; rr < kRowsPerWg; ++rr)
        if (r0 + rr < R) acc[rr] += e * (double)b.eps[(size_t)(r0 + rr) * p.Ks + k];
    }
#pragma unroll
    for (int rr = 0; rr < kRowsPerWg; ++rr) {
      const double tot = block_sum(acc[rr], lds);
      if (threadIdx.x == 0 && r0 + rr < R) b.upart[(size_t)(r0 + rr) * nch + c] = tot;
    }
  }
  if (threadIdx.x == 0) {
    __threadfence();
    const uint32_t prev = atomicAdd(&b.counters[1], 1u);
    is_last = (prev == gridDim.x * gridDim.y - 1);
  }
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  if (st.status == MPPI_OK) {
    const double scale = (double)p.alpha / st.eta;
    for (int r = threadIdx.x; r < R; r += kBlock) {
      double d = 0.0;
      for (int cc = 0; cc < nch; ++cc) d += b.upart[(size_t)r * nch + cc];
      b.U[r] = (float)((double)b.U[r] + scale * d);
    }
  }
  if (threadIdx.x == 0) {
    b.stats->iteration = st.iteration + 1;
    b.counters[1] = 0u;
  }
}

// ------------------------------------------------------------------ misc
__global__ void init_kernel(Buffers b, const float* __restrict__ U0, int R, int m,
                            float4 u_init, uint64_t start_iteration) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < R) {
    const int j = r % m;
    const float ui = j == 0 ? u_init.x : j == 1 ? u_init.y : j == 2 ? u_init.z : u_init.w;
    b.U[r] = U0 ? U0[r] : ui;
  }
  if (r == 0) {
    b.stats->rho = 0.0;
    b.stats->eta = 0.0;
    b.stats->status = MPPI_OK;
    b.stats->n_finite = 0;
    b.stats->iteration = start_iteration;
    b.counters[0] = 0u;
    b.counters[1] = 0u;
  }
}

// One workgroup of 1024 threads; reads of a chunk finish before its writes.
__global__ __launch_bounds__(1024) void shift_kernel(float* __restrict__ U, int R, int m,
                                                     float4 u_init) {
  const int i = threadIdx.x;
  for (int base = 0; base < R; base += 1024) {
    const int r = base + i;
    float v = 0.f;
    if (r < R) {
      if (r + m < R) {
        v = U[r + m];
      } else {
        const int j = r - (R - m);
        v = j == 0 ? u_init.x : j == 1 ? u_init.y : j == 2 ? u_init.z : u_init.w;
      }
    }
    __syncthreads();
    if (r < R) U[r] = v;
    __syncthreads();
  }
}

template <int DYN>
__global__ void plant_kernel(const DevParams p, float* __restrict__ x,
                             const float* __restrict__ u, const float* __restrict__ d) {
  using Md = Model<DYN>;
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  float s[Md::N], v[Md::M];
  const float gust[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int i = 0; i < Md::N; ++i) s[i] = x[i];
#pragma unroll
  for (int j = 0; j < Md::M; ++j) v[j] = u[j] + d[j];
  Md::step(s, v, gust, p.dt, p.mc);
#pragma unroll
  for (int i = 0; i < Md::N; ++i) x[i] = s[i];
}

__global__ void weights_kernel(const DevParams p, const Buffers b, double* __restrict__ W) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= p.K) return;
  const mppi_jump_stats st = *b.stats;
  W[k] = st.status == MPPI_OK ? b.E[k] * b.scale[k >> 8] / st.eta : 0.0;
}

__global__ void philox_kernel(const uint32_t* __restrict__ ctr, uint32_t k0, uint32_t k1,
                              uint32_t* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Words4 r = philox4x32_10(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], k0, k1);
  out[4 * i] = r.w0;
  out[4 * i + 1] = r.w1;
  out[4 * i + 2] = r.w2;
  out[4 * i + 3] = r.w3;
}

}  // namespace mppi
