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

// Arrival counters: [0] rollout arrivals, [1] update arrivals, then one per
// block of kPartRows rows for the deferred update (partial_update_kernel).
constexpr int kCounters = 2;
constexpr int kPartRows = 64;
__host__ __device__ constexpr int counter_count(int R) {
  return kCounters + (R + kPartRows - 1) / kPartRows;
}

struct DevParams {
  int K, T, Ks, n_th;
  uint32_t k0;                // global index of sample 0 (Philox counter)
  int wg_shift;               // log2 of the samples per rollout workgroup
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
  // full Gaussian covariance (full = 1): Cholesky factor L, and Sigma^-1
  // scaled by lambda c (Pc) and lambda (c - 1) / 2 (Pv), row-major 4 x 4;
  // read from the kernel arguments (staging them in LDS with the other
  // constants costs the light models ~45 vector registers)
  int full;
  float L[16], Pc[16], Pv[16];
};

struct Buffers {
  float* U;           // [T][m]
  float* eps;         // [T][m][Ks]
  double* S;          // [K]
  double* E;          // [K] exp(-(S_k - rho_wg)/lambda)
  WgPartial* part;    // [ceil(K/256)]
  double* scale;      // [ceil(K/256)] exp(-(rho_wg - rho)/lambda)
  double* upart;      // [T*m][nch]   chunk partials of update_kernel, partial_update_kernel
  double* wpart;      // [nwg][T*m]   workgroup partials of the fused and deferred epilogues
  mppi_jump_stats* stats;
  uint32_t* counters; // [counter_count(T*m)] arrival counters
  float* dbg_zD;      // [K][T][m]
  int32_t* dbg_N;     // [K][T]
  float* dbg_zJ;      // [K][T][q]
};

// Receding-horizon shift folded into the last iteration of a control step:
// u0_out[0..m) <- U[0] (device memory; may be null), U[t] <- U[t+1],
// U[T-1] <- u_init (Algorithm 1), applied after the update by the last
// workgroup of the fused epilogue.
struct ShiftArgs {
  float* u0_out;
  int on;
  int m;
  float4 u_init;
};

// Per-sample-step constants of the rollout, staged in LDS at kernel start
// (by the first 16 threads of any workgroup of at least 64 threads).
// Read with wavefront-uniform addresses they land in vector registers, which
// keeps the scalar register file free for the Philox key schedule and the
// loop state (the 12-state model otherwise spills scalar registers).
struct Consts {
  float Q[12], goal[12];
  ModelConsts mc;
  float sigma[4], sigJ[4], isc[4], isv[4], halfR[4];
  uint32_t th[8];
};

__device__ __forceinline__ void stage_consts(Consts& cs, const DevParams& p) {
  const int i = threadIdx.x;
  if (i < 12) {
    cs.Q[i] = p.Q[i];
    cs.goal[i] = p.goal[i];
  }
  if (i < 16) cs.mc.c[i] = p.mc.c[i];
  if (i < 4) {
    cs.sigma[i] = p.sigma[i];
    cs.sigJ[i] = p.sigJ[i];
    cs.isc[i] = p.isc[i];
    cs.isv[i] = p.isv[i];
    cs.halfR[i] = p.halfR[i];
  }
  if (i < 8) cs.th[i] = p.th[i];
  __syncthreads();
}

// ------------------------------------------------------------------ epilogue
// Most workgroups whose partials one workgroup combines in the fused
// epilogue (the size of its rescale table in LDS).
constexpr int kFusedMaxWg = 512;
// A single controller's iteration fuses the update up to these counts and
// defers it beyond (partial_update_kernel): the last workgroup's combine
// grows with workgroups x rows, the deferred form costs a second launch.
// Measured (T=100, us per iteration, fused -> deferred): wave-specialised
// 128 workgroups 22.8 -> 28.1 (cartpole), 47.8 -> 52.2 (quadrotor); 256:
// 26.7 -> 32.1, 57.6 -> 58.7; 512: 46.4 -> 39.2, 107.7 -> 75.0.  One sample
// per lane (256 threads, narrower combine batches) 128 workgroups: 69.8 ->
// 69.1, 159.0 -> 131.1; 512: 135.2 -> 98.2, 338.6 -> 204.0.
// Batches take only controllers within these limits, so a batched
// iteration runs the same epilogue as the controller's own.
constexpr int kFusedWgWs = 256;
constexpr int kFusedWgLane = 64;
static_assert(kFusedWgWs <= kFusedMaxWg && kFusedWgLane <= kFusedMaxWg, "fused limits");
constexpr int kStageRows = 1024;  // partial rows staged in LDS per pass

// Device-scope fences of the last-arrival pattern: the publishing side needs
// only release (its stores before its arrival increment), the last arrival
// only acquire (the others' stores before its loads).  A full fence would
// add the other half: an L2 invalidate on the publishing side, a write-back
// of this XCD's L2 on the combining side.
__device__ __forceinline__ void release_fence() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
__device__ __forceinline__ void acquire_fence() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

// Phase timestamps, compiled only into the phase-profiling build of the
// library (MPPI_PHASE_STAMPS defined): thread 0 of every workgroup of the
// wave-specialised rollout records the 100 MHz real-time counter at the
// phase boundaries of one iteration, in the record of launch (iteration
// mod kPhaseLaunches).  Slots: 0 workgroup start, 1 rollout done (costs
// known), 2 partials stored, 3 arrival counted, 4 combine done and 5
// epilogue done (the last workgroup only), 6 one for the last workgroup,
// else zero, 7 the consumer's first chunk ready, 8 acquire done (the last
// workgroup).  The batched grid launch also records each tile's start and
// end.
#ifdef MPPI_PHASE_STAMPS
constexpr int kPhaseSlots = 16, kPhaseLaunches = 8, kPhaseMaxWg = 256;
__device__ unsigned long long g_phase[kPhaseLaunches * kPhaseMaxWg * kPhaseSlots];
__device__ __forceinline__ void phase_mark(uint64_t it, int wg, int nwg, int slot,
                                           unsigned long long v) {
  if (threadIdx.x == 0 && wg < kPhaseMaxWg && nwg <= kPhaseMaxWg)
    g_phase[((it % kPhaseLaunches) * kPhaseMaxWg + wg) * kPhaseSlots + slot] = v;
}
#define MPPI_PHASE(it, wg, nwg, slot) \
  phase_mark((it), (wg), (nwg), (slot), __builtin_amdgcn_s_memrealtime())
#define MPPI_PHASE_VALUE(it, wg, nwg, slot, v) phase_mark((it), (wg), (nwg), (slot), (v))
// Batched form: start and end of every tile of the last launch (thread 0).
constexpr int kPhaseTiles = 8192;
__device__ unsigned long long g_phase_tiles[kPhaseTiles * 2];
#define MPPI_TILE_MARK(tile, slot)                          \
  do {                                                      \
    if (threadIdx.x == 0 && (tile) < kPhaseTiles)           \
      g_phase_tiles[(tile) * 2 + (slot)] = __builtin_amdgcn_s_memrealtime(); \
  } while (0)
#else
#define MPPI_TILE_MARK(tile, slot) ((void)0)
#define MPPI_PHASE(it, wg, nwg, slot) ((void)0)
#define MPPI_PHASE_VALUE(it, wg, nwg, slot, v) ((void)0)
#endif

// Rollout epilogue, in three parts that the one-iteration kernels chain with
// a last-arrival hand-off and the multi-iteration kernel with a grid-wide
// wait:
//   * publish: statistics of eq. (37) over the SPW samples of this
//     workgroup (threads below SPW hold a cost; the others pass active =
//     false): rho_wg = min of the finite S_k, E_k = exp(-(S_k - rho_wg)/
//     lambda), eta_wg = sum E_k, count of finite S_k; FUSED: the weighted
//     perturbation sums P[r][wg] = sum_k E_k eps[r][k] over the workgroup's
//     own eps tile.  Every global partial is stored by wavefront 0, so that
//     the single device-scope release fence that wavefront issues next
//     covers them all (a device-scope release writes back the L2 of this
//     XCD, so one per workgroup instead of one per wavefront).
//   * combine: the partials in index order with the rescale
//     exp(-(rho_wg - rho)/lambda), and, when FUSED,
//     U[r] += alpha * sum_wg scale_wg P[r][wg] / eta (eqs. (36) / (49)).
//   * the receding-horizon shift and the statistics record.
// tile / tstride (FUSED): the workgroup's perturbations, row r (= t m + j)
// of its SPW samples at tile[r tstride ..] (on chip, or its columns of the
// HBM array).  part / wpart: where this workgroup's partials go (row r of
// workgroup wg at wpart[wg R + r]).
// RB (256-sample workgroups): 0, the tile sums as described below; else
// each wavefront takes every fourth row, each lane the four consecutive
// samples 4 lane .. 4 lane + 3 with their weights held in registers, RB rows
// in flight at once (one float4 load per lane and row), each row's 64 lane
// sums added by a wavefront reduction (the order of a row's terms does not
// depend on RB).  The one-sample-per-lane kernels use it: their tiles come
// back from L2 or, in the deferred-update form, from HBM, and the quarter
// layout's loads (two in flight, each with four fp64 weights) leave that
// latency bound.  The wave-specialised kernels' 64-sample tiles keep the
// quarter layout.
template <int SPW, bool FUSED, int NT, int RB = 0>
__device__ __forceinline__ void epilogue_publish(const DevParams& p, const Buffers& b, double Sd,
                                                 bool active, int R, int wg, const float* tile,
                                                 int tstride, WgPartial* part, double* wpart) {
  constexpr int NW = NT / 64;
  constexpr int RPP = NT / 4;  // eps tile rows per pass, four threads per row
  __shared__ double lds[NW];
  __shared__ double e_lds[SPW];
  __shared__ double stage[FUSED ? kStageRows : 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool fin = active && isfinite(Sd);
  const int k0 = wg * SPW;
  // statistics of the workgroup; wavefront 0 ends up holding them
  double rho_wg = INFINITY, eta_wg = 0.0, nfin = 0.0;
  if constexpr (SPW == 64) {
    // the costs live in wavefront 0: wavefront reductions, no barriers
    if (wave == 0) {
      rho_wg = wave_min(fin ? Sd : INFINITY);
      const double e = fin ? exp(-(Sd - rho_wg) / p.lam_d) : 0.0;
      if (active) b.E[k0 + lane] = e;
      e_lds[lane] = e;
      eta_wg = wave_sum(e);
      nfin = (double)__popcll(__ballot(fin));
    }
    __syncthreads();  // e_lds
  } else {
    rho_wg = block_min<NW>(fin ? Sd : INFINITY, lds);
    const double e = fin ? exp(-(Sd - rho_wg) / p.lam_d) : 0.0;
    if (active) b.E[k0 + threadIdx.x] = e;
    if (threadIdx.x < SPW) e_lds[threadIdx.x] = e;
    eta_wg = block_sum<NW>(e, lds);
    nfin = block_sum<NW>(fin ? 1.0 : 0.0, lds);  // its barriers publish e_lds
  }
  if constexpr (FUSED && RB > 0) {
    static_assert(SPW == 256 && NT == 256, "four samples per lane, four wavefronts");
    double w4[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) w4[i] = e_lds[4 * lane + i];
    for (int base = 0; base < R; base += kStageRows) {
      const int nrow = min(kStageRows, R - base);
      for (int i0 = wave; i0 < nrow; i0 += 4 * RB) {
        float4 v[RB];
#pragma unroll
        for (int j = 0; j < RB; ++j) {
          const int i = min(i0 + 4 * j, nrow - 1);  // rows past the block: its last, unused
          v[j] = reinterpret_cast<const float4*>(tile + (size_t)(base + i) * tstride)[lane];
        }
#pragma unroll
        for (int j = 0; j < RB; ++j) {
          double a = w4[0] * (double)v[j].x;
          a += w4[1] * (double)v[j].y;
          a += w4[2] * (double)v[j].z;
          a += w4[3] * (double)v[j].w;
          a = wave_sum(a);
          if (lane == 0 && i0 + 4 * j < nrow) stage[i0 + 4 * j] = a;
        }
      }
      __syncthreads();
      if (wave == 0)
        for (int i = lane; i < nrow; i += 64) wpart[(size_t)wg * R + base + i] = stage[i];
      __syncthreads();
    }
  } else if constexpr (FUSED) {
    // the workgroup's own eps tile (written earlier in this kernel by its
    // threads, visible after the barriers above): row r is reduced by four
    // consecutive threads over a quarter of the samples each, in sample
    // order, the quarters added as (q0 + q1) + (q2 + q3); the row sums are
    // staged in LDS and stored by wavefront 0
    constexpr int SQ = SPW / 4;  // samples per thread
    const int q = threadIdx.x & 3, i4 = threadIdx.x >> 2;
    for (int base = 0; base < R; base += kStageRows) {
      const int nrow = min(kStageRows, R - base);
      for (int i0 = 0; i0 < nrow; i0 += RPP) {
        const int i = i0 + i4;
        double acc = 0.0;
        if (i < nrow) {
          const float4* row =
              reinterpret_cast<const float4*>(tile + (size_t)(base + i) * tstride + q * SQ);
          const double* ew = e_lds + q * SQ;
#pragma unroll 2
          for (int j = 0; j < SQ / 4; ++j) {
            const float4 v = row[j];
            acc += ew[4 * j] * (double)v.x;
            acc += ew[4 * j + 1] * (double)v.y;
            acc += ew[4 * j + 2] * (double)v.z;
            acc += ew[4 * j + 3] * (double)v.w;
          }
        }
        acc += dpp_f64<kDppXor1>(acc);
        acc += dpp_f64<kDppXor2>(acc);
        if (q == 0 && i < nrow) stage[i] = acc;
      }
      __syncthreads();
      if (wave == 0)
        for (int i = lane; i < nrow; i += 64) wpart[(size_t)wg * R + base + i] = stage[i];
      __syncthreads();
    }
  }
  if (wave == 0 && lane == 0) {
    part[wg].rho = rho_wg;
    part[wg].eta = eta_wg;
    part[wg].nfin = (int32_t)nfin;
  }
}

// Combination of n partials (every thread of the workgroup takes part; the
// partials are visible to it).  Returns (rho, eta, count of finite S_k) to
// every thread.  FUSED: Uout[r] = Uin[r] + alpha / eta * sum_j scale_j
// P[r][j] for every row (unchanged when no S_k is finite); Uin and Uout may
// be the same array (global or LDS).  scale (may be null): the rescales
// exp(-(rho_j - rho)/lambda) are stored there too.
struct Combined {
  double rho, eta, cnt;
};

template <bool FUSED, int NT>
__device__ __forceinline__ Combined epilogue_combine(const DevParams& p, const WgPartial* parts,
                                                     const double* rows, int n, int R,
                                                     const float* Uin, float* Uout,
                                                     double* scale) {
  constexpr int NW = NT / 64;
  __shared__ double lds[NW];
  __shared__ double sc_lds[FUSED ? kFusedMaxWg : 1];
  __shared__ double seg_lds[FUSED ? NT : 1];
  __shared__ double bc[3];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;

  // First pass of the fused update (rows [0, Rp)): when there are threads
  // to spare, each row's partials are split into S contiguous segments, one
  // thread each.  The segment's first kPre partials and the row's U are
  // loaded now, so that their latency overlaps the statistics below.
  constexpr int kPre = 16;
  int Rp = 1, S = 1, L = 0, seg = 0, rr = 0, j0 = 0, j1 = 0;
  double wpre[kPre];
  float uold = 0.f;
  if constexpr (FUSED) {
    Rp = min(NT, R);
    S = max(1, min(NT / Rp, (n + kPre - 1) / kPre));
    L = (n + S - 1) / S;
    seg = threadIdx.x / Rp;
    rr = threadIdx.x - seg * Rp;
    j0 = seg < S ? seg * L : 0;
    j1 = seg < S ? min(n, j0 + L) : 0;
    const double* wr = rows + rr;
#pragma unroll
    for (int q = 0; q < kPre; ++q) wpre[q] = j0 + q < j1 ? wr[(size_t)(j0 + q) * R] : 0.0;
    if (seg == 0) uold = Uin[rr];
  }
  // combination: rho = min of the partial minima, the rescales
  // exp(-(rho_j - rho)/lambda), eta and the finite count.  Up to 64
  // partials: wavefront 0 alone, one per lane held in registers; more: the
  // whole workgroup with block reductions.
  if (n <= 64) {
    if (wave == 0) {
      const bool h = lane < n;
      const double hrho = h ? parts[lane].rho : INFINITY;
      const double heta = h ? parts[lane].eta : 0.0;
      const int hfin = h ? parts[lane].nfin : 0;
      const double rho = wave_min(hfin > 0 ? hrho : INFINITY);
      double eta = 0.0, cnt = 0.0;
      if (h) {
        const double sc = hfin > 0 ? exp(-(hrho - rho) / p.lam_d) : 0.0;
        if (scale != nullptr) scale[lane] = sc;
        if constexpr (FUSED) sc_lds[lane] = sc;
        eta = heta * sc;
        cnt = hfin;
      }
      eta = wave_sum(eta);
      cnt = wave_sum(cnt);
      if (lane == 0) {
        bc[0] = rho;
        bc[1] = eta;
        bc[2] = cnt;
      }
    }
  } else {
    // a thread's first partial stays in registers across both passes, loaded
    // whole and unconditionally (one memory round trip, not a dependent load
    // per field); further ones (unfused statistics of very large K) reload
    WgPartial q0{INFINITY, 0.0, 0};
    if (threadIdx.x < n) q0 = parts[threadIdx.x];
    double m = q0.nfin > 0 ? q0.rho : INFINITY;
    // four partials' minima in flight at once (many partials: one memory
    // round trip per four instead of one each)
#pragma unroll 4
    for (int j = threadIdx.x + NT; j < n; j += NT) {
      const double rj = parts[j].rho;
      const int fj = parts[j].nfin;
      m = fj > 0 ? fmin(m, rj) : m;
    }
    const double rho = block_min<NW>(m, lds);
    double eta = 0.0, cnt = 0.0;
    // the next partial is loaded while this one's rescale is formed
    WgPartial qn = q0;
    for (int j = threadIdx.x; j < n; j += NT) {
      const WgPartial q = qn;
      if (j + NT < n) qn = parts[j + NT];
      const double sc = (q.nfin > 0) ? exp(-(q.rho - rho) / p.lam_d) : 0.0;
      if (scale != nullptr) scale[j] = sc;
      if constexpr (FUSED) sc_lds[j] = sc;
      eta += q.eta * sc;
      cnt += q.nfin;
    }
    eta = block_sum<NW>(eta, lds);
    cnt = block_sum<NW>(cnt, lds);
    if (threadIdx.x == 0) {
      bc[0] = rho;
      bc[1] = eta;
      bc[2] = cnt;
    }
  }
  __syncthreads();  // bc and sc_lds
  const Combined out{bc[0], bc[1], bc[2]};
  if constexpr (FUSED) {
    // U[r] += alpha / eta * sum_j scale_j P[r][j]: each segment is summed
    // with four accumulators in a fixed pattern, the segment sums in segment
    // order
    if (out.cnt > 0) {
      const double f = (double)p.alpha / out.eta;
      for (int base = 0; base < R; base += NT) {
        const bool first = base == 0;
        if (!first) {
          Rp = min(NT, R - base);
          S = max(1, min(NT / Rp, (n + kPre - 1) / kPre));
          L = (n + S - 1) / S;
          seg = threadIdx.x / Rp;
          rr = threadIdx.x - seg * Rp;
          j0 = seg < S ? seg * L : 0;
          j1 = seg < S ? min(n, j0 + L) : 0;
        }
        double acc = 0.0;
        if (seg < S) {
          const double* wr = rows + base + rr;  // partial j of the row at wr[j R]
          double d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;
          int j = j0;
          if (first) {
            // the preloaded groups of four (kPre is a multiple of four)
#pragma unroll
            for (int q = 0; q < kPre; q += 4) {
              if (j + 4 <= j1) {
                d0 += sc_lds[j] * wpre[q];
                d1 += sc_lds[j + 1] * wpre[q + 1];
                d2 += sc_lds[j + 2] * wpre[q + 2];
                d3 += sc_lds[j + 3] * wpre[q + 3];
                j += 4;
              }
            }
            if (j1 - j0 < kPre) {
              // the segment's tail is preloaded too (constant register
              // indices: the q loop is unrolled)
              const int jt = j;
#pragma unroll
              for (int q = 0; q < kPre; ++q)
                if (j0 + q >= jt && j0 + q < j1) d0 += sc_lds[j0 + q] * wpre[q];
              j = j1;
            }
          }
          // the rest in batches of kBatch loads issued together (one memory
          // round trip each), accumulated in the same pattern as below; only
          // in the eight-wave workgroups, which have the registers to spare
          // (the 256-thread kernels would lose occupancy)
          constexpr int kBatch = NT >= 512 ? 32 : 4;
          for (; NT >= 512 && j + kBatch <= j1; j += kBatch) {
            double w[kBatch];
#pragma unroll
            for (int q = 0; q < kBatch; ++q) w[q] = wr[(size_t)(j + q) * R];
#pragma unroll
            for (int q = 0; q < kBatch; q += 4) {
              d0 += sc_lds[j + q] * w[q];
              d1 += sc_lds[j + q + 1] * w[q + 1];
              d2 += sc_lds[j + q + 2] * w[q + 2];
              d3 += sc_lds[j + q + 3] * w[q + 3];
            }
          }
#pragma unroll 4
          for (; j + 4 <= j1; j += 4) {
            d0 += sc_lds[j] * wr[(size_t)j * R];
            d1 += sc_lds[j + 1] * wr[(size_t)(j + 1) * R];
            d2 += sc_lds[j + 2] * wr[(size_t)(j + 2) * R];
            d3 += sc_lds[j + 3] * wr[(size_t)(j + 3) * R];
          }
          for (; j < j1; ++j) d0 += sc_lds[j] * wr[(size_t)j * R];
          acc = (d0 + d1) + (d2 + d3);
        }
        if (S > 1) {
          seg_lds[threadIdx.x] = acc;
          __syncthreads();
          if (seg == 0)
            for (int s2 = 1; s2 < S; ++s2) acc += seg_lds[s2 * Rp + rr];
        }
        if (seg == 0) {
          const float uo = first ? uold : Uin[base + rr];
          Uout[base + rr] = (float)((double)uo + f * acc);
        }
        if (S > 1) __syncthreads();
      }
    }
  }
  return out;
}

// Receding-horizon shift of U (R floats, m per step) by the whole
// workgroup, after its update is visible to the workgroup: u0_out[0..m) <-
// U[0] (may be null), U[t] <- U[t+1], U[T-1] <- u_init.  Uin and Uout may be
// the same array.
template <int NT>
__device__ __forceinline__ void epilogue_shift(const ShiftArgs& sh, const float* Uin, float* Uout,
                                               int R) {
  const int m = sh.m;
  if (sh.u0_out != nullptr && threadIdx.x < m) sh.u0_out[threadIdx.x] = Uin[threadIdx.x];
  for (int base = 0; base < R; base += NT) {
    const int r = base + threadIdx.x;
    float v = 0.f;
    if (r < R) {
      if (r + m < R) {
        v = Uin[r + m];
      } else {
        const int j = r - (R - m);
        v = j == 0 ? sh.u_init.x : j == 1 ? sh.u_init.y : j == 2 ? sh.u_init.z : sh.u_init.w;
      }
    }
    __syncthreads();
    if (r < R) Uout[r] = v;
    __syncthreads();
  }
}

__device__ __forceinline__ void record_stats(const Buffers& b, const Combined& c,
                                             uint64_t iteration, bool advance) {
  b.stats->rho = c.rho;
  b.stats->eta = c.eta;
  b.stats->n_finite = (int32_t)c.cnt;
  b.stats->status = c.cnt > 0 ? MPPI_OK : MPPI_ENONFINITE;
  if (advance) b.stats->iteration = iteration;
}

// The one-iteration epilogue: publish, then the last workgroup to arrive
// combines, applies the update (FUSED) and, when sh.on, the shift, records
// the statistics and advances the iteration counter (FUSED).
// DEFER (with FUSED): the weighted tile sums are published as in the fused
// form, but the last workgroup forms only the statistics and the rescales
// (stored to b.scale); partial_update_kernel then applies the update.  For
// rollouts with too many workgroups for one workgroup to combine.
// wg / nwg: this workgroup's index among the nwg workgroups of its controller.
template <int SPW, bool FUSED, int NT = kBlock, bool DEFER = false, int RB = 8>
__device__ __forceinline__ void rollout_epilogue(const DevParams& p, const Buffers& b, double Sd,
                                                 bool active, int R, const ShiftArgs sh, int wg,
                                                 int nwg, const float* tile, int tstride) {
  __shared__ int is_last;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#ifdef MPPI_PHASE_STAMPS
  const uint64_t it = b.stats->iteration;
#endif
  MPPI_PHASE(it, wg, nwg, 1);
  epilogue_publish<SPW, FUSED, NT, SPW == 256 ? RB : 0>(p, b, Sd, active, R, wg, tile, tstride,
                                                        b.part, b.wpart);
  MPPI_PHASE(it, wg, nwg, 2);
  if (wave == 0) {
    release_fence();
    if (lane == 0) {
      const uint32_t prev = atomicAdd(&b.counters[0], 1u);
      is_last = (prev == (uint32_t)nwg - 1);
    }
  }
  __syncthreads();
  MPPI_PHASE(it, wg, nwg, 3);
  MPPI_PHASE_VALUE(it, wg, nwg, 6, is_last ? 1ull : 0ull);
  if (!is_last) return;
  acquire_fence();
  MPPI_PHASE(it, wg, nwg, 8);
  constexpr bool UPDATE = FUSED && !DEFER;
  const Combined c = epilogue_combine<UPDATE, NT>(p, b.part, b.wpart, nwg, R, b.U, b.U, b.scale);
  MPPI_PHASE(it, wg, nwg, 4);
  if constexpr (UPDATE) {
    if (sh.on) {
      __syncthreads();  // the updated rows are visible to the whole block
      epilogue_shift<NT>(sh, b.U, b.U, R);
    }
  }
  MPPI_PHASE(it, wg, nwg, 5);
  if (threadIdx.x == 0) {
    record_stats(b, c, b.stats->iteration + 1, UPDATE);
    b.counters[0] = 0u;
  }
}

// ------------------------------------------------------------------ rollout
// Draws of one (sample, step): standard normals, the control perturbation
// eps (plus the jump when it enters through the control channel), the
// body-force disturbance (when it does not), and the jump count.  Branch
// free: sqrt(0) = 0 removes a zero count's jump.
template <int DYN, bool JUMPS>
struct Noise {
  using Md = Model<DYN>;
  static constexpr int NN = JUMPS ? Md::M + Md::Q : Md::M;   // normals needed
  static constexpr int NW = !JUMPS               ? 2 * ((Md::M + 1) / 2)
                            : Md::COUNT_WORD < 0 ? 2 * ((Md::M + Md::Q + 1) / 2)
                                                 : Md::COUNT_WORD + 1;
  static constexpr int NB = (NW + 3) / 4;                     // Philox blocks
  float z[NN + 1];
  float eps[Md::M];
  float gust[3];
  int n;
};

// FULL: the Gaussian part is L z for a full covariance L L^T (multi-channel
// models only; the factor is read from the kernel arguments).
template <int DYN, bool JUMPS, bool FULL = false>
__device__ __forceinline__ void draw_noise(Noise<DYN, JUMPS>& o, const DevParams& p,
                                           const Consts& cs, uint32_t t, uint32_t k, uint32_t it) {
  using Md = Model<DYN>;
  using Nz = Noise<DYN, JUMPS>;
  uint32_t w[4 * Nz::NB];
#pragma unroll
  for (int blk = 0; blk < Nz::NB; ++blk) {
    const Words4 r = philox4x32_10(t, k, it, p.ctr3 | (uint32_t)blk, p.key0, p.key1);
    w[4 * blk + 0] = r.w0;
    w[4 * blk + 1] = r.w1;
    w[4 * blk + 2] = r.w2;
    w[4 * blk + 3] = r.w3;
  }
#pragma unroll
  for (int i = 0; i < Nz::NN; i += 2) {
    if (i + 1 < Nz::NN)
      box_muller(w[i], w[i + 1], o.z[i], o.z[i + 1]);
    else
      o.z[i] = box_muller_cos(w[i], w[i + 1]);
  }
  // (one-channel models: the host passes a full covariance as sigma = L00)
  if constexpr (FULL) {
    // eps_D = L z (lower-triangular factor of the covariance)
#pragma unroll
    for (int j = 0; j < Md::M; ++j) {
      float e = 0.f;
#pragma unroll
      for (int k = 0; k <= j; ++k) e += p.L[4 * j + k] * o.z[k];
      o.eps[j] = e;
    }
  } else {
#pragma unroll
    for (int j = 0; j < Md::M; ++j) o.eps[j] = cs.sigma[j] * o.z[j];
  }
  o.gust[0] = o.gust[1] = o.gust[2] = 0.f;
  o.n = 0;
  if constexpr (JUMPS) {
    // count word: the word after the last Box-Muller pair, or, when the
    // pairs fill whole blocks (COUNT_WORD < 0), the low bytes of words 0-3,
    // which Box-Muller does not use (it takes the top 24 bits of a word)
    uint32_t wc;
    if constexpr (Md::COUNT_WORD < 0)
      wc = (w[0] & 255u) | (w[1] & 255u) << 8 | (w[2] & 255u) << 16 | w[3] << 24;
    else
      wc = w[Md::COUNT_WORD];
    o.n = jump_count(wc, cs.th, p.th, p.n_th);
    const float sq = __builtin_amdgcn_sqrtf((float)o.n);
    if constexpr (Md::JUMP_IN_CONTROL) {
#pragma unroll
      for (int j = 0; j < Md::M; ++j) o.eps[j] += cs.sigJ[j] * sq * o.z[Md::M + j];
    } else {
#pragma unroll
      for (int i = 0; i < Md::Q; ++i) o.gust[i] = cs.sigJ[i] * sq * o.z[Md::M + i];
    }
  }
}

// Path-cost accumulation: the stage costs of each block of kCostBlock time
// steps (t = 16 c .. 16 c + 15) are summed in fp32 and the block sums in
// fp64, so the fp32 sum holds at most 16 terms.  Its rounding (~16 ulps of
// the block's term magnitudes) stays below the fp32 trajectory error that
// bounds S~ anyway (an fp32 emulation gives the same maximum error with
// compensated, blocked or plain summation); the consumer wave of the
// wave-specialised schedule, which runs the serial recursion, then spends
// one add per step on the sum instead of four.  Both schedules block the
// same steps, so their costs agree bitwise.
constexpr int kCostBlock = 16;

struct CostSum {
  float blk = 0.f;   // sum of the current block's stage costs
  double S = 0.0;    // sum of the completed blocks
  __device__ __forceinline__ void add(float term) { blk += term; }
  __device__ __forceinline__ void close_block() {
    S += (double)blk;
    blk = 0.f;
  }
};

// State-free part of the stage cost of eqs. (34)-(35): nominal control cost
// times dt plus the importance-sampling terms (IT form), or the control cost
// of the applied control times dt (SO form).
template <int M, int FORM, bool FULL = false>
__device__ __forceinline__ float state_free_cost(const DevParams& p, const Consts& cs,
                                                 const float* u, const float* eps) {
  if constexpr (FORM == MPPI_COST_IT) {
    float ctrl = 0.f, is = 0.f;
    if constexpr (FULL) {
      // lambda c u^T Sigma^-1 eps + lambda (c - 1) / 2 eps^T Sigma^-1 eps
#pragma unroll
      for (int j = 0; j < M; ++j) {
        ctrl += cs.halfR[j] * u[j] * u[j];
        float a = 0.f;
#pragma unroll
        for (int k = 0; k < M; ++k) a += p.Pc[4 * j + k] * u[k] + p.Pv[4 * j + k] * eps[k];
        is += a * eps[j];
      }
    } else {
#pragma unroll
      for (int j = 0; j < M; ++j) {
        ctrl += cs.halfR[j] * u[j] * u[j];
        is += (cs.isc[j] * u[j] + cs.isv[j] * eps[j]) * eps[j];
      }
    }
    return ctrl * p.dt + is;
  } else {
    float ctrl = 0.f;
#pragma unroll
    for (int j = 0; j < M; ++j) {
      const float v = u[j] + eps[j];
      ctrl += cs.halfR[j] * v * v;
    }
    return ctrl * p.dt;
  }
}

// FORM: MPPI_COST_IT or MPPI_COST_SO.  FUSED: the epilogue also applies the
// update (one kernel per iteration); otherwise it only forms the statistics
// and update_kernel follows.
// One workgroup (tile wg of nwg) of the one-sample-per-lane rollout.  U is
// not restrict-qualified: in the fused form the last workgroup writes the
// same array (through b.U) while the kernel runs.  DEFER: the epilogue's
// deferred-update form (rollout_epilogue).
template <int DYN, bool JUMPS, bool DEBUG, int FORM, bool FUSED, bool FULL = false,
          bool DEFER = false>
__device__ __forceinline__ void rollout_lane_tile(const DevParams& p, const Buffers& b,
                                                  const float* __restrict__ x0,
                                                  const float* U, int R,
                                                  const ShiftArgs& sh, int wg, int nwg) {
  using Md = Model<DYN>;
  constexpr int N = Md::N, M = Md::M, Q = Md::Q;
  const int k = wg * kBlock + threadIdx.x;
  const bool active = k < p.K;
  const uint32_t it = (uint32_t)b.stats->iteration;
  __shared__ Consts cs;
  stage_consts(cs, p);

  float x[N];
#pragma unroll
  for (int i = 0; i < N; ++i) x[i] = x0[i];
  bool crashed = Md::CAN_CRASH ? Md::crashed(x, cs.mc) : false;
  CostSum S;

  // software pipeline: the draws of step t + 1 are formed while step t's
  // dynamics run (they do not depend on the state); the last step draws
  // nothing ahead
  Noise<DYN, JUMPS> nxt;
  draw_noise<DYN, JUMPS, FULL>(nxt, p, cs, 0u, p.k0 + (uint32_t)k, it);
  for (int t = 0; t < p.T; ++t) {
    const Noise<DYN, JUMPS> cur = nxt;
    if (t + 1 < p.T)
      draw_noise<DYN, JUMPS, FULL>(nxt, p, cs, (uint32_t)(t + 1), p.k0 + (uint32_t)k, it);

    // modified path cost, eqs. (34)-(35), on the pre-step state
    float u[M];
#pragma unroll
    for (int j = 0; j < M; ++j) u[j] = U[t * M + j];
    float qx = 0.f;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const float d = x[i] - cs.goal[i];
      qx += cs.Q[i] * d * d;
    }
    if constexpr (Md::CAN_CRASH) qx += crashed ? p.pen : 0.f;
    const float term = qx * p.dt + state_free_cost<M, FORM, FULL>(p, cs, u, cur.eps);
    S.add(term);
    if ((t & (kCostBlock - 1)) == kCostBlock - 1 || t == p.T - 1) S.close_block();

    float v[M];
#pragma unroll
    for (int j = 0; j < M; ++j) v[j] = u[j] + cur.eps[j];
    if constexpr (Md::CAN_CRASH) {
      float xn[N];
#pragma unroll
      for (int i = 0; i < N; ++i) xn[i] = x[i];
      Md::step(xn, v, cur.gust, p.dt, cs.mc);
#pragma unroll
      for (int i = 0; i < N; ++i) x[i] = crashed ? x[i] : xn[i];
      crashed = crashed || Md::crashed(x, cs.mc);
    } else {
      Md::step(x, v, cur.gust, p.dt, cs.mc);
    }

    // every lane of the grid stores (rows are padded to whole workgroups);
    // lanes past K carry zero weight
#pragma unroll
    for (int j = 0; j < M; ++j) b.eps[(size_t)(t * M + j) * p.Ks + k] = cur.eps[j];
    if constexpr (DEBUG) {
      if (active) {
        const size_t kt = (size_t)k * p.T + t;
#pragma unroll
        for (int j = 0; j < M; ++j) b.dbg_zD[kt * M + j] = cur.z[j];
        b.dbg_N[kt] = cur.n;
#pragma unroll
        for (int i = 0; i < Q; ++i) b.dbg_zJ[kt * Q + i] = JUMPS ? cur.z[M + i] : 0.f;
      }
    }
  }
  float qf = 0.f;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const float d = x[i] - cs.goal[i];
    qf += p.Qf[i] * d * d;
  }
  if constexpr (Md::CAN_CRASH) qf += crashed ? p.pen : 0.f;
  const double Sd = S.S + (double)qf;
  if (active) b.S[k] = Sd;
  // rows of the epilogue's tile sums in flight per wavefront: four keep
  // the one-channel deferred kernels at their rollout's 68 registers (eight
  // take 88 and cost occupancy: cartpole K=2^20, T=100 0.517 -> 0.532 ms
  // per iteration); the 12-state model's rollout holds 120, which sixteen
  // rows reuse
  constexpr int RB = M > 1 ? 16 : 4;
  rollout_epilogue<kBlock, FUSED, kBlock, DEFER, RB>(p, b, Sd, active, R, sh, wg, nwg,
                                                     b.eps + (size_t)wg * kBlock, p.Ks);
}

template <int DYN, bool JUMPS, bool DEBUG, int FORM, bool FUSED, bool FULL, bool DEFER = false>
__global__ __launch_bounds__(256) void rollout_kernel(const DevParams p, const Buffers b,
                                                      const float* __restrict__ x0,
                                                      const float* U, int R,
                                                      const ShiftArgs sh) {
  rollout_lane_tile<DYN, JUMPS, DEBUG, FORM, FUSED, FULL, DEFER>(p, b, x0, U, R, sh, blockIdx.x,
                                                                gridDim.x);
}

// Statistics of caller-provided costs (mppi_jump_set of S), with the
// workgroup size of the context's rollout schedule.
template <int SPW>
__global__ __launch_bounds__(256) void restats_kernel(const DevParams p, const Buffers b) {
  const int k = blockIdx.x * SPW + threadIdx.x;
  const bool active = threadIdx.x < SPW && k < p.K;
  const double Sd = active ? b.S[k] : 0.0;
  rollout_epilogue<SPW, false>(p, b, Sd, active, 0, ShiftArgs{}, blockIdx.x, gridDim.x, nullptr,
                               0);
}

// ------------------------------------------------------------------ update
// A workgroup takes kRowsPerWg rows of eps over one chunk of samples; each
// thread four consecutive samples at a time (one 16-byte load per row and
// the four weights), so that every row's stream and the weights are read
// with wide coalesced loads and many bytes are in flight per thread.  The
// weights are read once per row block: more rows per workgroup read them
// fewer times.  Per thread the terms of a row are added in sample order;
// the block sum and the chunk order then fix the rest of the order.
constexpr int kRowsPerWg = 16;

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
    // k is a multiple of four below K <= Ks (a multiple of 256), so the four
    // eps entries stay inside the padded row; weights past K are zero
    // (branch free, so that all the step's loads are issued together: rows
    // past R read row R - 1 and are never stored, indices past the chunk
    // read its last sample with zero weight)
    // The next step's loads are issued before this step's sums.
    auto load = [&](int k, double* e, float4* v) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int kq = min(k + q, kend - 1);
        const double w = b.E[kq] * b.scale[kq >> p.wg_shift];
        e[q] = k + q < kend ? w : 0.0;
      }
#pragma unroll
      for (int rr = 0; rr < kRowsPerWg; ++rr)
        v[rr] = *reinterpret_cast<const float4*>(b.eps + (size_t)min(r0 + rr, R - 1) * p.Ks + k);
    };
    int k = c * chunk + 4 * threadIdx.x;
    double e[4];
    float4 v[kRowsPerWg];
    if (k < kend) load(k, e, v);
    for (; k < kend; k += 4 * kBlock) {
      double en[4];
      float4 vn[kRowsPerWg];
      const int kn = k + 4 * kBlock;
      if (kn < kend) load(kn, en, vn);
#pragma unroll
      for (int rr = 0; rr < kRowsPerWg; ++rr) {
        acc[rr] += e[0] * (double)v[rr].x;
        acc[rr] += e[1] * (double)v[rr].y;
        acc[rr] += e[2] * (double)v[rr].z;
        acc[rr] += e[3] * (double)v[rr].w;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) e[q] = en[q];
#pragma unroll
      for (int rr = 0; rr < kRowsPerWg; ++rr) v[rr] = vn[rr];
    }
#pragma unroll
    for (int rr = 0; rr < kRowsPerWg; ++rr) {
      const double tot = block_sum(acc[rr], lds);
      if (threadIdx.x == 0 && r0 + rr < R) b.upart[(size_t)(r0 + rr) * nch + c] = tot;
    }
  }
  if (threadIdx.x == 0) {
    release_fence();
    const uint32_t prev = atomicAdd(&b.counters[1], 1u);
    is_last = (prev == gridDim.x * gridDim.y - 1);
  }
  __syncthreads();
  if (!is_last) return;
  acquire_fence();
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

// Deferred update, eq. (36) from the workgroup partials of eq. (37):
// U[r] += alpha / eta * sum_wg scale_wg P[wg][r], for rollouts with too
// many workgroups for the last one to combine (the rollout's epilogue has
// published P and stored the rescales scale_wg).  Workgroup (rb, c) takes
// the kPartRows rows of block rb over the partials of chunk c: wavefront q
// sums partials q, q + 4, ... of the chunk in order (each a coalesced load
// of the block's rows; kPartLoads of them in flight per thread), and the four
// wavefront sums, added as (s0 + s1) + (s2 + s3), go to upart[r][c].  The
// last workgroup of a row block to arrive adds its rows' chunk sums in chunk
// order (four contiguous runs of chunks, one per wavefront, combined the
// same way) and updates U; the one of block 0 advances the iteration counter.
constexpr int kPartLoads = 16;
constexpr int kPartMaxChunks = 64;

__global__ __launch_bounds__(256) void partial_update_kernel(const DevParams p, const Buffers b,
                                                             int R, int nwg, int nch, int chunk) {
  __shared__ double sums[4][kPartRows];
  __shared__ int is_last;
  const mppi_jump_stats st = *b.stats;
  const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int rb = blockIdx.x, c = blockIdx.y;
  const int r = rb * kPartRows + lane;
  const bool live = r < R;
  const int rr = min(r, R - 1);  // rows past R read row R - 1 and are never stored
  const bool ok = st.status == MPPI_OK;
  {
    // the loads do not wait for the status (they stay inside the partials
    // either way); only the store does
    const int j0 = c * chunk, j1 = min(nwg, j0 + chunk);
    double acc = 0.0;
    for (int jb = j0 + q; jb < j1; jb += 4 * kPartLoads) {
      double w[kPartLoads], sc[kPartLoads];
#pragma unroll
      for (int i = 0; i < kPartLoads; ++i) {
        const int j = min(jb + 4 * i, j1 - 1);
        w[i] = b.wpart[(size_t)j * R + rr];
        sc[i] = b.scale[j];
      }
#pragma unroll
      for (int i = 0; i < kPartLoads; ++i)
        if (jb + 4 * i < j1) acc += sc[i] * w[i];
    }
    sums[q][lane] = acc;
    __syncthreads();
    if (ok && q == 0 && live)
      b.upart[(size_t)r * nch + c] = (sums[0][lane] + sums[1][lane]) + (sums[2][lane] + sums[3][lane]);
  }
  if (q == 0) {
    release_fence();  // wavefront 0's chunk sums before its arrival
    if (lane == 0) is_last = atomicAdd(&b.counters[kCounters + rb], 1u) == (uint32_t)nch - 1;
  }
  __syncthreads();
  if (!is_last) return;
  acquire_fence();
  if (ok) {
    const int L = (nch + 3) / 4;  // at most kPartMaxChunks / 4
    const int c0 = q * L, c1 = min(nch, c0 + L);
    double v[kPartMaxChunks / 4];
#pragma unroll
    for (int i = 0; i < kPartMaxChunks / 4; ++i)
      v[i] = c0 + i < c1 ? b.upart[(size_t)rr * nch + c0 + i] : 0.0;
    double d = 0.0;
#pragma unroll
    for (int i = 0; i < kPartMaxChunks / 4; ++i)
      if (c0 + i < c1) d += v[i];
    sums[q][lane] = d;
    __syncthreads();
    if (q == 0 && live) {
      const double tot = (sums[0][lane] + sums[1][lane]) + (sums[2][lane] + sums[3][lane]);
      b.U[r] = (float)((double)b.U[r] + (double)p.alpha / st.eta * tot);
    }
  }
  if (threadIdx.x == 0) {
    b.counters[kCounters + rb] = 0u;
    if (rb == 0) b.stats->iteration = st.iteration + 1;
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
    for (int i = 0; i < counter_count(R); ++i) b.counters[i] = 0u;
  }
}

// Statistics, iteration counter and arrival counters of a workspace reset,
// leaving U alone (the no-allocation control step, whose sequence belongs
// to the caller).
__global__ void stats_init_kernel(Buffers b, int R, uint64_t start_iteration) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    b.stats->rho = 0.0;
    b.stats->eta = 0.0;
    b.stats->status = MPPI_OK;
    b.stats->n_finite = 0;
    b.stats->iteration = start_iteration;
    for (int i = 0; i < counter_count(R); ++i) b.counters[i] = 0u;
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

// One explicit Euler step of the plant under u + d and, for the models that
// take one, the world-frame body force (null: none).
template <int DYN>
__global__ void plant_kernel(const DevParams p, float* __restrict__ x,
                             const float* __restrict__ u, const float* __restrict__ d,
                             const float* __restrict__ force) {
  using Md = Model<DYN>;
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  float s[Md::N], v[Md::M];
  float gust[3] = {0.f, 0.f, 0.f};
  if (force != nullptr) {
    gust[0] = force[0];
    gust[1] = force[1];
    gust[2] = force[2];
  }
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
  W[k] = st.status == MPPI_OK ? b.E[k] * b.scale[k >> p.wg_shift] / st.eta : 0.0;
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

#include "rollout_ws.hpp"
#include "batch.hpp"
