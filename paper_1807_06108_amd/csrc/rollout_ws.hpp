// Wave-specialised rollout: a workgroup of W wavefronts serves 64 samples.
// W - 1 producer waves form the draws (Philox, Box-Muller,
// jump counts), the applied controls v = U[t] + eps and the state-free part of
// the stage cost for a chunk of time steps and pass them through an LDS ring;
// the consumer wave runs the state recursion (dynamics and state cost) of
// the previous chunk meanwhile.  The per-step instruction stream of the
// serial recursion then holds only the dynamics and the state cost, which
// is what bounds the iteration latency when K is too small to fill the chip.
// Results are identical to the one-sample-per-lane rollout: the same draws
// from the same counters and the same fp32 arithmetic in the same order.
#pragma once
#include "kernels.hpp"

namespace mppi {

constexpr int kWsSamples = 64;  // samples per workgroup
constexpr int kWsChunk = 16;    // time steps per ring slot (one cost block)

// Wavefronts per workgroup: eight (two per SIMD, one consumer and seven
// producers).  Measured on the light models, 4, 6 and 12 are slower; for the
// 12-state model eight waves cap the registers at 256 per lane (a few are
// spilled) yet beat four waves with 512 (57.9 vs 60.3 us at K=8192, T=100):
// with three producers it is the draws that bound the iteration.
template <int DYN>
struct WsWaves {
  static constexpr int W = 8;
};

// Steps of a chunk per producer wave with eight waves.  The waves of a
// workgroup sit on the four SIMDs round-robin, so wave 4 shares SIMD 0 with
// the consumer: it takes MATE steps and the rest are split evenly over
// SIMDs 1-3 (waves 1 and 5, 2 and 6, 3 and 7), each wave a contiguous range.
// On the light models the consumer's recursion sets the pace and its mate
// takes one step (measured: 0 and 2 are slower); the 12-state model's two
// draw blocks per step keep the producers close to the consumer's pace, and
// its mate keeps an even share (two steps: the per-wave counts of a
// round-robin split; one step measures the same, three are slower).
template <int DYN, int CH = kWsChunk>
struct WsSplit {
  static constexpr int MATE = DYN == MPPI_DYN_QUADROTOR ? 2 : 1;
  __host__ __device__ static constexpr int count(int w) {
    if (w <= 0 || w > 7) return 0;
    if (w == 4) return MATE;
    const int rem = CH - MATE;
    const int simd = w & 3;  // 1..3
    const int n = rem / 3 + (simd - 1 < rem % 3 ? 1 : 0);
    return w < 4 ? (n + 1) / 2 : n / 2;
  }
  __host__ __device__ static constexpr int first(int w) {
    int f = 0;
    for (int v = 1; v < w; ++v) f += count(v);
    return f;
  }
};
static_assert(kWsChunk == kCostBlock, "a ring chunk is one cost block (schedules agree bitwise)");
static_assert(WsSplit<MPPI_DYN_CARTPOLE>::first(8) == kWsChunk, "split covers the chunk");
static_assert(WsSplit<MPPI_DYN_QUADROTOR>::first(8) == kWsChunk, "split covers the chunk");
static_assert(WsSplit<MPPI_DYN_LINEAR>::first(8) == kWsChunk, "split covers the chunk");

// Steps of a full chunk that the consumer's loop unrolls.  Fully unrolled,
// the 12-state model's chunk has the ring reads of many steps hoisted and
// spills registers; four steps per trip keep it spill-free and measure
// fastest for it (K=8192, T=100: 16 steps 52.7 us, 8 steps 52.3, 4 steps
// 50.7; the same costs and updates bitwise).
template <int DYN>
struct WsConsumeUnroll {
  static constexpr int U = DYN == MPPI_DYN_QUADROTOR ? 4 : kWsChunk;
};

// Fields of a ring slot, per step and sample: the applied controls v[M]
// (HAS_V), the body force gust[NG] and the state-free part of the stage
// cost.  With the perturbation tile on chip (TILE) a multi-channel model's
// ring omits v: the consumer forms v = U[t] + eps from the tile (the same
// fp32 sum the producer would form), which shrinks its ring by half so that
// ring and tile fit in LDS together.
template <int DYN, bool TILE = false>
struct WsRing {
  using Md = Model<DYN>;
  static constexpr bool HAS_V = !(TILE && Md::M > 1);
  static constexpr int NV = HAS_V ? Md::M : 0;
  static constexpr int NG = Md::JUMP_IN_CONTROL ? 0 : 3;  // disturbance floats
  static constexpr int NF = NV + NG + 1;                  // v[NV], gust[NG], state-free cost
};

template <int DYN, bool TILE = false>
constexpr size_t ws_ring_bytes() {
  return sizeof(float) * 2 * kWsChunk * WsRing<DYN, TILE>::NF * 64;
}

// On-chip perturbation tile of the fused wave-specialised rollout
// (EPS_LDS): the workgroup's eps[t][j][k] for its 64 samples, R = T m rows
// of 64 floats after the ring in dynamic LDS.  The epilogue's weighted sums
// read it from there, and the perturbations never go to HBM (eq. (37)'s
// weights are only known once every cost is, so the tile must be kept until
// then; on chip it costs neither the store and re-read nor the write-back of
// the L2 lines that the release fence would otherwise flush).  Used when the
// ring and the tile fit beside the kernel's static LDS: T <= 496 for the
// one-channel models, T <= 108 for the 12-state model (whose ring then omits
// v, above).
// The single-controller kernels also stage the control sequence U (R
// floats) after the ring and the tile: read once at kernel start, all lines
// at once, instead of one L2 miss after another as the producers reach new
// steps (the sequence was just written by the previous launch, on another
// XCD).
constexpr size_t kLdsBytes = 160 * 1024;     // LDS of a gfx950 compute unit
constexpr size_t kWsStaticLds = 18 * 1024;   // bound on the kernel's static LDS
template <int DYN>
constexpr size_t ws_lds_bytes(int R) {
  return ws_ring_bytes<DYN, false>() + sizeof(float) * (size_t)R;
}
template <int DYN>
constexpr size_t ws_eps_lds_bytes(int R) {
  return ws_ring_bytes<DYN, true>() + sizeof(float) * (size_t)R * (kWsSamples + 1);
}
// The tile fits when `per_cu` workgroups of the kernel still fit in a
// compute unit's LDS: one for the fused form (at most 512 workgroups, two
// per compute unit at most), two for the deferred form, whose thousands of
// workgroups need the occupancy more than the saved HBM pass (quadrotor
// K=65536, T=100: the tile on chip, 147 KB of LDS and one workgroup per
// compute unit, 187.9 us per iteration; in HBM, 75 KB and two, 135.2 us).
template <int DYN>
constexpr bool ws_eps_fits(int R, int per_cu = 1) {
  return (ws_eps_lds_bytes<DYN>(R) + kWsStaticLds) * per_cu <= kLdsBytes;
}

// The part of a step's production that needs U: the applied controls, the
// state-free cost and the stores of the draws nz of step t.
template <int DYN, bool JUMPS, bool DEBUG, int FORM, bool FULL, bool EPS_LDS>
__device__ __forceinline__ void ws_finish(const DevParams& p, const Consts& cs, const Buffers& b,
                                          const Noise<DYN, JUMPS>& nz, const float* U,
                                          float* slot, float* epsl, int t, int k, bool active) {
  using Md = Model<DYN>;
  using Rg = WsRing<DYN, EPS_LDS>;
  constexpr int M = Md::M, Q = Md::Q;
  float u[M];
#pragma unroll
  for (int j = 0; j < M; ++j) u[j] = U[t * M + j];
  const int lane = threadIdx.x & 63;
  if constexpr (Rg::HAS_V) {
#pragma unroll
    for (int j = 0; j < M; ++j) slot[j * 64 + lane] = u[j] + nz.eps[j];
  }
#pragma unroll
  for (int i = 0; i < Rg::NG; ++i) slot[(Rg::NV + i) * 64 + lane] = nz.gust[i];
  slot[(Rg::NF - 1) * 64 + lane] = state_free_cost<M, FORM, FULL>(p, cs, u, nz.eps);
  if constexpr (EPS_LDS) {
#pragma unroll
    for (int j = 0; j < M; ++j) epsl[(t * M + j) * kWsSamples + lane] = nz.eps[j];
  } else {
#pragma unroll
    for (int j = 0; j < M; ++j) b.eps[(size_t)(t * M + j) * p.Ks + k] = nz.eps[j];
  }
  if constexpr (DEBUG) {
    if (active) {
      const size_t kt = (size_t)k * p.T + t;
#pragma unroll
      for (int j = 0; j < M; ++j) b.dbg_zD[kt * M + j] = nz.z[j];
      b.dbg_N[kt] = nz.n;
#pragma unroll
      for (int i = 0; i < Q; ++i) b.dbg_zJ[kt * Q + i] = JUMPS ? nz.z[M + i] : 0.f;
    }
  }
}

template <int DYN, bool JUMPS, bool DEBUG, int FORM, bool FULL, bool EPS_LDS>
__device__ __forceinline__ void ws_produce(const DevParams& p, const Consts& cs, const Buffers& b,
                                           const float* U, float* slot, float* epsl, int t,
                                           int k, bool active, uint32_t it) {
  Noise<DYN, JUMPS> nz;
  draw_noise<DYN, JUMPS, FULL>(nz, p, cs, (uint32_t)t, p.k0 + (uint32_t)k, it);
  ws_finish<DYN, JUMPS, DEBUG, FORM, FULL, EPS_LDS>(p, cs, b, nz, U, slot, epsl, t, k, active);
}

template <int DYN>
struct WsState {
  float x[Model<DYN>::N];
  CostSum S;
  bool crashed;
};

// One step of the state recursion: running cost on the pre-step state, then
// the explicit Euler step (frozen once crashed).  v: applied controls, gust:
// body-force disturbance (zero for jumps through the control channel), pre:
// the state-free part of the stage cost.
template <int DYN>
__device__ __forceinline__ void ws_step(const DevParams& p, const Consts& cs, WsState<DYN>& st,
                                        const float* v, const float* gust, float pre) {
  using Md = Model<DYN>;
  constexpr int N = Md::N;
  float qx = 0.f;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const float d = st.x[i] - cs.goal[i];
    qx += cs.Q[i] * d * d;
  }
  if constexpr (Md::CAN_CRASH) qx += st.crashed ? p.pen : 0.f;
  st.S.add(qx * p.dt + pre);
  if constexpr (Md::CAN_CRASH) {
    float xn[N];
#pragma unroll
    for (int i = 0; i < N; ++i) xn[i] = st.x[i];
    Md::step(xn, v, gust, p.dt, cs.mc);
#pragma unroll
    for (int i = 0; i < N; ++i) st.x[i] = st.crashed ? st.x[i] : xn[i];
    st.crashed = st.crashed || Md::crashed(st.x, cs.mc);
  } else {
    Md::step(st.x, v, gust, p.dt, cs.mc);
  }
}

// A ring slot's values for one step: applied controls, body force, the
// state-free part of the stage cost.
template <int DYN>
struct WsSlot {
  float v[Model<DYN>::M], gust[3], pre;
};

// The values of step t from its ring slot; without v in the ring, v = U[t] +
// eps[t] from the on-chip tile.
template <int DYN, bool TILE>
__device__ __forceinline__ WsSlot<DYN> ws_read(const float* slot, const float* epsl,
                                               const float* U, int t) {
  using Rg = WsRing<DYN, TILE>;
  constexpr int M = Model<DYN>::M;
  const int lane = threadIdx.x & 63;
  WsSlot<DYN> o;
  if constexpr (Rg::HAS_V) {
#pragma unroll
    for (int j = 0; j < M; ++j) o.v[j] = slot[j * 64 + lane];
  } else {
#pragma unroll
    for (int j = 0; j < M; ++j) o.v[j] = U[t * M + j] + epsl[(t * M + j) * kWsSamples + lane];
  }
  o.gust[0] = o.gust[1] = o.gust[2] = 0.f;
#pragma unroll
  for (int i = 0; i < Rg::NG; ++i) o.gust[i] = slot[(Rg::NV + i) * 64 + lane];
  o.pre = slot[(Rg::NF - 1) * 64 + lane];
  return o;
}

// The n steps of a chunk starting at step t0.  For the one-channel models
// each slot is read one step ahead, so that the LDS latency hides behind the
// previous step's recursion (their step is short enough for the compiler's
// own placement to leave it exposed: C1 19.0 -> 18.8 us); the 12-state model
// reads each slot at its step (reading ahead measured slower there: K=8192
// 50.7 -> 52.2 us).
template <int DYN, int UNROLL, bool TILE>
__device__ __forceinline__ void ws_consume_chunk(const DevParams& p, const Consts& cs,
                                                 WsState<DYN>& st, const float* buf, int slot_floats,
                                                 int n, int t0, const float* epsl, const float* U) {
  if constexpr (Model<DYN>::M == 1) {
    WsSlot<DYN> cur = ws_read<DYN, TILE>(buf, epsl, U, t0);
#pragma unroll UNROLL
    for (int s = 0; s < n; ++s) {
      WsSlot<DYN> nxt = cur;
      if (s + 1 < n) nxt = ws_read<DYN, TILE>(buf + (s + 1) * slot_floats, epsl, U, t0 + s + 1);
      ws_step<DYN>(p, cs, st, cur.v, cur.gust, cur.pre);
      cur = nxt;
    }
  } else {
#pragma unroll UNROLL
    for (int s = 0; s < n; ++s) {
      const WsSlot<DYN> cur = ws_read<DYN, TILE>(buf + s * slot_floats, epsl, U, t0 + s);
      ws_step<DYN>(p, cs, st, cur.v, cur.gust, cur.pre);
    }
  }
}

// The rollout of one workgroup (tile wg, W waves) at iteration `it`:
// returns S~_k of sample wg * 64 + lane in wavefront 0 (also stored to b.S).
// cs: the staged constants; Ug: the control sequence (global memory), which
// with STAGE_U is copied to Ul (LDS, R floats) and read from there.  With
// EPS_LDS the perturbation tile is left on chip for the epilogue.
template <int DYN, bool JUMPS, bool DEBUG, int FORM, int W, bool FULL, bool EPS_LDS,
          bool STAGE_U = false>
__device__ __forceinline__ double ws_rollout(const DevParams& p, const Consts& cs,
                                             const Buffers& b, const float* __restrict__ x0,
                                             const float* Ug, float* Ul, int R, int wg,
                                             uint32_t it) {
  using Md = Model<DYN>;
  using Rg = WsRing<DYN, EPS_LDS>;
  constexpr int N = Md::N;
  constexpr int NP = W - 1;  // producer waves
  constexpr int CH = kWsChunk;
  constexpr int SLOT = Rg::NF * 64;  // floats per (step) slot
  // the ring lives in dynamic LDS (ws_ring_bytes<DYN, EPS_LDS>() at launch,
  // plus the perturbation tile with EPS_LDS), so that kernels containing
  // several model variants share one allocation
  extern __shared__ float ws_dyn_lds[];
  float(*ring)[CH][SLOT] = reinterpret_cast<float(*)[CH][SLOT]>(ws_dyn_lds);
  float* epsl = ws_dyn_lds + 2 * CH * SLOT;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int k = wg * kWsSamples + lane;
  const bool active = k < p.K;
  const int T = p.T;
  const int nch = (T + CH - 1) / CH;

  // eight waves: this producer's contiguous range of each chunk's steps
  int s0 = 0, s1 = 0;
  if constexpr (W == 8) {
    const int w = __builtin_amdgcn_readfirstlane(wave);
    s0 = WsSplit<DYN>::first(w);
    s1 = s0 + WsSplit<DYN>::count(w);
  }

  WsState<DYN> st;
#pragma unroll
  for (int i = 0; i < N; ++i) st.x[i] = x0[i];
  st.crashed = Md::CAN_CRASH ? Md::crashed(st.x, cs.mc) : false;
  st.S = CostSum{};

  // The first chunk is produced by all W waves (the consumer has nothing
  // to do before it), CH / W steps each, so the recursion starts sooner.
  // Then producers and the consumer run separate loops (the branch is
  // uniform per wavefront), so the register allocation of each holds only
  // its own live values and constants, not the union of both.  Both sides
  // pass nch + 1 barriers: chunk c is produced before barrier c and consumed
  // after it.
  // With STAGE_U the sequence is copied to LDS (Ul) here: its load (the
  // previous launch wrote it, from another XCD) is issued before the first
  // chunk's draws, which do not need it, and waited for only after them.
  static_assert(CH % W == 0, "the first chunk splits evenly over the waves");
  const float* U = STAGE_U ? static_cast<const float*>(Ul) : Ug;
  {
    constexpr int NS = CH / W;
    const int w = __builtin_amdgcn_readfirstlane(wave);
    float u_mine = 0.f;
    if constexpr (STAGE_U) {
      if ((int)threadIdx.x < R) u_mine = Ug[threadIdx.x];
    }
    Noise<DYN, JUMPS> nz[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i)
      if (w * NS + i < T)
        draw_noise<DYN, JUMPS, FULL>(nz[i], p, cs, (uint32_t)(w * NS + i), p.k0 + (uint32_t)k, it);
    if constexpr (STAGE_U) {
      if ((int)threadIdx.x < R) Ul[threadIdx.x] = u_mine;
      for (int r = threadIdx.x + 64 * W; r < R; r += 64 * W) Ul[r] = Ug[r];
      __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < NS; ++i)
      if (w * NS + i < T)
        ws_finish<DYN, JUMPS, DEBUG, FORM, FULL, EPS_LDS>(p, cs, b, nz[i], U, ring[0][w * NS + i],
                                                           epsl, w * NS + i, k, active);
  }
  __syncthreads();
  MPPI_PHASE(b.stats->iteration, wg, (p.K + kWsSamples - 1) / kWsSamples, 7);
  if (__builtin_amdgcn_readfirstlane(wave) > 0) {
    for (int c = 1; c < nch; ++c) {
      float(*buf)[SLOT] = ring[c & 1];
      if constexpr (W == 8) {
        for (int s = s0; s < s1; ++s) {
          const int t = c * CH + s;
          if (t < T)
            ws_produce<DYN, JUMPS, DEBUG, FORM, FULL, EPS_LDS>(p, cs, b, U, buf[s], epsl, t, k,
                                                                active, it);
        }
      } else {
        for (int s = wave - 1; s < CH; s += NP) {
          const int t = c * CH + s;
          if (t < T)
            ws_produce<DYN, JUMPS, DEBUG, FORM, FULL, EPS_LDS>(p, cs, b, U, buf[s], epsl, t, k,
                                                                active, it);
        }
      }
      __syncthreads();
    }
    __syncthreads();
  } else {
    constexpr int kUnroll = WsConsumeUnroll<DYN>::U;
    for (int cc = 0; cc < nch; ++cc) {
      float(*buf)[SLOT] = ring[cc & 1];
      if ((cc + 1) * CH <= T)
        ws_consume_chunk<DYN, kUnroll, EPS_LDS>(p, cs, st, buf[0], SLOT, CH, cc * CH, epsl, U);
      else
        ws_consume_chunk<DYN, 1, EPS_LDS>(p, cs, st, buf[0], SLOT, T - cc * CH, cc * CH, epsl, U);
      st.S.close_block();  // a chunk is one cost block
      __syncthreads();
    }
  }

  double Sd = 0.0;
  if (wave == 0) {
    float qf = 0.f;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const float d = st.x[i] - cs.goal[i];
      qf += p.Qf[i] * d * d;
    }
    if constexpr (Md::CAN_CRASH) qf += st.crashed ? p.pen : 0.f;
    Sd = st.S.S + (double)qf;
    if (active) b.S[k] = Sd;
  }
  return Sd;
}

// One workgroup (tile wg of nwg) of the wave-specialised rollout, W waves,
// with its one-iteration epilogue.  U_LDS: U is staged in LDS after the
// ring and the tile while the first chunk's draws are formed (the
// single-controller kernels; the batched ones, whose controllers differ in
// R, read it from global memory).  DEFER: the
// epilogue's deferred-update form (rollout_epilogue), for more workgroups
// than one combines.
template <int DYN, bool JUMPS, bool DEBUG, int FORM, bool FUSED, int W, bool FULL = false,
          bool EPS_LDS = false, bool U_LDS = false, bool DEFER = false>
__device__ __forceinline__ void rollout_ws_tile(const DevParams& p, const Buffers& b,
                                                const float* __restrict__ x0,
                                                const float* U, int R,
                                                const ShiftArgs& sh, int wg, int nwg) {
  static_assert(!EPS_LDS || FUSED, "the on-chip tile serves the fused epilogue");
  MPPI_PHASE(b.stats->iteration, wg, nwg, 0);
  extern __shared__ float ws_dyn_lds[];
  constexpr int kRingFloats = 2 * kWsChunk * WsRing<DYN, EPS_LDS>::NF * 64;
  float* Ul = ws_dyn_lds + kRingFloats + (EPS_LDS ? (size_t)R * kWsSamples : 0);
  __shared__ Consts cs;
  stage_consts(cs, p);
  const uint32_t it = (uint32_t)b.stats->iteration;
  const double Sd = ws_rollout<DYN, JUMPS, DEBUG, FORM, W, FULL, EPS_LDS, U_LDS>(p, cs, b, x0, U,
                                                                                Ul, R, wg, it);
  // the epilogue's weighted sums read the tile on chip, or the workgroup's
  // columns of the HBM perturbations
  const float* tile = EPS_LDS ? ws_dyn_lds + kRingFloats : b.eps + (size_t)wg * kWsSamples;
  const int tstride = EPS_LDS ? kWsSamples : p.Ks;
  const int k = wg * kWsSamples + (threadIdx.x & 63);
  const bool holds = (threadIdx.x >> 6) == 0 && k < p.K;  // wavefront 0 holds the costs
  rollout_epilogue<kWsSamples, FUSED, 64 * W, DEFER>(p, b, Sd, holds, R, sh, wg, nwg, tile,
                                                     tstride);
}

template <int DYN, bool JUMPS, bool DEBUG, int FORM, bool FUSED, bool FULL, bool EPS_LDS,
          bool DEFER = false>
__global__ __launch_bounds__(64 * WsWaves<DYN>::W) void rollout_ws_kernel(const DevParams p,
                                                                         const Buffers b,
                                                                         const float* __restrict__ x0,
                                                                         const float* U,
                                                                         int R, const ShiftArgs sh) {
  rollout_ws_tile<DYN, JUMPS, DEBUG, FORM, FUSED, WsWaves<DYN>::W, FULL, EPS_LDS, true, DEFER>(
      p, b, x0, U, R, sh, blockIdx.x, gridDim.x);
}

}  // namespace mppi
