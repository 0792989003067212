// Batched form: one launch advances many independent controllers (uneven K,
// T, dynamics, jump rates) by one iteration each.  A device descriptor table
// holds every controller's parameters and buffers; a tile list maps each
// workgroup of the grid to (controller, tile), ordered longest-first so the
// hardware dispatcher starts the long tiles early.  Each controller's own
// last-arriving tile combines its partials and applies its update (and, on
// the last iteration of a control step, its shift), exactly as in the
// single-controller kernels: results are identical to running the
// controllers one by one.
#pragma once
#include "kernels.hpp"

namespace mppi {

struct BatchDesc {
  DevParams p;
  Buffers b;
  const float* x0;
  float* u0_out;  // this controller's u_0 slot (device), may be null
  float4 u_init;
  int R, nwg, dyn, jumps, form, m;
};

struct BatchTile {
  int ctl;
  int wg;
};

// The wave-specialised tiles here run four waves (one consumer, three
// producers) in 256-thread blocks.  Eight waves, as in the single-controller
// kernel, measured no faster over a mixed batch (the per-tile switch over
// all twelve instantiations already costs the registers that the extra
// producers would need, and the eight-wave build spills).
// MASK: the dynamics ids compiled in (bit DYN); a batch of one model runs a
// kernel holding only that model's variants (fewer registers).
constexpr int kMaskAll = 7, kMaskCartpole = 1 << MPPI_DYN_CARTPOLE,
              kMaskQuadrotor = 1 << MPPI_DYN_QUADROTOR;

template <bool WS, int MASK = kMaskAll>
__device__ __forceinline__ void batch_tile(const BatchDesc& d, const float* x0, const ShiftArgs& sh,
                                           int wg) {
  const int sel = d.dyn * 4 + d.jumps * 2 + (d.form == MPPI_COST_SO ? 1 : 0);
#define MPPI_BATCH_CASE(DYN, J, F)                                                            \
  case DYN * 4 + J * 2 + (F == MPPI_COST_SO ? 1 : 0):                                       \
    if constexpr ((MASK >> DYN) & 1) {                                                        \
      if constexpr (WS)                                                                       \
        rollout_ws_tile<DYN, J, false, F, true, 4>(d.p, d.b, x0, d.b.U, d.R, sh, wg, d.nwg); \
      else                                                                                    \
        rollout_lane_tile<DYN, J, false, F, true>(d.p, d.b, x0, d.b.U, d.R, sh, wg, d.nwg);  \
    }                                                                                         \
    break;
  switch (sel) {
    MPPI_BATCH_CASE(MPPI_DYN_LINEAR, 0, MPPI_COST_IT)
    MPPI_BATCH_CASE(MPPI_DYN_LINEAR, 0, MPPI_COST_SO)
    MPPI_BATCH_CASE(MPPI_DYN_LINEAR, 1, MPPI_COST_IT)
    MPPI_BATCH_CASE(MPPI_DYN_LINEAR, 1, MPPI_COST_SO)
    MPPI_BATCH_CASE(MPPI_DYN_CARTPOLE, 0, MPPI_COST_IT)
    MPPI_BATCH_CASE(MPPI_DYN_CARTPOLE, 0, MPPI_COST_SO)
    MPPI_BATCH_CASE(MPPI_DYN_CARTPOLE, 1, MPPI_COST_IT)
    MPPI_BATCH_CASE(MPPI_DYN_CARTPOLE, 1, MPPI_COST_SO)
    MPPI_BATCH_CASE(MPPI_DYN_QUADROTOR, 0, MPPI_COST_IT)
    MPPI_BATCH_CASE(MPPI_DYN_QUADROTOR, 0, MPPI_COST_SO)
    MPPI_BATCH_CASE(MPPI_DYN_QUADROTOR, 1, MPPI_COST_IT)
    MPPI_BATCH_CASE(MPPI_DYN_QUADROTOR, 1, MPPI_COST_SO)
    default: break;
  }
#undef MPPI_BATCH_CASE
}

__device__ __forceinline__ ShiftArgs batch_shift(const BatchDesc& d, int shift) {
  ShiftArgs sh;
  sh.on = shift;
  sh.u0_out = d.u0_out;
  sh.m = d.m;
  sh.u_init = d.u_init;
  return sh;
}

// Grid launch: one workgroup per tile; the hardware dispatcher starts them
// in tile-list order as compute units free up.  shift != 0: this launch is
// the last iteration of a control step.
template <bool WS, int MASK>
__global__ __launch_bounds__(256) void batch_rollout_kernel(const BatchDesc* __restrict__ descs,
                                                            const BatchTile* __restrict__ tiles,
                                                            int shift) {
  MPPI_TILE_MARK(blockIdx.x, 0);
  const BatchTile tl = tiles[blockIdx.x];
  const BatchDesc& d = descs[tl.ctl];
  batch_tile<WS, MASK>(d, d.x0, batch_shift(d, shift), tl.wg);
  MPPI_TILE_MARK(blockIdx.x, 1);
}

// Work queue of the persistent launch: the next tile to take and the number
// of workgroups that have left.  Zero before a launch; the last workgroup to
// leave zeroes it again for the next one.
struct BatchQueue {
  uint32_t head;
  uint32_t done;
};

// Persistent launch: as many workgroups as the GPU holds at once, each
// taking the next tile of the longest-first list from the queue until none
// is left.  Nothing waits on another workgroup (a controller's last tile
// combines its partials as in the grid launch), so every workgroup reaches
// the end once the list is exhausted.
template <bool WS, int MASK>
__global__ __launch_bounds__(256) void batch_persistent_kernel(const BatchDesc* __restrict__ descs,
                                                               const BatchTile* __restrict__ tiles,
                                                               int ntiles, int shift,
                                                               BatchQueue* queue) {
  __shared__ int next;
  for (;;) {
    __syncthreads();  // the previous tile is done with LDS and with `next`
    if (threadIdx.x == 0) next = (int)atomicAdd(&queue->head, 1u);
    __syncthreads();
    const int t = next;
    if (t >= ntiles) break;
    const BatchTile tl = tiles[t];
    const BatchDesc& d = descs[tl.ctl];
    batch_tile<WS, MASK>(d, d.x0, batch_shift(d, shift), tl.wg);
  }
  if (threadIdx.x == 0) {
    __threadfence();  // this workgroup's queue increments precede its exit count
    if (atomicAdd(&queue->done, 1u) == gridDim.x - 1) {
      atomicExch(&queue->head, 0u);
      atomicExch(&queue->done, 0u);
    }
  }
}

}  // namespace mppi

namespace mppi {

// Serving form: a tick advances a subset of a resident pool.  The request
// record of a tick (device memory) holds, in longest-first order, the
// controller ids [count], the tile prefix [count + 1], the states
// [count][12] and the plant disturbances [count][kPoolDist] (words 0..3
// added to the control channels, words 4..6 a world-frame body force for
// the models that take one); workgroup b finds its
// request by binary search over the prefix.  Request i writes u_0 to
// out[16 i .. 16 i + m) and, when the plant runs, the next plant state to
// out[16 i + 4 .. 16 i + 4 + n).
struct PoolTick {
  const int* ids;
  const int* prefix;
  const float* states;
  const float* dist;
  float* out;
  int count;
  int shift;
};

constexpr int kPoolOut = 16;
constexpr int kPoolDist = 8;

__device__ __forceinline__ int find_request(const int* prefix, int count, int b) {
  int lo = 0, hi = count;  // prefix[lo] <= b < prefix[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (prefix[mid] <= b)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

template <bool WS>
__global__ __launch_bounds__(256) void pool_rollout_kernel(const BatchDesc* __restrict__ descs,
                                                           const PoolTick tick) {
  const int i = find_request(tick.prefix, tick.count, blockIdx.x);
  const BatchDesc& d = descs[tick.ids[i]];
  ShiftArgs sh;
  sh.on = tick.shift;
  sh.u0_out = tick.out + kPoolOut * i;
  sh.m = d.m;
  sh.u_init = d.u_init;
  batch_tile<WS, kMaskAll>(d, tick.states + 12 * i, sh, blockIdx.x - tick.prefix[i]);
}

template <int DYN>
__device__ __forceinline__ void pool_plant_one(const DevParams& p, const float* x, const float* d,
                                               float* out) {
  using Md = Model<DYN>;
  float s[Md::N], v[Md::M];
  const float gust[3] = {d[4], d[5], d[6]};
#pragma unroll
  for (int j = 0; j < Md::N; ++j) s[j] = x[j];
#pragma unroll
  for (int j = 0; j < Md::M; ++j) v[j] = out[j] + d[j];
  Md::step(s, v, gust, p.dt, p.mc);
#pragma unroll
  for (int j = 0; j < Md::N; ++j) out[4 + j] = s[j];
}

// Simulated plant of each request: one explicit Euler step from the request
// state under u_0 + disturbance and, for the quadrotor, the body force (the
// step of plant_kernel with a gust input).
__global__ __launch_bounds__(64) void pool_plant_kernel(const BatchDesc* __restrict__ descs,
                                                        const PoolTick tick) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  if (i >= tick.count) return;
  const BatchDesc& d = descs[tick.ids[i]];
  const float* x = tick.states + 12 * i;
  const float* w = tick.dist + kPoolDist * i;
  float* out = tick.out + kPoolOut * i;
  switch (d.dyn) {
    case MPPI_DYN_LINEAR: pool_plant_one<MPPI_DYN_LINEAR>(d.p, x, w, out); break;
    case MPPI_DYN_CARTPOLE: pool_plant_one<MPPI_DYN_CARTPOLE>(d.p, x, w, out); break;
    default: pool_plant_one<MPPI_DYN_QUADROTOR>(d.p, x, w, out); break;
  }
}

}  // namespace mppi
