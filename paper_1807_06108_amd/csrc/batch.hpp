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

template <bool WS>
__device__ __forceinline__ void batch_tile(const BatchDesc& d, const ShiftArgs& sh, int wg) {
  const int sel = d.dyn * 4 + d.jumps * 2 + (d.form == MPPI_COST_SO ? 1 : 0);
#define MPPI_BATCH_CASE(DYN, J, F)                                                            \
  case DYN * 4 + J * 2 + (F == MPPI_COST_SO ? 1 : 0):                                       \
    if constexpr (WS)                                                                         \
      rollout_ws_tile<DYN, J, false, F, true, 4>(d.p, d.b, d.x0, d.b.U, d.R, sh, wg, d.nwg); \
    else                                                                                      \
      rollout_lane_tile<DYN, J, false, F, true>(d.p, d.b, d.x0, d.b.U, d.R, sh, wg, d.nwg);  \
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

// shift != 0: this launch is the last iteration of a control step.
template <bool WS>
__global__ __launch_bounds__(256) void batch_rollout_kernel(const BatchDesc* __restrict__ descs,
                                                            const BatchTile* __restrict__ tiles,
                                                            int shift) {
  const BatchTile tl = tiles[blockIdx.x];
  const BatchDesc& d = descs[tl.ctl];
  ShiftArgs sh;
  sh.on = shift;
  sh.u0_out = d.u0_out;
  sh.m = d.m;
  sh.u_init = d.u_init;
  batch_tile<WS>(d, sh, tl.wg);
}

}  // namespace mppi
