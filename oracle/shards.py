"""Test infrastructure: the oracle with its samples split over worker
processes, for timing the oracle on all host cores.

Same arithmetic as oracle.mppi: each sample's draws, rollout and path cost
depend on that sample alone (Algorithm 1 treats the K trajectories
independently until the weights), so each worker runs mppi.iteration on a
contiguous range of sample indices, and the parent forms the weights of
eq. (37) and the update of eq. (36) over all samples, in sample order.  The
result equals mppi.iteration / mppi.control_step exactly (a CPU test checks
it).  Only the tests and the benchmark's CPU-baseline leg use this module.
"""

import numpy as np

from . import mppi


def _part(args):
    cfg, x0, U, it, lo, hi = args
    out = mppi.iteration(cfg, x0, U, it, np.arange(lo, hi))
    return out["S"], out["eps"]


def iteration_U(pool, nshards, cfg, x0, U, it):
    """U after one iteration, the samples split into nshards ranges mapped
    over pool (anything with a map method)."""
    K = int(cfg["K"])
    bounds = np.linspace(0, K, nshards + 1).round().astype(int)
    jobs = [(cfg, x0, U, it, int(bounds[i]), int(bounds[i + 1]))
            for i in range(nshards) if bounds[i + 1] > bounds[i]]
    parts = list(pool.map(_part, jobs))
    S = np.concatenate([p[0] for p in parts])
    eps = np.concatenate([p[1] for p in parts])
    w, _, _, status = mppi.weights(S, float(mppi.f32(cfg["lambda"])))
    U = np.asarray(U, dtype=np.float64).reshape(cfg["T"], -1)
    if status != mppi.STATUS_OK:
        return U
    return mppi.update(U, w, eps, float(mppi.f32(cfg.get("alpha", 1.0))))


def control_step(pool, nshards, cfg, x0, U, it0, iters):
    """mppi.control_step with each iteration's samples split over pool."""
    for i in range(iters):
        U = iteration_U(pool, nshards, cfg, x0, U, it0 + i)
    return mppi.shift(U, mppi.f32(cfg["u_init"][:U.shape[1]]))
