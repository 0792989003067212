"""Benchmark of the MPPI-on-jump-diffusion hot path on one MI355X.

Default workload: closed-loop cartpole swing-up MPC, K=4096 samples, T=100
steps, dt=0.02, 5 iterations per control step, receding-horizon shift and a
simulated plant (jumps at 5/s with N(0, 10^2) amplitudes plus N(0, 1) noise)
between control steps.  One bench "step" = one control step = 5 iterations
(sampling, rollout, costs, weights, update) + shift + plant step, all on the
device with the state and disturbances resident in HBM.  value =
rollout-steps/s = K * T * iters * steps / wall time of the timed steps.

Prints one JSON line with, besides the throughput, the per-control-step
latency distribution (HIP events between steps), the dominant kernel's
roofline (the fused rollout; VALU issue bound) and the CPU oracle baseline.
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

# Algorithmic work of one sample-step of the fused rollout (the unit of the
# throughput metric), counted from the method's operations, each weighted by
# the VALU issue slots its gfx950 instruction occupies per lane (full rate = 1;
# 32x32->64 multiply and transcendentals = 4, measured by an instruction-rate
# probe).  Derivation per system in the design notes.
ALG = {
    # cartpole: Philox4x32-10 (20 mul64, 20 xor3-equivalents), Box-Muller
    # (2 cvt, 2 mul, log, sqrt, sin, cos, 3 mul), count compare (6),
    # perturbation (2), cost + IS + Kahan (24), dynamics + Euler (26 incl.
    # sin, cos, rcp)
    1: dict(fp32_flop=61, slots=20 * 4 + 20 + 4 + 4 * 4 + 5 + 6 + 2 + 24 + 23 + 3 * 4),
    # quadrotor: 3 Philox blocks, 4 Box-Muller pairs, cost over 12 states,
    # rigid-body dynamics with 6 sin/cos and 1 rcp
    2: dict(fp32_flop=228, slots=3 * (20 * 4 + 20) + 4 * (4 * 4 + 7) + 9 + 70 + 110 + 7 * 4),
}
VALU_PEAK_SLOTS = 256 * 4 * 16 * 2.4e9    # CUs x SIMDs x lanes x clock
FP32_PEAK_NONPACKED = 78.6e12             # v_fma_f32 on every lane


def cpu_baseline(cfg, x0, U0, iters, budget_s=12.0):
    """Oracle (FP64 NumPy) on a bounded sample of the same closed loop."""
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    from oracle import mppi as omppi
    from oracle import models
    from paper_1807_06108_amd import workloads
    dist = workloads.plant_disturbance(10_000, cfg["dt"], 1.0, cfg["nu"], cfg["sigma_J"][0])
    x = x0.astype(np.float64)
    U = U0.astype(np.float64)
    P = omppi.f32(cfg["params"])
    t0 = time.perf_counter()
    steps = 0
    while True:
        u0, U = omppi.control_step(cfg, x, U, steps * iters, iters)
        x = models.euler_step(cfg["dynamics"], x[None], (u0 + dist[steps])[None],
                              np.zeros((1, 3)), float(omppi.f32(cfg["dt"])), P)[0]
        steps += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return dict(value=cfg["K"] * cfg["T"] * iters * steps / dt, unit="rollout-steps/s",
                cores=1, kind="oracle",
                sample="%d closed-loop control steps of the same workload (%d iterations each), "
                       "%.1f s" % (steps, iters, dt))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="cartpole_mpc",
                    choices=["cartpole_mpc", "cartpole_single", "quadrotor_hover"])
    ap.add_argument("--iters", type=int, default=None)
    ap.add_argument("--schedule", default="auto", choices=["auto", "lane", "ws"],
                    help="rollout schedule (identical results)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the method's data-parallel axis (samples) "
              "fits one MI355X and this build runs no multi-GPU path; use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1807_06108_amd import workloads
    from paper_1807_06108_amd.controller import Controller

    torch.cuda.set_device(0)
    cfg = workloads.PRESETS[args.workload]()
    cfg["schedule"] = {"auto": 0, "lane": 1, "ws": 2}[args.schedule]
    iters = args.iters or (5 if args.workload == "cartpole_mpc" else 1)
    K, T = cfg["K"], cfg["T"]
    n, m = len(workloads.x0_for(cfg)), workloads.DIMS[cfg["dynamics"]][1]
    x0 = workloads.x0_for(cfg)
    U0 = workloads.U0_for(cfg)
    total = args.steps + args.warmup
    dist = np.zeros((total, m), dtype=np.float32)
    if cfg["dynamics"] == 1:
        dist[:, 0] = workloads.plant_disturbance(total, cfg["dt"], 1.0, cfg["nu"], cfg["sigma_J"][0])

    ctl = Controller(cfg, U0)
    x = torch.tensor(x0, device="cuda")
    d = torch.tensor(dist, device="cuda")
    u0 = torch.empty(m, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()

    def control_step(i):
        ctl.step(x, iters)
        ctl.shift(out=u0)
        ctl.plant_step(x, u0, d[i])

    for i in range(args.warmup):
        control_step(i)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    ctl.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(args.steps):
        control_step(args.warmup + i)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctl.profile(False)
    roll_ms, launches = ctl.profile_read()
    lat = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)])
    unit_steps = K * T * iters * args.steps
    value = unit_steps / wall
    avg_roll_s = roll_ms / launches * 1e-3
    alg = ALG[cfg["dynamics"]]
    achieved = alg["slots"] * K * T / avg_roll_s
    flops = alg["fp32_flop"] * K * T / avg_roll_s
    line = {
        "metric": "rollout-steps/sec (K*T*iters), plain per-controller launch",
        "value": value,
        "unit": "rollout-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded Philox draws; seeded plant disturbances)",
        "config": {"workload": args.workload, "K": K, "T": T, "dt": cfg["dt"],
                   "iters_per_control_step": iters, "dynamics": cfg["dynamics"],
                   "nu": cfg["nu"], "form": "plain", "schedule": args.schedule},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "what": "device time per control step (iters + shift + plant)"},
        "roofline": {"bound": "alu", "kernel": "rollout_kernel",
                     "achieved": achieved / 1e12, "peak": VALU_PEAK_SLOTS / 1e12,
                     "unit": "T VALU-slot/s", "frac": achieved / VALU_PEAK_SLOTS,
                     "traffic": None, "avg_launch_us": avg_roll_s * 1e6,
                     "fp32_tflops": flops / 1e12,
                     "fp32_frac_nonpacked": flops / FP32_PEAK_NONPACKED},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(cfg, x0, U0, iters, args.cpu_budget)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
