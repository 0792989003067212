"""Benchmark of the MPPI-on-jump-diffusion hot path on one MI355X.

Default workload (`cartpole_mpc`): closed-loop cartpole swing-up MPC, K=4096
samples, T=100 steps, dt=0.02, 5 iterations per control step, receding-horizon
shift, and a simulated plant (jumps at 5/s with N(0, 10^2) amplitudes plus
N(0, 1) noise) between control steps.  One bench "step" = one control step =
5 iterations (sampling, rollout, costs, weights, update) + shift + plant step,
all on the device with state, control sequence and disturbances resident in
HBM.  value = rollout-steps/s = K * T * iters * steps / wall time of the timed
steps.

The JSON line also carries
  latency_ms       device time per control step (HIP events between steps),
  host_loop_ms     state uploaded -> control step -> u0 downloaded, per control
                   step (PCIe-inclusive; not the value),
  roofline         the rollout kernel (dominant) against the VALU issue peak;
                   its average duration comes from HIP events on its own
                   stream, sampled on every PROFILE_EVERY-th control step of
                   the timed region (events on every launch would perturb it),
  batched          256 uneven controllers advanced by one graph-replayed launch
                   per tick against the same controllers launched one by one,
  serving          1024 resident controllers under Poisson arrivals at 20k
                   MPC-step requests/s: p50/p99 latency (arrival to u0 on the
                   host) of pooled ticks against per-controller launches, and
                   the capacity of each back end,
  saturation       the same rollout at a shape that fills the GPU (K=2^20,
                   lane schedule) per model: the kernel against its roofline
                   where occupancy does not bound it, and the whole iteration
                   (its update a second kernel at this K) against the same
                   peak,
  other_configs    the other single-GPU configurations, each with its value,
                   time per iteration, roofline and oracle timings: the single
                   cartpole iteration (K=256, T=50) and the quadrotor hover
                   iteration (K=8192, T=100),
  cpu_baseline     the FP64 oracle on a bounded sample of the same loop, one
                   thread, with the host's processor, nproc and usable cores,
  cpu_baseline_all_cores
                   the same with each iteration's samples split over the host
                   cores (worker processes, at most 16: the host CPU share of
                   one GPU on the measurement machines).
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

# Algorithmic VALU work of one sample-step (the unit of the throughput
# metric), counted from the method's operations, each weighted by the issue
# slots of the gfx950 instruction that implements it (full rate 1; 32x32->64
# multiply and transcendental 4, as measured by the instruction-rate probe).
# Derivation in the design notes (rollout roofline section).
ALG_SLOTS = {0: 184, 1: 216, 2: 534}
ALG_FP32_FLOP = {0: 37, 1: 68, 2: 228}
# 256 CUs x 128 full-rate lane-slots per CU-clock x 2.4 GHz (measured issue
# rate of v_fma_f32; at 2 FLOP per slot this is the 157.3 TFLOP/s FP32 peak)
VALU_PEAK_SLOTS = 256 * 128 * 2.4e9
FP32_PEAK = 157.3e12
PROFILE_EVERY = 8
CSRC = os.path.join(ROOT, "paper_1807_06108_amd", "csrc")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "rollout_traffic.json")


# sources that define the plain rollout kernels and their launch
# the rollout kernels: one iteration per launch, or a control step's
# iterations in one launch
DOMINANT_KERNELS = ("void mppi::rollout", "void mppi::control_step")
KERNEL_SOURCES = ("kernels.hpp", "rollout_ws.hpp", "rng.hpp", "models.hpp", "reduce.hpp",
                  "mppi_jump.hip")


def source_hash():
    """Digest of the rollout kernel sources (ties counter results to a kernel)."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def progress(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def measured_traffic(workload):
    """HBM bytes per rollout launch from the committed counter runs, if they
    were taken on the current kernel sources (else None)."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != source_hash():
        return None
    w = rec.get("workloads", {}).get(workload)
    return None if w is None else w["bytes_per_launch"]


def cpu_baseline(cfg, x0, U0, iters, dist, budget_s):
    """The oracle (FP64 NumPy, one thread) on a bounded sample of the same
    closed loop: control steps with the same iteration indices and plant."""
    from oracle import models
    from oracle import mppi as omppi
    x = x0.astype(np.float64)
    U = U0.astype(np.float64)
    P = omppi.f32(cfg["params"])
    dt = float(omppi.f32(cfg["dt"]))
    t0 = time.perf_counter()
    steps = 0
    while True:
        u0, U = omppi.control_step(cfg, x, U, steps * iters, iters)
        x = models.euler_step(cfg["dynamics"], x[None], (u0 + dist[steps])[None],
                              np.zeros((1, 3)), dt, P)[0]
        steps += 1
        if time.perf_counter() - t0 > budget_s or steps >= len(dist):
            break
    el = time.perf_counter() - t0
    return dict(value=cfg["K"] * cfg["T"] * iters * steps / el, unit="rollout-steps/s",
                ms_per_control_step=1e3 * el / steps,
                cores=1, kind="oracle", **host_info(),
                sample="%d closed-loop control steps of this workload (%d iterations each, "
                       "K=%d, T=%d), %.1f s, single thread" % (steps, iters, cfg["K"],
                                                               cfg["T"], el))


def host_cpu():
    """Model name of the host processor (lscpu, else /proc/cpuinfo)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_info():
    """The host's processor, its logical CPU count (nproc) and the cores this
    process may use (its affinity set)."""
    return {"cpu": host_cpu(), "nproc": os.cpu_count(),
            "usable_cores": len(os.sched_getaffinity(0))}


# Worker processes of the all-cores oracle timing: the usable cores, at most
# 16, the host CPU share of one GPU on the measurement machines (their nproc
# is larger; host_info reports it).
MAX_CPU_WORKERS = 16


def cpu_iterations(cfg, x0, U0, budget_s, pool=None, workers=1):
    """The oracle on a bounded sample of a single-iteration workload:
    iterations from the same state with fresh iteration indices, each from
    the previous one's sequence, until budget_s has passed; on one thread, or
    with each iteration's samples split over `workers` processes of `pool`."""
    from oracle import mppi as omppi
    from oracle import shards
    x = x0.astype(np.float64)
    U = U0.astype(np.float64)
    t0 = time.perf_counter()
    n = 0
    while True:
        if pool is None:
            U = omppi.iteration(cfg, x, U, n)["U"]
        else:
            U = shards.iteration_U(pool, workers, cfg, x, U, n)
        n += 1
        if time.perf_counter() - t0 > budget_s:
            break
    el = time.perf_counter() - t0
    return dict(value=cfg["K"] * cfg["T"] * n / el, unit="rollout-steps/s",
                ms_per_iteration=1e3 * el / n, cores=workers, kind="oracle",
                sample="%d iterations (K=%d, T=%d), %.1f s, %s" % (
                    n, cfg["K"], cfg["T"], el,
                    "single thread" if pool is None else
                    "samples split over %d worker processes" % workers),
                **host_info())


def oracle_pool(workers):
    """A pool of `workers` fresh interpreter processes with one BLAS thread
    each (started and warmed up outside any timed region)."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    keys = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")
    saved = {k: os.environ.get(k) for k in keys}
    for k in keys:
        os.environ[k] = "1"
    try:
        pool = ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn"))
        list(pool.map(abs, range(workers)))  # start every worker
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    return pool


def cpu_baseline_all_cores(cfg, x0, U0, iters, dist, budget_s, pool, workers):
    """The same oracle with each iteration's samples split over the `workers`
    processes of `pool` (oracle.shards: the parent forms the weights and
    update; results equal the one-thread oracle).  A worker that dies raises
    (BrokenProcessPool) instead of being replaced."""
    from oracle import models, shards
    from oracle import mppi as omppi
    x = x0.astype(np.float64)
    U = U0.astype(np.float64)
    P = omppi.f32(cfg["params"])
    dt = float(omppi.f32(cfg["dt"]))
    t0 = time.perf_counter()
    steps = 0
    while True:
        u0, U = shards.control_step(pool, workers, cfg, x, U, steps * iters, iters)
        x = models.euler_step(cfg["dynamics"], x[None], (u0 + dist[steps])[None],
                              np.zeros((1, 3)), dt, P)[0]
        steps += 1
        if time.perf_counter() - t0 > budget_s or steps >= len(dist):
            break
    el = time.perf_counter() - t0
    return dict(value=cfg["K"] * cfg["T"] * iters * steps / el, unit="rollout-steps/s",
                ms_per_control_step=1e3 * el / steps,
                cores=workers, kind="oracle", **host_info(),
                sample="%d closed-loop control steps of this workload, each iteration's "
                       "K=%d samples split over %d worker processes, %.1f s"
                       % (steps, cfg["K"], workers, el))


def iteration_measure(name, calls, warmup, **over):
    """One plain-form controller of a preset single-iteration workload
    (fields overridden by `over`): `calls` iterations (the rollout kernel
    timed by HIP events on its stream around every launch) from the preset
    state, each from the previous one's sequence.  Returns the workload's
    sub-object of the line (its cpu_baseline legs are added by the caller)."""
    import torch
    from paper_1807_06108_amd import workloads
    from paper_1807_06108_amd.controller import Controller
    cfg = workloads.PRESETS[name](**over)
    K, T, dyn = cfg["K"], cfg["T"], cfg["dynamics"]
    ctl = Controller(cfg, workloads.U0_for(cfg))
    x = torch.tensor(workloads.x0_for(cfg), device="cuda")
    for _ in range(warmup):
        ctl.step(x, 1)
    torch.cuda.synchronize()
    ctl.profile(True)
    t0 = time.perf_counter()
    for _ in range(calls):
        ctl.step(x, 1)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctl.profile(False)
    roll_ms, launches, _ = ctl.profile_read()
    avg_roll_s = roll_ms / launches * 1e-3
    achieved = ALG_SLOTS[dyn] * K * T / avg_roll_s
    flops = ALG_FP32_FLOP[dyn] * K * T / avg_roll_s
    return {"workload": name, "K": K, "T": T, "dt": cfg["dt"], "dynamics": dyn, "nu": cfg["nu"],
            "schedule": {0: "auto", 1: "lane", 2: "ws"}[cfg.get("schedule", 0)],
            "iterations": calls, "value": K * T * calls / wall, "unit": "rollout-steps/s",
            "ms_per_iteration": wall / calls * 1e3,
            "roofline": {"bound": "alu",
                         "kernel": "rollout (sampling, propagation, cost, weights, update)",
                         "achieved": achieved / 1e12, "peak": VALU_PEAK_SLOTS / 1e12,
                         "unit": "T VALU-slot/s", "frac": achieved / VALU_PEAK_SLOTS,
                         "traffic": measured_traffic(name) if not over else None,
                         "avg_launch_us": avg_roll_s * 1e6, "launches_timed": launches,
                         "slots_per_sample_step": ALG_SLOTS[dyn],
                         "fp32_tflops": flops / 1e12, "fp32_frac": flops / FP32_PEAK,
                         # the same slots over the whole iteration (every
                         # kernel of it, wall clock): where the update runs
                         # as a kernel of its own, this is the figure to read
                         "iteration_frac": ALG_SLOTS[dyn] * K * T * calls / wall / VALU_PEAK_SLOTS}}


def batched_measure(n_ctl, ticks, warmup, seed=42):
    """Batched form against plain per-controller launches on the same
    controller set (half cartpole, half quadrotor, K in {512..8192}, T in
    [30, 150], nu in [0, 10]/s): one tick = one iteration + shift of every
    controller from its own state.  The batched tick is one graph replay of
    the layout the autotuner measured fastest (schedule, grid or persistent
    launch, one kernel or one per model on its own stream); the plain tick is
    n_ctl control-step launches in sequence."""
    import torch
    from paper_1807_06108_amd import autotune, workloads
    from paper_1807_06108_amd.controller import Controller
    cset = workloads.random_controllers(n_ctl, seed=seed)
    cfgs = [c for c, _ in cset]
    states = [torch.tensor(x, device="cuda") for _, x in cset]
    work = sum(c["K"] * c["T"] for c in cfgs)
    stream = torch.cuda.current_stream()

    def timed(fn, n):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(n + 1)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev[0].record(stream)
        for i in range(n):
            fn()
            ev[i + 1].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        lat = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(n)])
        return dict(value=work * n / wall, unit="rollout-steps/s", ms_per_tick=wall / n * 1e3,
                    mean_ms=float(lat.mean()), p50_ms=float(np.percentile(lat, 50)),
                    p99_ms=float(np.percentile(lat, 99)))

    ctls, batch, report = autotune.build_batch(cfgs, states)
    for _ in range(warmup):
        batch.step(iters=1, shift=True)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        batch.step(iters=1, shift=True)
    torch.cuda.synchronize()
    batched = timed(g.replay, ticks)
    plain_ctls = [Controller(dict(c, schedule=0)) for c in cfgs]
    u0 = torch.empty(4, device="cuda")

    def plain_tick():
        for c, x in zip(plain_ctls, states):
            c.control_step(x, 1, u0)
    for _ in range(warmup):
        plain_tick()
    plain = timed(plain_tick, ticks)
    # VALU issue of one tick against the chip's peak (the per-sample-step
    # slot counts of each controller's model), over the tick's device time
    # (HIP events on the replay stream around every replay, averaged)
    slots = sum(ALG_SLOTS[c["dynamics"]] * c["K"] * c["T"] for c in cfgs)
    achieved = slots / (batched["mean_ms"] * 1e-3)
    return {"controllers": n_ctl, "rollout_steps_per_tick": work,
            "layout": report["plan"], "autotune_ms_per_tick": report["timings_ms"],
            "batched_graph": batched, "plain_sequential": plain,
            "speedup": batched["value"] / plain["value"],
            "roofline": {"bound": "alu", "achieved": achieved / 1e12,
                         "peak": VALU_PEAK_SLOTS / 1e12, "unit": "T VALU-slot/s",
                         "frac": achieved / VALU_PEAK_SLOTS,
                         "what": "issue slots of every controller's sample-steps per tick / mean "
                                 "device time of a tick (HIP events around each graph replay)"}}


def serving_measure(rate, seconds, warm, n_ctl=1024, seed=4):
    """Serving form against plain per-controller launches under the same
    request stream: n_ctl resident controllers (half cartpole, half
    quadrotor, K in {1024..8192}, T in [50, 150]), Poisson arrivals at `rate`
    requests/s, each one MPC step (1 iteration + shift) from the
    controller's own plant state, plant stepped on the device.  Latency is
    arrival to u_0 on the host.  Then the capacity of each back end: the
    throughput it sustains under an offered rate above it."""
    from paper_1807_06108_amd import autotune, serving, workloads
    cs = workloads.serving_controllers(n_ctl, seed=seed)
    cfgs = [c for c, _ in cs]
    x0s = [x for _, x in cs]
    dist = [workloads.serving_disturbances(c, 256, seed=2000 + i) for i, c in enumerate(cfgs)]
    import torch
    sched, report = autotune.choose_schedule(
        cfgs, [torch.tensor(x, device="cuda") for x in x0s], subset=4)

    def run(backend, schedule, r, secs, w, cap=64 << 30):
        t, ids = workloads.serving_arrivals(r, secs + w, n_ctl, seed=9)
        srv = serving.Server(cfgs, x0s, dist, hbm_cap_bytes=cap, max_inflight=4,
                             backend=backend, schedule=schedule)
        res = srv.run(t, ids, warmup_s=w)
        res.update(admitted=len(srv.admitted), resident_gb_at_end=srv.resident_bytes / 2**30)
        srv.close()
        torch.cuda.synchronize()
        return res

    out = {"controllers": n_ctl, "rate_per_s": rate, "measured_s": seconds, "warmup_s": warm,
           "hbm_cap_gb": 64, "schedule": {1: "lane", 2: "ws"}[int(sched)],
           "autotune_ms": report["timings_ms"]}
    progress("serving: pooled ticks at %.0f requests/s" % rate)
    out["pool"] = run("pool", sched, rate, seconds, warm)
    progress("serving: per-controller launches at %.0f requests/s" % rate)
    out["plain"] = run("plain", sched, rate, seconds, warm)
    out["p99_ratio_plain_over_pool"] = out["plain"]["latency_ms"]["p99"] / out["pool"]["latency_ms"]["p99"]
    # a cap that holds about a quarter of the controllers' workspaces:
    # requests wait for admission, idle residents are evicted (state saved on
    # the host) and rebuilt on their next request.  Three quarters of the
    # requests then need an admission, which is host work, so the offered
    # rate is a tenth of the one above.
    total = sum(serving.footprint_bytes(c) for c in cfgs)
    bounded, b_rate, b_secs = total // 4, rate / 10, min(seconds, 3.0)
    progress("serving: pooled ticks under a %.2f GiB residency cap, %.0f requests/s"
             % (bounded / 2**30, b_rate))
    out["pool_bounded"] = dict(run("pool", sched, b_rate, b_secs, 1.0, cap=bounded),
                               offered_per_s=b_rate, hbm_cap_gb=bounded / 2**30,
                               workspaces_gb=total / 2**30)
    cap = {}
    for name, backend, schedule, offered in (("pool_lane", "pool", 1, 300e3),
                                             ("pool_ws", "pool", 2, 250e3),
                                             ("plain", "plain", sched, 40e3)):
        progress("serving capacity: %s" % name)
        r = run(backend, schedule, offered, 1.0, 0.5)
        cap[name] = {"offered_per_s": offered, "requests_per_s": r["requests_per_s"],
                     "rollout_steps_per_s": r["rollout_steps_per_s"],
                     "mean_tick_requests": r["mean_tick_requests"],
                     "latency_p50_ms": r["latency_ms"]["p50"]}
    out["capacity"] = cap
    return out


def counter_per_dispatch(csv_dir, counter, kernel_prefix):
    """(mean value per dispatch, dispatches) of one rocprofv3 counter over
    the dispatches of kernels whose name starts with kernel_prefix (a string
    or a tuple of them), from the
    *counter_collection.csv files under csv_dir."""
    import csv
    import glob
    vals = {}
    for path in glob.glob(os.path.join(csv_dir, "**", "*counter_collection.csv"), recursive=True):
        with open(path) as f:
            for row in csv.DictReader(f):
                name = row.get("Kernel_Name", "")
                if row.get("Counter_Name") != counter or not name.startswith(kernel_prefix):
                    continue
                key = (path, row.get("Dispatch_Id"))
                vals[key] = vals.get(key, 0.0) + float(row["Counter_Value"])
    if not vals:
        raise ValueError("no %s dispatches of %s under %s" % (counter, kernel_prefix, csv_dir))
    return sum(vals.values()) / len(vals), len(vals)


def traffic_summary(pmc_dir, workloads):
    """HBM bytes per rollout launch from FETCH_SIZE and WRITE_SIZE runs (KiB
    per dispatch), each scaled by what the same counter reads for the copy
    of known size (bench.py --calibrate-copy).  Expects pmc_dir/<counter>_copy
    and pmc_dir/<counter>_<workload> for both counters."""
    copy_bytes = 256 << 20
    # the copy dispatches of calibrate_copy (its fill kernel excluded)
    copy_kernel = "__amd_rocclr_copyBuffer"
    cf, _ = counter_per_dispatch(os.path.join(pmc_dir, "FETCH_SIZE_copy"), "FETCH_SIZE",
                                 copy_kernel)
    cw, _ = counter_per_dispatch(os.path.join(pmc_dir, "WRITE_SIZE_copy"), "WRITE_SIZE",
                                 copy_kernel)
    fetch_scale, write_scale = copy_bytes / (cf * 1024), copy_bytes / (cw * 1024)
    out = {"source_hash": source_hash(),
           "what": "HBM bytes per launch of the rollout kernel: rocprofv3 FETCH_SIZE and "
                   "WRITE_SIZE (KiB per dispatch), each scaled by the reading of the same "
                   "counter for a 256 MiB device-to-device copy",
           "copy_calibration": {"bytes": copy_bytes, "FETCH_SIZE_kib": cf, "WRITE_SIZE_kib": cw,
                                "fetch_scale": fetch_scale, "write_scale": write_scale},
           "workloads": {}}
    for w in workloads:
        f, nf = counter_per_dispatch(os.path.join(pmc_dir, "FETCH_SIZE_" + w), "FETCH_SIZE",
                                     DOMINANT_KERNELS)
        wr, nw = counter_per_dispatch(os.path.join(pmc_dir, "WRITE_SIZE_" + w), "WRITE_SIZE",
                                      DOMINANT_KERNELS)
        out["workloads"][w] = {"FETCH_SIZE_kib": f, "WRITE_SIZE_kib": wr, "dispatches": [nf, nw],
                               "bytes_per_launch": 1024 * (f * fetch_scale + wr * write_scale)}
    return out


def calibrate_copy(nbytes=256 << 20, reps=4):
    """A plain device copy of known size, for scaling the HBM byte counters."""
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_bytes": nbytes, "launches": reps}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="cartpole_mpc",
                    choices=["cartpole_mpc", "cartpole_single", "quadrotor_hover"])
    ap.add_argument("--iters", type=int, default=None)
    ap.add_argument("--K", type=int, default=None, help="override the preset's sample count")
    ap.add_argument("--T", type=int, default=None, help="override the preset's horizon")
    ap.add_argument("--schedule", default="auto", choices=["auto", "lane", "ws"],
                    help="rollout schedule (identical results)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--iteration-calls", type=int, default=300,
                    help="iterations timed on each other single-GPU configuration "
                         "(cartpole K=256 T=50, quadrotor K=8192 T=100); 0 skips them")
    ap.add_argument("--saturation-calls", type=int, default=10,
                    help="iterations timed at the saturating shape K=2^20 (lane schedule) of "
                         "each model; 0 skips them")
    ap.add_argument("--cpu-workers", type=int, default=None,
                    help="worker processes of the all-cores oracle timing (default: the "
                         "usable host cores, at most 16; 0 skips it)")
    ap.add_argument("--host-loop-steps", type=int, default=100)
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--traffic-summary", metavar="PMC_DIR",
                    help="print the HBM bytes per rollout launch from the FETCH_SIZE / "
                         "WRITE_SIZE counter runs under PMC_DIR (no GPU needed)")
    ap.add_argument("--batched-controllers", type=int, default=256)
    ap.add_argument("--batched-ticks", type=int, default=20,
                    help="0 skips the batched-form comparison")
    ap.add_argument("--serving-seconds", type=float, default=10.0,
                    help="measured seconds of the serving comparison (0 skips it)")
    ap.add_argument("--serving-warmup", type=float, default=2.0)
    ap.add_argument("--serving-rate", type=float, default=20000.0)
    args = ap.parse_args()
    if args.traffic_summary:
        print(json.dumps(traffic_summary(args.traffic_summary,
                                         ("cartpole_mpc", "cartpole_single", "quadrotor_hover")),
                         indent=1))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the method's parallel axis (samples) fits one "
              "MI355X and no multi-GPU path is built; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1807_06108_amd import workloads
    from paper_1807_06108_amd.controller import Controller

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        calibrate_copy()
        return
    cfg = workloads.PRESETS[args.workload]()
    cfg["schedule"] = {"auto": 0, "lane": 1, "ws": 2}[args.schedule]
    if args.K:
        cfg["K"] = args.K
    if args.T:
        cfg["T"] = args.T
    iters = args.iters or (5 if args.workload == "cartpole_mpc" else 1)
    K, T, dyn = cfg["K"], cfg["T"], cfg["dynamics"]
    n, m, q = workloads.DIMS[dyn]
    x0 = workloads.x0_for(cfg)
    U0 = workloads.U0_for(cfg)
    total = args.steps + args.warmup + args.host_loop_steps
    dist = np.zeros((total, m), dtype=np.float32)
    if dyn == 1:
        dist[:, 0] = workloads.plant_disturbance(total, cfg["dt"], 1.0, cfg["nu"],
                                                 cfg["sigma_J"][0])

    stream = torch.cuda.current_stream()
    ctl = Controller(cfg, U0)
    x = torch.tensor(x0, device="cuda")
    d = torch.tensor(dist, device="cuda")
    u0 = torch.empty(m, dtype=torch.float32, device="cuda")

    def control_step(i):
        ctl.control_step(x, iters, u0)
        ctl.plant_step(x, u0, d[i])

    for i in range(args.warmup):
        control_step(i)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(args.steps):
        prof = i % PROFILE_EVERY == 0
        if prof:
            ctl.profile(True)
        control_step(args.warmup + i)
        if prof:
            ctl.profile(False)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    roll_ms, launches, roll_iters = ctl.profile_read()
    lat = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)])

    # host in the loop: state uploaded, control step, u0 downloaded (timed);
    # the plant then steps on the device and the state comes back (untimed)
    host_lat = []
    x_host = torch.empty(n, dtype=torch.float32, pin_memory=True)
    u0_host = torch.empty(m, dtype=torch.float32, pin_memory=True)
    x_host.copy_(x)
    for i in range(args.host_loop_steps):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        x.copy_(x_host, non_blocking=True)
        ctl.control_step(x, iters, u0)
        u0_host.copy_(u0, non_blocking=True)
        torch.cuda.synchronize()
        host_lat.append((time.perf_counter() - t1) * 1e3)
        ctl.plant_step(x, u0, d[args.warmup + args.steps + i])
        x_host.copy_(x)

    value = K * T * iters * args.steps / wall
    # the dominant kernel: one launch per control step (all its iterations)
    # or one per iteration; its algorithmic work per launch is that of the
    # iterations it runs
    avg_roll_s = roll_ms / launches * 1e-3
    per_launch = roll_iters / launches
    achieved = ALG_SLOTS[dyn] * K * T * per_launch / avg_roll_s
    flops = ALG_FP32_FLOP[dyn] * K * T * per_launch / avg_roll_s
    line = {
        "metric": "rollout-steps/sec (K*T*iters) + p99 MPC-step latency, plain "
                  "per-controller launch",
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
        "data": "synthetic (seeded Philox draws, seeded plant disturbances)",
        "config": {"workload": args.workload, "K": K, "T": T, "dt": cfg["dt"],
                   "iters_per_control_step": iters, "dynamics": dyn, "nu": cfg["nu"],
                   "form": "plain", "schedule": args.schedule},
        "latency_ms": {"p50": float(np.percentile(lat, 50)),
                       "p99": float(np.percentile(lat, 99)),
                       "what": "device time per control step (iterations + shift + plant)"},
        "host_loop_ms": ({"p50": float(np.percentile(host_lat, 50)),
                          "p99": float(np.percentile(host_lat, 99)), "steps": len(host_lat),
                          "what": "state host->device, control step, u0 device->host, "
                                  "synchronise"} if host_lat else None),
        "roofline": {"bound": "alu",
                     "kernel": ("control step, %d iterations in one launch (sampling, "
                                "propagation, cost, weights, update, shift)" % per_launch
                                if per_launch > 1 else
                                "rollout (sampling, propagation, cost, weights, update)"),
                     "achieved": achieved / 1e12, "peak": VALU_PEAK_SLOTS / 1e12,
                     "unit": "T VALU-slot/s", "frac": achieved / VALU_PEAK_SLOTS,
                     "traffic": (measured_traffic(args.workload)
                                 if args.K is None and args.T is None else None),
                     "avg_launch_us": avg_roll_s * 1e6, "launches_timed": launches,
                     "iterations_per_launch": per_launch,
                     "slots_per_sample_step": ALG_SLOTS[dyn],
                     "fp32_tflops": flops / 1e12, "fp32_frac": flops / FP32_PEAK},
    }
    progress("plain form done: %.4f ms per control step" % (wall / args.steps * 1e3))
    if args.batched_ticks > 0:
        progress("batched form")
        line["batched"] = batched_measure(args.batched_controllers, args.batched_ticks, 3)
    if args.serving_seconds > 0:
        progress("serving form (about %.0f s)" % (2 * (args.serving_seconds + args.serving_warmup) + 15))
        line["serving"] = serving_measure(args.serving_rate, args.serving_seconds,
                                          args.serving_warmup)
    # the other single-GPU configurations: the single cartpole iteration
    # (K=256, T=50) and the quadrotor hover iteration (K=8192, T=100)
    others = []
    if args.iteration_calls > 0 and args.K is None and args.T is None:
        for name in ("cartpole_single", "quadrotor_hover"):
            if name != args.workload:
                progress("plain form: %s" % name)
                others.append(iteration_measure(name, args.iteration_calls, 20))
        line["other_configs"] = others
    # saturating shapes: one controller of 2^20 samples (4096 lane-schedule
    # workgroups fill every compute unit several times over; the update then
    # runs as its own HBM-bound kernel), per model
    if args.saturation_calls > 0 and args.K is None and args.T is None:
        line["saturation"] = []
        for name in ("cartpole_mpc", "quadrotor_hover"):
            progress("saturating shape: %s, K=2^20" % name)
            line["saturation"].append(iteration_measure(name, args.saturation_calls, 2,
                                                        K=1 << 20, schedule=1))
    if not args.no_cpu_baseline:
        progress("oracle on one host core (about %.0f s)" % args.cpu_budget)
        line["cpu_baseline"] = cpu_baseline(cfg, x0, U0, iters,
                                            dist[args.warmup:].astype(np.float64),
                                            args.cpu_budget)
        from paper_1807_06108_amd import workloads as wl
        for o in others:
            c = wl.PRESETS[o["workload"]]()
            progress("oracle on one host core: %s (about %.0f s)" % (o["workload"],
                                                                    args.cpu_budget / 2))
            o["cpu_baseline"] = cpu_iterations(c, wl.x0_for(c), wl.U0_for(c),
                                               args.cpu_budget / 2)
        workers = args.cpu_workers
        if workers is None:
            workers = min(MAX_CPU_WORKERS, len(os.sched_getaffinity(0)))
        if workers > 1:
            try:
                pool = oracle_pool(workers)
            except Exception as e:  # the GPU figures stand without it
                pool = None
                line["cpu_baseline_all_cores"] = {"error": repr(e)}
            if pool is not None:
                with pool:
                    progress("oracle on %d host cores (about %.0f s)" % (workers,
                                                                         args.cpu_budget / 2))
                    try:
                        line["cpu_baseline_all_cores"] = cpu_baseline_all_cores(
                            cfg, x0, U0, iters, dist[args.warmup:].astype(np.float64),
                            args.cpu_budget / 2, pool, workers)
                        for o in others:
                            c = wl.PRESETS[o["workload"]]()
                            progress("oracle on %d host cores: %s" % (workers, o["workload"]))
                            o["cpu_baseline_all_cores"] = cpu_iterations(
                                c, wl.x0_for(c), wl.U0_for(c), args.cpu_budget / 3, pool, workers)
                    except Exception as e:
                        line["cpu_baseline_all_cores"] = {"error": repr(e)}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
