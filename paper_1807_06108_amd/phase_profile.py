"""Phase timeline of the wave-specialised rollout kernel, from the
phase-profiling build of the library (libmppi_jump_phases.so, the same
sources with per-workgroup timestamps compiled in; include/mppi_jump_phases.h).

One control step of a preset workload (its iterations are back-to-back
launches of the one-iteration kernel, the last one with the shift) is run
`reps` times after a warm-up; per launch the tool reports, as the median over
the repetitions, in microseconds from the first workgroup start of the first
launch:

  start     first .. last workgroup start,
  first chunk  the last consumer wavefront to start its recursion (the
            constants, U and the first ring chunk ready),
  rollout   the last workgroup to finish its rollout (all costs known),
  publish   the last workgroup to have stored its partials (statistics and,
            fused, the weighted perturbation sums of eq. (37)),
  arrival   the last workgroup to have counted its arrival (release fence
            and atomic),
  acquire   the combining (last) workgroup past its acquire fence,
  combine   the combining workgroup done with eq. (37)'s combine and
            the eq. (36) update,
  end       the combining workgroup done with the shift (last launch),
and the phase lengths: to the first chunk (from the first workgroup start),
the rollout loop, publish, arrival, acquire, combine, shift and record, and
the gap from the end of one launch to the first workgroup start of the
next.

    python -m paper_1807_06108_amd.phase_profile --workload cartpole_mpc

With --batched N it profiles instead the batched form's grid launch over N
mixed controllers (random_controllers, lane schedule): each tile's start and
end, hence how many tiles are resident over the tick, the mean of that over
the tick, the tail where it falls below 90 % of its peak, and each model's
tile time per horizon step.

    python -m paper_1807_06108_amd.phase_profile --batched 256
"""

import argparse
import ctypes
import sys

import numpy as np

SLOTS, LAUNCHES, MAX_WG, TILES = 16, 8, 256, 8192
TICK_US = 0.01  # the real-time counter runs at 100 MHz


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="cartpole_mpc")
    ap.add_argument("--iters", type=int, default=None,
                    help="iterations per control step (default: 5 for cartpole_mpc, else 3)")
    ap.add_argument("--reps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--batched", type=int, default=0,
                    help="profile the batched grid launch over this many controllers instead")
    args = ap.parse_args(argv)

    # torch first: the library then binds to the HIP runtime torch loaded
    import torch

    from . import build, native, workloads
    from .controller import Controller
    native.use_library(build.PHASE_LIB)
    L = native.lib()
    L.mppi_phase_read.restype = ctypes.c_int
    L.mppi_phase_read.argtypes = [ctypes.c_void_p, ctypes.c_size_t]
    if args.batched:
        return batched(args, L, torch)

    cfg = dict(workloads.PRESETS[args.workload](), schedule=native.C["MPPI_SCHED_WAVE_SPECIALISED"])
    iters = args.iters or (5 if args.workload == "cartpole_mpc" else 3)
    if iters > LAUNCHES:
        raise SystemExit("at most %d iterations per control step are recorded" % LAUNCHES)
    nwg = (cfg["K"] + 63) // 64
    if nwg > MAX_WG:
        raise SystemExit("at most %d workgroups are recorded" % MAX_WG)
    ctl = Controller(cfg, workloads.U0_for(cfg))
    x = torch.tensor(workloads.x0_for(cfg), device="cuda")
    for _ in range(args.warmup):
        ctl.control_step(x, iters)
    torch.cuda.synchronize()
    buf = np.zeros(LAUNCHES * MAX_WG * SLOTS, dtype=np.uint64)
    runs = []
    for _ in range(args.reps):
        it0 = ctl.stats()["iteration"]
        ctl.control_step(x, iters)
        torch.cuda.synchronize()
        rc = L.mppi_phase_read(buf.ctypes.data, buf.size)
        if rc != 0:
            raise RuntimeError("mppi_phase_read: %d" % rc)
        rec = buf.reshape(LAUNCHES, MAX_WG, SLOTS)[:, :nwg].astype(np.int64)
        t0 = rec[it0 % LAUNCHES, :, 0].min()
        rows = []
        for i in range(iters):
            a = rec[(it0 + i) % LAUNCHES]
            last = np.flatnonzero(a[:, 6] == 1)
            if len(last) != 1:
                raise RuntimeError("launch %d: %d combining workgroups recorded" % (i, len(last)))
            j = last[0]
            rows.append([a[:, 0].min(), a[:, 0].max(), a[:, 1].max(), a[:, 2].max(),
                         a[:, 3].max(), a[j, 4], a[j, 5], a[:, 7].max(), a[j, 8]])
        runs.append((np.array(rows, dtype=np.float64) - t0) * TICK_US)
    m = np.median(np.stack(runs), axis=0)

    print("# Phases of the rollout kernel: %s (K=%d, T=%d, %d workgroups, %d iterations per "
          "control step)\n" % (args.workload, cfg["K"], cfg["T"], nwg, iters))
    print("Median of %d control steps, us from the first workgroup start of the first launch.\n"
          % args.reps)
    print("| launch | start | first chunk | rollout | publish | arrival | acquire | combine | end |")
    print("|---|---|---|---|---|---|---|---|---|")
    for i in range(iters):
        r = m[i]
        print("| %d | %.2f..%.2f | %.2f | %.2f | %.2f | %.2f | %.2f | %.2f | %.2f |" % (
            i, r[0], r[1], r[7], r[2], r[3], r[4], r[8], r[5], r[6]))
    print("\nPhase lengths (us), mean over the launches:\n")
    start = m[:, 7] - m[:, 0]
    loop = m[:, 2] - m[:, 7]
    pub = m[:, 3] - m[:, 2]
    arr = m[:, 4] - m[:, 3]
    acq = m[:, 8] - m[:, 4]
    comb = m[:, 5] - m[:, 8]
    tail = m[:, 6] - m[:, 5]
    gap = m[1:, 0] - m[:-1, 6]
    total = (m[-1, 6] - m[0, 0]) / iters
    print("| to first chunk | rollout loop | publish | arrival | acquire | combine | shift / record "
          "| gap to next launch | per launch |")
    print("|---|---|---|---|---|---|---|---|---|")
    print("| %.2f | %.2f | %.2f | %.2f | %.2f | %.2f | %.2f | %.2f | %.2f |" % (
        start.mean(), loop.mean(), pub.mean(), arr.mean(), acq.mean(), comb.mean(), tail.mean(),
        gap.mean() if len(gap) else float("nan"), total))
    return 0


def batched(args, L, torch):
    """Tile timeline of the batched form's grid launch."""
    from . import autotune, workloads
    L.mppi_phase_read_tiles.restype = ctypes.c_int
    L.mppi_phase_read_tiles.argtypes = [ctypes.c_void_p, ctypes.c_size_t]
    cset = workloads.random_controllers(args.batched, seed=42)
    cfgs = [c for c, _ in cset]
    states = [torch.tensor(x, device="cuda") for _, x in cset]
    _, b = autotune.make_batch(cfgs, states, (autotune.LANE, autotune.GRID, False))
    for _ in range(5):
        b.step(iters=1, shift=True)
    torch.cuda.synchronize()
    buf = np.zeros(TILES * 2, dtype=np.uint64)
    spans, means, tails, ideal, per_step = [], [], [], [], {1: [], 2: []}
    order = tile_order(cfgs)
    if len(order) > TILES:
        raise SystemExit("at most %d tiles are recorded" % TILES)
    for _ in range(args.reps):
        b.step(iters=1, shift=True)
        torch.cuda.synchronize()
        rc = L.mppi_phase_read_tiles(buf.ctypes.data, buf.size)
        if rc != 0:
            raise RuntimeError("mppi_phase_read_tiles: %d" % rc)
        r = buf.reshape(TILES, 2)[:len(order)].astype(np.int64)
        st = (r[:, 0] - r[:, 0].min()) * TICK_US
        en = (r[:, 1] - r[:, 0].min()) * TICK_US
        span = en.max()
        grid = np.linspace(0.0, span, 201)[1:-1]
        conc = np.array([((st <= t) & (en > t)).sum() for t in grid])
        spans.append(span)
        means.append((en - st).sum() / span)
        tails.append(span * (conc < 0.9 * conc.max()).mean())
        ideal.append((en - st).sum() / conc.max())
        dur = en - st
        for d in (1, 2):
            m = np.array([cfgs[c]["dynamics"] == d for c in order])
            T = np.array([cfgs[c]["T"] for c in order])
            per_step[d].append(np.median(dur[m] / T[m]))
        peak = conc.max()
    work = sum(c["K"] * c["T"] for c in cfgs)
    print("# Tile timeline of the batched grid launch: %d controllers (random_controllers, seed 42, "
          "lane schedule), %d tiles, %.3g sample-steps per tick\n" % (len(cfgs), len(order), work))
    print("Median over %d ticks (us; tile start and end by thread 0 of each tile).\n" % args.reps)
    print("| tick span | peak resident tiles | mean resident tiles | summed tile time / peak "
          "| time below 90 % of peak | cartpole tile time per step | quadrotor tile time per step |")
    print("|---|---|---|---|---|---|---|")
    print("| %.1f | %d | %.1f | %.1f | %.1f | %.3f | %.3f |" % (
        np.median(spans), peak, np.median(means), np.median(ideal), np.median(tails),
        np.median(per_step[1]), np.median(per_step[2])))
    b.close()
    return 0


def tile_order(cfgs):
    """Controller of every tile in launch order: controllers longest first
    (tile cost K-independent per tile: T times the model's issue slots per
    sample-step), each with its ceil(K / 256) lane-schedule tiles."""
    cost = {0: 184, 1: 216, 2: 534}
    idx = sorted(range(len(cfgs)), key=lambda i: -cfgs[i]["T"] * cost[cfgs[i]["dynamics"]])
    return [i for i in idx for _ in range((cfgs[i]["K"] + 255) // 256)]


if __name__ == "__main__":
    sys.exit(main())
