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
"""

import argparse
import ctypes
import sys

import numpy as np

SLOTS, LAUNCHES, MAX_WG = 16, 8, 256
TICK_US = 0.01  # the real-time counter runs at 100 MHz


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="cartpole_mpc")
    ap.add_argument("--iters", type=int, default=None,
                    help="iterations per control step (default: 5 for cartpole_mpc, else 3)")
    ap.add_argument("--reps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=30)
    args = ap.parse_args(argv)

    # torch first: the library then binds to the HIP runtime torch loaded
    import torch

    from . import build, native, workloads
    from .controller import Controller
    native.use_library(build.PHASE_LIB)
    L = native.lib()
    L.mppi_phase_read.restype = ctypes.c_int
    L.mppi_phase_read.argtypes = [ctypes.c_void_p, ctypes.c_size_t]

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


if __name__ == "__main__":
    sys.exit(main())
