"""Schedule autotuner for the batched and serving forms.

A batch can be laid out on the GPU in several ways that give the same
results: the rollout schedule of its tiles (one sample per lane, 256 samples
per workgroup; or wave-specialised, 64 samples per workgroup), the launch
(one workgroup per tile under the hardware dispatcher, or resident
workgroups taking tiles from a device work queue), and whether the
controllers share one kernel or run one sub-batch per model (each sub-batch's
kernel holds only that model's variants and has its own stream, the
sub-batches overlapping on the device).  Which is fastest depends on the mix
of K, T and models and on how many controllers share the GPU, so the choice
is measured, not guessed: every candidate is built on the caller's
controller set, timed over a few warm ticks on the device, and the fastest
is kept.  Decisions are cached per batch signature (model mix and (K, T)
multiset), so a serving loop pays the measurement once per distinct shape.
"""

import hashlib
import json

import torch

from . import native
from .controller import Batch, BatchGroup, Controller

LANE = native.C["MPPI_SCHED_LANE"]
WS = native.C["MPPI_SCHED_WAVE_SPECIALISED"]
GRID = native.C["MPPI_BATCH_GRID"]
PERSISTENT = native.C["MPPI_BATCH_PERSISTENT"]

# schedules timed for a serving pool (its ticks are grid launches)
CANDIDATES = (LANE, WS)

# layouts of a batch: (rollout schedule, launch, one sub-batch per model)
PLANS = (
    (LANE, GRID, False),
    (LANE, PERSISTENT, False),
    (WS, GRID, False),
    (WS, PERSISTENT, False),
    (LANE, GRID, True),
    (LANE, PERSISTENT, True),
)
_cache = {}
_plan_cache = {}


def signature(cfgs):
    """Shape signature of a controller set (order independent)."""
    key = sorted((c["dynamics"], c["K"], c["T"], c.get("cost_form", 0), c["nu"] > 0) for c in cfgs)
    return hashlib.sha1(json.dumps(key).encode()).hexdigest()[:16]


def plan_name(plan):
    sched, launch, split = plan
    return "%s-%s%s" % ("lane" if sched == LANE else "ws",
                        "grid" if launch == GRID else "persistent", "-per-model" if split else "")


def _time_batch(batch, ticks, warmup, stream):
    for _ in range(warmup):
        batch.step(iters=1, shift=True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(ticks):
        batch.step(iters=1, shift=True)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / ticks


def _subset(cfgs, states, subset, seed):
    if subset is not None and subset < len(cfgs):
        import numpy as np
        pick = np.random.default_rng(seed).choice(len(cfgs), size=subset, replace=False)
        return [cfgs[i] for i in pick], [states[i] for i in pick]
    return cfgs, states


def make_batch(cfgs, states, plan, U0s=None):
    """Controllers for cfgs laid out by `plan` and the object that steps them
    (a Batch, or a BatchGroup of one Batch per model on its own stream).
    Returns (controllers in the order of cfgs, stepper)."""
    sched, launch, split = plan
    ctls = [Controller(dict(c, schedule=sched), None if U0s is None else U0s[i])
            for i, c in enumerate(cfgs)]
    if not split:
        return ctls, Batch(ctls, states, launch=launch)
    groups = {}
    for i, c in enumerate(cfgs):
        groups.setdefault(c["dynamics"], []).append(i)
    if len(groups) < 2:
        raise ValueError("one model only: nothing to split")
    batches = [Batch([ctls[i] for i in idx], [states[i] for i in idx], stream=torch.cuda.Stream(),
                     launch=launch) for _, idx in sorted(groups.items())]
    return ctls, BatchGroup(batches)


def choose_plan(cfgs, states, plans=PLANS, ticks=3, warmup=1, subset=None, seed=0):
    """The fastest measured layout (schedule, launch, per-model split) for
    cfgs (cached per signature) and a report of the timings in ms per tick."""
    cfgs, states = _subset(cfgs, states, subset, seed)
    sig = signature(cfgs)
    report = {"signature": sig, "timings_ms": {}, "controllers_timed": len(cfgs)}
    if sig in _plan_cache:
        report.update(cached=True, plan=plan_name(_plan_cache[sig]))
        return _plan_cache[sig], report
    stream = torch.cuda.current_stream()
    best, best_t = None, None
    for plan in plans:
        try:
            ctls, b = make_batch(cfgs, states, plan)
        except (native.MppiError, ValueError):
            continue  # e.g. one model only, or a controller too large for this schedule
        t = _time_batch(b, ticks, warmup, stream)
        report["timings_ms"][plan_name(plan)] = t
        b.close()
        del ctls
        if best_t is None or t < best_t:
            best, best_t = plan, t
    if best is None:
        raise RuntimeError("no layout supports this controller set")
    _plan_cache[sig] = best
    report.update(cached=False, plan=plan_name(best))
    return best, report


def choose_schedule(cfgs, states, candidates=CANDIDATES, ticks=3, warmup=1, subset=None,
                    seed=0):
    """The fastest measured rollout schedule for a serving pool over cfgs
    (grid-launched ticks; cached per signature) and a report of the timings.
    With `subset`, each candidate is timed on a batch of that many
    controllers drawn (seeded) from cfgs: the shape of a serving tick rather
    than of the whole resident set."""
    cfgs, states = _subset(cfgs, states, subset, seed)
    sig = signature(cfgs)
    report = {"signature": sig, "timings_ms": {}, "controllers_timed": len(cfgs)}
    if sig in _cache:
        report.update(cached=True, schedule=int(_cache[sig]))
        return _cache[sig], report
    stream = torch.cuda.current_stream()
    best, best_t = None, None
    for sched in candidates:
        try:
            ctls = [Controller(dict(c, schedule=sched)) for c in cfgs]
            b = Batch(ctls, states)
        except native.MppiError:
            continue
        t = _time_batch(b, ticks, warmup, stream)
        report["timings_ms"][int(sched)] = t
        b.close()
        del ctls
        if best_t is None or t < best_t:
            best, best_t = sched, t
    if best is None:
        raise RuntimeError("no schedule supports this controller set")
    _cache[sig] = best
    report.update(cached=False, schedule=int(best))
    return best, report


def build_batch(cfgs, states, U0s=None, plans=PLANS, ticks=3, warmup=1, verbose=False):
    """Controllers for cfgs with the fastest measured layout, and their stepper.

    The timing runs advance freshly built controllers that are then discarded,
    so the returned controllers start from U0s (default u_init) and their
    start iterations.  Returns (controllers, stepper, report)."""
    best, report = choose_plan(cfgs, states, plans, ticks, warmup)
    if verbose:
        print("autotune", report, flush=True)
    ctls, stepper = make_batch(cfgs, states, best, U0s)
    return ctls, stepper, report
