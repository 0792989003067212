"""Schedule autotuner for the batched form.

A batch can run its controllers with either rollout schedule (one sample per
lane, 256 samples per workgroup; or wave-specialised, 64 samples per
workgroup).  Which is faster depends on the mix of K, T and models and on
how many controllers share the GPU, so the choice is measured, not guessed:
every candidate is built on the caller's controller set, timed over a few
warm ticks on the device, and the fastest is kept.  Decisions are cached per
batch signature (model mix and (K, T) multiset), so a serving loop pays the
measurement once per distinct batch shape.
"""

import hashlib
import json

import torch

from . import native
from .controller import Batch, Controller

CANDIDATES = (native.C["MPPI_SCHED_LANE"], native.C["MPPI_SCHED_WAVE_SPECIALISED"])
_cache = {}


def signature(cfgs):
    """Shape signature of a controller set (order independent)."""
    key = sorted((c["dynamics"], c["K"], c["T"], c.get("cost_form", 0), c["nu"] > 0) for c in cfgs)
    return hashlib.sha1(json.dumps(key).encode()).hexdigest()[:16]


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


def choose_schedule(cfgs, states, candidates=CANDIDATES, ticks=3, warmup=1, subset=None,
                    seed=0):
    """The fastest measured schedule for cfgs (cached per signature) and a
    report of the timings.  With `subset`, each candidate is timed on a batch
    of that many controllers drawn (seeded) from cfgs: the shape of a serving
    tick rather than of the whole resident set."""
    if subset is not None and subset < len(cfgs):
        import numpy as np
        pick = np.random.default_rng(seed).choice(len(cfgs), size=subset, replace=False)
        cfgs = [cfgs[i] for i in pick]
        states = [states[i] for i in pick]
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
            continue  # e.g. a controller too large for a fused update in this schedule
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


def build_batch(cfgs, states, U0s=None, candidates=CANDIDATES, ticks=3, warmup=1, verbose=False):
    """Controllers for cfgs with the fastest measured schedule, and their Batch.

    The timing runs advance freshly built controllers that are then discarded,
    so the returned controllers start from U0s (default u_init) and their
    start iterations.  Returns (controllers, batch, report)."""
    best, report = choose_schedule(cfgs, states, candidates, ticks, warmup)
    if verbose:
        print("autotune", report, flush=True)
    ctls = [Controller(dict(c, schedule=best), None if U0s is None else U0s[i])
            for i, c in enumerate(cfgs)]
    return ctls, Batch(ctls, states), report
