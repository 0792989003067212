"""Serving form: continuous batching of MPC-step requests over resident
controllers.

Requests arrive for individual controllers (one MPC step each: `iters`
iterations of Algorithm 1 from the controller's current plant state, then the
receding-horizon shift).  The server keeps every admitted controller resident
on the GPU (workspace, warm control sequence and noise-stream position) and,
whenever one of its `max_inflight` slots is free, launches one tick over every
controller that has a request waiting and no tick in flight.  Ticks on
different slots run on different streams, so a small tick does not wait for a
large one.  A controller's requests are served in arrival order, one per
tick; its result depends only on its own request sequence.

Admission is by HBM footprint: controllers are admitted in order while the
sum of their workspaces stays within the cap; the rest are refused.

Two back ends run the same scheduler: `pool` (one grid per tick over all of
its requests, the library's pool entry points) and `plain` (one control-step
launch and one plant launch per request), for comparison.
"""

import collections
import time

import numpy as np
import torch

from . import native
from .controller import Controller, Pool


def footprint_bytes(cfg):
    """HBM held resident by one controller: its workspace."""
    return native.workspace_bytes(cfg)


def admit(cfgs, cap_bytes):
    """Indices admitted in order while the summed footprint stays within
    cap_bytes, the refused indices, and the admitted bytes."""
    used, ok, refused = 0, [], []
    for i, c in enumerate(cfgs):
        b = footprint_bytes(c)
        if used + b <= cap_bytes:
            used += b
            ok.append(i)
        else:
            refused.append(i)
    return ok, refused, used


class PlainBackend:
    """Per-request launches: control_step then plant_step for each request,
    on the slot's stream; states and results staged through pinned buffers."""

    def __init__(self, controllers, max_inflight):
        n = len(controllers)
        self.controllers = controllers
        self.x = [torch.zeros(n, 12, device="cuda") for _ in range(max_inflight)]
        self.u0 = [torch.zeros(n, 4, device="cuda") for _ in range(max_inflight)]
        self.d = [torch.zeros(n, 4, device="cuda") for _ in range(max_inflight)]
        self.h_in = [torch.zeros(n, 16, pin_memory=True) for _ in range(max_inflight)]
        self.h_out = [torch.zeros(n, 16, pin_memory=True) for _ in range(max_inflight)]
        self.ev = [torch.cuda.Event() for _ in range(max_inflight)]
        self.ids = [None] * max_inflight

    def tick(self, ids, states, dist, iters, slot, stream):
        c = len(ids)
        hin = self.h_in[slot].numpy()
        hin[:c, :12] = states
        hin[:c, 12:] = dist
        with torch.cuda.stream(stream):
            buf = self.h_in[slot][:c].to("cuda", non_blocking=True)
            self.x[slot][:c].copy_(buf[:, :12])
            self.d[slot][:c].copy_(buf[:, 12:])
            for j, cid in enumerate(ids):
                ctl = self.controllers[cid]
                x = self.x[slot][j, :ctl.n]
                u = self.u0[slot][j, :ctl.m]
                ctl.stream = stream
                ctl.control_step(x, iters, u0_out=u)
                ctl.plant_step(x, u, self.d[slot][j, :ctl.m])
            self.h_out[slot][:c, :4].copy_(self.u0[slot][:c], non_blocking=True)
            self.h_out[slot][:c, 4:].copy_(self.x[slot][:c], non_blocking=True)
            self.ev[slot].record(stream)
        self.ids[slot] = np.array(ids, dtype=np.int32)

    def finished(self, slot):
        return self.ev[slot].query()

    def results(self, slot):
        ids = self.ids[slot]
        out = self.h_out[slot].numpy()[:len(ids)]
        return ids, out[:, :4].copy(), out[:, 4:].copy()


class PoolBackend:
    def __init__(self, controllers, max_inflight):
        self.pool = Pool(controllers, max_inflight)

    def tick(self, ids, states, dist, iters, slot, stream):
        self.pool.tick(ids, states, dist, iters=iters, slot=slot, stream=stream)

    def finished(self, slot):
        return self.pool.finished(slot)

    def results(self, slot):
        return self.pool.results(slot, plant=True)


class Server:
    """Continuous-batching MPC server over resident controllers.

    cfgs, x0s: controller configurations and initial plant states (all with
    the same rollout schedule, or schedule 0 to let the library choose).
    dist: per-controller plant disturbance tables [n][steps, 4]; request r of
    controller c uses dist[c][r mod steps]."""

    def __init__(self, cfgs, x0s, dist, hbm_cap_bytes=64 << 30, max_inflight=4, iters=1,
                 backend="pool", schedule=None):
        if schedule is not None:
            cfgs = [dict(c, schedule=int(schedule)) for c in cfgs]
        self.admitted, self.refused, self.admitted_bytes = admit(cfgs, hbm_cap_bytes)
        if not self.admitted:
            raise ValueError("no controller fits the HBM cap")
        self.cfgs = [cfgs[i] for i in self.admitted]
        self.controllers = [Controller(c) for c in self.cfgs]
        n = len(self.controllers)
        self.state = np.zeros((n, 12), dtype=np.float32)
        for j, i in enumerate(self.admitted):
            x = np.asarray(x0s[i], dtype=np.float32)
            self.state[j, :len(x)] = x
        self.dist = [np.asarray(dist[i], dtype=np.float32) for i in self.admitted]
        self.iters = int(iters)
        self.max_inflight = int(max_inflight)
        self.streams = [torch.cuda.Stream() for _ in range(self.max_inflight)]
        if backend == "pool":
            self.backend = PoolBackend(self.controllers, self.max_inflight)
        elif backend == "plain":
            self.backend = PlainBackend(self.controllers, self.max_inflight)
        else:
            raise ValueError("backend must be 'pool' or 'plain'")
        self.served = np.zeros(n, dtype=np.int64)
        self.sample_steps = np.array([c["K"] * c["T"] * self.iters for c in self.cfgs],
                                     dtype=np.float64)

    def _dist(self, ids):
        return np.stack([self.dist[c][self.served[c] % len(self.dist[c])] for c in ids])

    def run(self, arrival_t, arrival_ctl, warmup_s=0.0):
        """Serve the request stream (times in s from the start of the call,
        controller index into the admitted set) in real time; returns the
        latency and throughput statistics of the requests that arrived after
        warmup_s."""
        n = len(self.controllers)
        arrival_t = np.asarray(arrival_t, dtype=np.float64)
        arrival_ctl = np.asarray(arrival_ctl, dtype=np.int64)
        total = len(arrival_t)
        pend = [collections.deque() for _ in range(n)]
        busy = np.zeros(n, dtype=bool)
        queued = np.zeros(n, dtype=bool)
        ready = []
        free = collections.deque(range(self.max_inflight))
        inflight = {}
        lat, done_t, steps_done = [], [], []
        tick_sizes = []
        nxt, finished = 0, 0
        t0 = time.perf_counter()
        while finished < total:
            now = time.perf_counter() - t0
            while nxt < total and arrival_t[nxt] <= now:
                c = arrival_ctl[nxt]
                pend[c].append(arrival_t[nxt])
                if not busy[c] and not queued[c]:
                    queued[c] = True
                    ready.append(c)
                nxt += 1
            for slot in list(inflight):
                if not self.backend.finished(slot):
                    continue
                ids, u0, xn = self.backend.results(slot)
                tdone = time.perf_counter() - t0
                del inflight[slot]
                free.append(slot)
                self.state[ids] = xn
                self.served[ids] += 1
                busy[ids] = False
                for c in ids:
                    a = pend[c].popleft()
                    if a >= warmup_s:
                        lat.append(tdone - a)
                        done_t.append(tdone)
                        steps_done.append(self.sample_steps[c])
                    if pend[c]:
                        queued[c] = True
                        ready.append(c)
                finished += len(ids)
            if ready and free:
                slot = free.popleft()
                ids = np.array(ready, dtype=np.int32)
                ready = []
                queued[ids] = False
                busy[ids] = True
                self.backend.tick(ids, self.state[ids], self._dist(ids), self.iters, slot,
                                  self.streams[slot])
                inflight[slot] = ids
                tick_sizes.append(len(ids))
            elif not inflight and nxt < total:
                # idle until the next arrival
                wait = arrival_t[nxt] - (time.perf_counter() - t0)
                if wait > 2e-4:
                    time.sleep(wait - 1e-4)
        torch.cuda.synchronize()
        lat = np.asarray(lat)
        done_t = np.asarray(done_t)
        span = done_t.max() - warmup_s if len(done_t) else float("nan")
        return {
            "requests": int(len(lat)),
            "requests_per_s": len(lat) / span,
            "rollout_steps_per_s": float(np.sum(steps_done)) / span,
            "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3),
                           "p99": float(np.percentile(lat, 99) * 1e3),
                           "max": float(lat.max() * 1e3)},
            "ticks": len(tick_sizes),
            "mean_tick_requests": float(np.mean(tick_sizes)),
            "span_s": float(span),
        }

    def close(self):
        b = getattr(self.backend, "pool", None)
        if b is not None:
            b.close()
        for c in self.controllers:
            c.close()
