"""Serving form: continuous batching of MPC-step requests over controllers
resident on the GPU.

Requests arrive for individual controllers (one MPC step each: `iters`
iterations of Algorithm 1 from the controller's current plant state, then the
receding-horizon shift).  Whenever one of the server's `max_inflight` slots
is free, it launches one tick over every resident controller that has a
request waiting and no tick in flight.  Ticks on different slots run on
different streams, so a small tick does not wait for a large one.  A
controller's requests are served in arrival order, one per tick; its result
depends only on its own request sequence.

Residency is bounded by HBM footprint: the workspaces of the resident
controllers sum to at most the cap.  A controller whose workspace alone
exceeds the cap is refused.  The others start resident in order while they
fit; a request for one that is not resident waits until it is admitted,
which evicts the least recently used idle residents (no request waiting, no
tick in flight) until its workspace fits.  An evicted controller keeps its
whole state on the host (its control sequence and its iteration counter,
which fixes its noise stream) and is rebuilt from it on admission, so
eviction changes latency, never results.

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
    """Indices that start resident (in order while the summed footprint stays
    within cap_bytes), the indices that wait, and the resident bytes."""
    used, ok, rest = 0, [], []
    for i, c in enumerate(cfgs):
        b = footprint_bytes(c)
        if used + b <= cap_bytes:
            used += b
            ok.append(i)
        else:
            rest.append(i)
    return ok, rest, used


class PlainBackend:
    """Per-request launches: control_step then plant_step for each request,
    on the slot's stream; states and results staged through pinned buffers.
    Ticks name pool positions, as in the pool back end."""

    def __init__(self, controllers, max_inflight):
        n = len(controllers)
        self.controllers = list(controllers)
        self.x = [torch.zeros(n, 12, device="cuda") for _ in range(max_inflight)]
        self.u0 = [torch.zeros(n, 4, device="cuda") for _ in range(max_inflight)]
        self.d = [torch.zeros(n, 8, device="cuda") for _ in range(max_inflight)]
        self.h_in = [torch.zeros(n, 20, pin_memory=True) for _ in range(max_inflight)]
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
            for j, pos in enumerate(ids):
                ctl = self.controllers[pos]
                x = self.x[slot][j, :ctl.n]
                u = self.u0[slot][j, :ctl.m]
                ctl.stream = stream
                ctl.control_step(x, iters, u0_out=u)
                ctl.plant_step(x, u, self.d[slot][j, :ctl.m], self.d[slot][j, 4:7])
            self.h_out[slot][:c, :4].copy_(self.u0[slot][:c], non_blocking=True)
            self.h_out[slot][:c, 4:].copy_(self.x[slot][:c], non_blocking=True)
            self.ev[slot].record(stream)
        self.ids[slot] = np.array(ids, dtype=np.int32)

    def replace(self, pos, ctl):
        self.controllers[pos] = ctl

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

    def replace(self, pos, ctl):
        self.pool.replace(pos, ctl)

    def finished(self, slot):
        return self.pool.finished(slot)

    def results(self, slot):
        return self.pool.results(slot, plant=True)


class Server:
    """Continuous-batching MPC server with HBM-bounded residency.

    cfgs, x0s: controller configurations and initial plant states (all with
    the same rollout schedule, or schedule 0 to let the library choose).
    dist: per-controller plant disturbance tables [n][steps, 8] (words 0..3
    added to the control channels, 4..6 the quadrotor's body force); request
    r of controller c uses dist[c][r mod steps].  Controllers are named by
    their index into `admitted` (the configurations that fit the cap)."""

    def __init__(self, cfgs, x0s, dist, hbm_cap_bytes=64 << 30, max_inflight=4, iters=1,
                 backend="pool", schedule=None):
        if schedule is not None:
            cfgs = [dict(c, schedule=int(schedule)) for c in cfgs]
        self.cap = int(hbm_cap_bytes)
        self.admitted = [i for i, c in enumerate(cfgs) if footprint_bytes(c) <= self.cap]
        self.refused = [i for i, c in enumerate(cfgs) if footprint_bytes(c) > self.cap]
        if not self.admitted:
            raise ValueError("no controller fits the HBM cap")
        self.cfgs = [cfgs[i] for i in self.admitted]
        n = len(self.cfgs)
        self.footprint = np.array([footprint_bytes(c) for c in self.cfgs], dtype=np.int64)
        first, _, self.resident_bytes = admit(self.cfgs, self.cap)
        # resident controller -> pool position and back; evicted controllers'
        # saved (U, iteration)
        self.pos = np.full(n, -1, dtype=np.int64)
        self.at = list(first)
        self.pos[first] = np.arange(len(first))
        self.controllers = [None] * n
        for c in first:
            self.controllers[c] = Controller(self.cfgs[c])
        self.saved = [None] * n
        self.state = np.zeros((n, 12), dtype=np.float32)
        for j, i in enumerate(self.admitted):
            x = np.asarray(x0s[i], dtype=np.float32)
            self.state[j, :len(x)] = x
        self.dist = [np.asarray(dist[i], dtype=np.float32).reshape(len(dist[i]), -1)
                     for i in self.admitted]
        self.iters = int(iters)
        self.max_inflight = int(max_inflight)
        self.streams = [torch.cuda.Stream() for _ in range(self.max_inflight)]
        ctls = [self.controllers[c] for c in first]
        if backend == "pool":
            self.backend = PoolBackend(ctls, self.max_inflight)
        elif backend == "plain":
            self.backend = PlainBackend(ctls, self.max_inflight)
        else:
            raise ValueError("backend must be 'pool' or 'plain'")
        self.served = np.zeros(n, dtype=np.int64)
        self.admissions = 0
        self.evictions = 0
        self.sample_steps = np.array([c["K"] * c["T"] * self.iters for c in self.cfgs],
                                     dtype=np.float64)

    @property
    def admitted_bytes(self):
        return self.resident_bytes

    def iteration(self, c):
        """Iteration counter of controller c (resident or evicted)."""
        if self.controllers[c] is not None:
            return self.controllers[c].stats()["iteration"]
        if self.saved[c] is not None:
            return self.saved[c][1]
        return self.cfgs[c]["start_iteration"]

    def _dist(self, ids):
        out = np.zeros((len(ids), 8), dtype=np.float32)
        for j, c in enumerate(ids):
            row = self.dist[c][self.served[c] % len(self.dist[c])]
            out[j, :len(row)] = row
        return out

    def _evict(self, c, free):
        ctl = self.controllers[c]
        st = ctl.stats()
        self.saved[c] = (ctl.U.cpu().numpy(), int(st["iteration"]))
        ctl.close()
        ctl.ws = None
        self.controllers[c] = None
        p = int(self.pos[c])
        self.pos[c] = -1
        self.at[p] = -1
        free.append(p)
        self.resident_bytes -= int(self.footprint[c])
        self.evictions += 1

    def _admit(self, c, idle, busy, free, pend, lost):
        """Make c resident, evicting until its workspace fits and a position
        is free: first the least recently used idle residents (`idle`, oldest
        first), then, so that c is not starved, residents not in flight whose
        next request arrived after c's (latest first).  Evicted controllers
        are appended to `lost`.  False if c cannot fit yet."""
        need = int(self.footprint[c])
        head = pend[c][0]
        while self.resident_bytes + need > self.cap or not free:
            if idle:
                v, _ = idle.popitem(last=False)
            else:
                later = [r for r in self.at if r >= 0 and not busy[r] and pend[r]
                         and pend[r][0] > head]
                if not later:
                    return False
                v = max(later, key=lambda r: pend[r][0])
            self._evict(v, free)
            lost.append(v)
        p = free.pop()
        if self.saved[c] is None:
            ctl = Controller(self.cfgs[c])
        else:
            U, it = self.saved[c]
            ctl = Controller(dict(self.cfgs[c], start_iteration=it), U0=U)
            self.saved[c] = None
        self.backend.replace(p, ctl)
        self.controllers[c] = ctl
        self.pos[c] = p
        self.at[p] = c
        self.resident_bytes += need
        self.admissions += 1
        return True

    def run(self, arrival_t, arrival_ctl, warmup_s=0.0, record=False):
        """Serve the request stream (times in s from the start of the call,
        controller index into the admitted set) in real time; returns the
        latency and throughput statistics of the requests that arrived after
        warmup_s.  record: also keep every request's u_0, per controller in
        service order, in self.log."""
        n = len(self.cfgs)
        arrival_t = np.asarray(arrival_t, dtype=np.float64)
        arrival_ctl = np.asarray(arrival_ctl, dtype=np.int64)
        total = len(arrival_t)
        pend = [collections.deque() for _ in range(n)]
        busy = np.zeros(n, dtype=bool)
        queued = np.zeros(n, dtype=bool)
        ready = []                        # resident, request waiting, not in flight
        waiting = collections.deque()     # not resident, request waiting
        in_wait = np.zeros(n, dtype=bool)
        idle = collections.OrderedDict()  # resident, nothing waiting, LRU first
        free = collections.deque()        # pool positions of evicted controllers
        for c in range(n):
            if self.pos[c] >= 0:
                idle[c] = True
        slots = collections.deque(range(self.max_inflight))
        inflight = {}
        if record:
            self.log = [[] for _ in range(n)]
        lat, done_t, steps_done, tick_sizes = [], [], [], []
        nxt, finished = 0, 0
        t0 = time.perf_counter()
        while finished < total:
            now = time.perf_counter() - t0
            while nxt < total and arrival_t[nxt] <= now:
                c = int(arrival_ctl[nxt])
                pend[c].append(arrival_t[nxt])
                idle.pop(c, None)
                if self.pos[c] < 0:
                    if not in_wait[c]:
                        in_wait[c] = True
                        waiting.append(c)
                elif not busy[c] and not queued[c]:
                    queued[c] = True
                    ready.append(c)
                nxt += 1
            for slot in list(inflight):
                if not self.backend.finished(slot):
                    continue
                pos, u0, xn = self.backend.results(slot)
                tdone = time.perf_counter() - t0
                ids = inflight.pop(slot)
                slots.append(slot)
                assert np.array_equal(self.pos[ids], pos)
                self.state[ids] = xn
                self.served[ids] += 1
                busy[ids] = False
                for j, c in enumerate(ids):
                    a = pend[c].popleft()
                    if record:
                        self.log[c].append(u0[j, :self.controllers[c].m].copy())
                    if a >= warmup_s:
                        lat.append(tdone - a)
                        done_t.append(tdone)
                        steps_done.append(self.sample_steps[c])
                    if pend[c]:
                        queued[c] = True
                        ready.append(c)
                    else:
                        idle[c] = True
                finished += len(ids)
            while waiting:
                c = waiting[0]
                lost = []
                ok = self._admit(c, idle, busy, free, pend, lost)
                for v in lost:
                    # an evicted resident with a request waiting waits again
                    queued[v] = False
                    if pend[v]:
                        in_wait[v] = True
                        waiting.append(v)
                if not ok:
                    break
                waiting.popleft()
                in_wait[c] = False
                queued[c] = True
                ready.append(c)
            if ready and slots:
                ids = []
                for c in ready:
                    if queued[c] and self.pos[c] >= 0:
                        queued[c] = False
                        ids.append(c)
                ready = []
                if ids:
                    ids = np.array(ids, dtype=np.int64)
                    slot = slots.popleft()
                    busy[ids] = True
                    self.backend.tick(self.pos[ids].astype(np.int32), self.state[ids],
                                      self._dist(ids), self.iters, slot, self.streams[slot])
                    inflight[slot] = ids
                    tick_sizes.append(len(ids))
            elif not inflight and nxt < total and not ready and not waiting:
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
            "admissions": self.admissions,
            "evictions": self.evictions,
        }

    def close(self):
        b = getattr(self.backend, "pool", None)
        if b is not None:
            b.close()
        for c in self.controllers:
            if c is not None:
                c.close()
