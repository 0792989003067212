"""Serving form: ticks over a resident pool.  A request's result is the same
whether it is served alone or in a mixed tick (bitwise: same kernels, same
per-controller noise and combine), equals the plain per-controller control
step, matches the oracle's costs, and the pool rejects unsafe reuse."""

import numpy as np
import pytest
import torch

from gpu_util import check_S
from oracle import mppi as omppi
from paper_1807_06108_amd import native, serving, workloads
from paper_1807_06108_amd.controller import Controller, Pool

pytestmark = pytest.mark.gpu

LANE = native.C["MPPI_SCHED_LANE"]
WS = native.C["MPPI_SCHED_WAVE_SPECIALISED"]


def _set(schedule, n=10, seed=3):
    out = []
    for cfg, x0 in workloads.random_controllers(n, seed=seed):
        cfg = dict(cfg, schedule=schedule, K=min(cfg["K"], 2048), T=min(cfg["T"], 60))
        out.append((cfg, x0))
    out.append((dict(workloads.double_integrator(K=300, T=17, seed=77, controller_id=600),
                     schedule=schedule), workloads.x0_for(workloads.double_integrator())))
    return out


def _states(cset):
    st = np.zeros((len(cset), 12), dtype=np.float32)
    for i, (_, x0) in enumerate(cset):
        st[i, :len(x0)] = x0
    return st


def _dists(cset, steps=8):
    return [workloads.serving_disturbances(c, steps, seed=500 + i) for i, (c, _) in enumerate(cset)]


def _serve(pool, cset, schedule_of_ticks, streams):
    """Run ticks (lists of controller indices; consecutive lists may share a
    slot only after the earlier one finished) and return per-controller
    (u0, x_next) sequences."""
    st = _states(cset)
    dist = _dists(cset)
    count = np.zeros(len(cset), dtype=int)
    seq = [[] for _ in cset]
    inflight = {}
    for t, ids in enumerate(schedule_of_ticks):
        slot = t % pool.max_inflight
        if slot in inflight:
            torch.cuda.synchronize()
            _collect(pool, slot, inflight.pop(slot), st, seq)
        for s2 in list(inflight):  # a controller of this tick may be in flight elsewhere
            if set(inflight[s2]) & set(ids):
                torch.cuda.synchronize()
                _collect(pool, s2, inflight.pop(s2), st, seq)
        ids = np.array(ids, dtype=np.int32)
        d = np.stack([dist[c][count[c]] for c in ids])
        count[ids] += 1
        pool.tick(ids, st[ids], d, iters=2, slot=slot, stream=streams[slot])
        inflight[slot] = list(ids)
    torch.cuda.synchronize()
    for slot, ids in inflight.items():
        _collect(pool, slot, ids, st, seq)
    return seq


def _collect(pool, slot, ids, st, seq):
    assert pool.finished(slot)
    rid, u0, xn = pool.results(slot)
    assert list(rid) == list(ids)
    for j, c in enumerate(rid):
        seq[c].append((u0[j].copy(), xn[j].copy()))
        st[c] = xn[j]


@pytest.mark.parametrize("schedule", [LANE, WS])
def test_alone_equals_in_the_mix(schedule):
    cset = _set(schedule)
    n = len(cset)
    print("pool of", n, "controllers, schedule", schedule, flush=True)
    rng = np.random.default_rng(1)
    mixed = [list(rng.choice(n, size=rng.integers(1, n + 1), replace=False)) for _ in range(6)]
    per_ctl = [[t for t in mixed if c in t] for c in range(n)]
    alone = [[c] for c in range(n) for _ in per_ctl[c]]
    streams = [torch.cuda.Stream() for _ in range(3)]
    a_ctl = [Controller(c) for c, _ in cset]
    b_ctl = [Controller(c) for c, _ in cset]
    pa, pb = Pool(a_ctl, 3), Pool(b_ctl, 3)
    sa = _serve(pa, cset, mixed, streams)
    sb = _serve(pb, cset, alone, streams)
    for c in range(n):
        assert len(sa[c]) == len(sb[c]) == len(per_ctl[c])
        for (ua, xa), (ub, xb) in zip(sa[c], sb[c]):
            assert np.array_equal(ua, ub), c
            assert np.array_equal(xa[:a_ctl[c].n], xb[:a_ctl[c].n]), c
        assert np.array_equal(a_ctl[c].U.cpu().numpy(), b_ctl[c].U.cpu().numpy())
        assert a_ctl[c].stats() == b_ctl[c].stats()


def test_pool_equals_plain_control_step():
    cset = _set(LANE, n=6, seed=8)
    n = len(cset)
    a_ctl = [Controller(c) for c, _ in cset]
    b_ctl = [Controller(c) for c, _ in cset]
    pool = Pool(a_ctl, 2)
    st = _states(cset)
    dist = _dists(cset)
    for step in range(3):
        ids = np.arange(n, dtype=np.int32)[::-1].copy()
        d = np.stack([dist[c][step] for c in ids])
        pool.tick(ids, st[ids], d, iters=2, slot=step % 2)
        torch.cuda.synchronize()
        rid, u0, xn = pool.results(step % 2)
        for j, c in enumerate(rid):
            ctl = b_ctl[c]
            x = torch.tensor(st[c, :ctl.n], device="cuda")
            u = ctl.control_step(x, 2)
            ctl.plant_step(x, u, torch.tensor(d[j, :ctl.m], device="cuda"),
                           torch.tensor(d[j, 4:7], device="cuda"))
            np.testing.assert_array_max_ulp(u0[j, :ctl.m], u.cpu().numpy(), maxulp=1)
            assert not u0[j, ctl.m:].any()
            np.testing.assert_allclose(xn[j, :ctl.n], x.cpu().numpy(), rtol=1e-5, atol=1e-5)
            st[c] = xn[j]
        for ca, cb in zip(a_ctl, b_ctl):
            np.testing.assert_array_max_ulp(ca.U.cpu().numpy(), cb.U.cpu().numpy(), maxulp=1)


def test_pool_costs_match_the_oracle():
    cset = _set(WS, n=4, seed=12)
    ctls = [Controller(c, workloads.U0_for(c, "random", seed=i + 3)) for i, (c, _) in enumerate(cset)]
    pool = Pool(ctls, 1)
    st = _states(cset)
    ids = np.array([2, 0, 4, 1, 3], dtype=np.int32)
    pool.tick(ids, st[ids], None, iters=1, slot=0)
    torch.cuda.synchronize()
    rid, u0, _ = pool.results(0, plant=False)
    for i, (cfg, x0) in enumerate(cset):
        U0 = workloads.U0_for(cfg, "random", seed=i + 3).astype(np.float64)
        ref = omppi.iteration(cfg, x0, U0, 0)
        check_S(ctls[i], ref, exclude=ref["margin"] < 1e-4)


def test_pool_guards():
    cset = _set(LANE, n=3, seed=2)
    ctls = [Controller(c) for c, _ in cset]
    pool = Pool(ctls, 2)
    st = _states(cset)

    def code(f):
        with pytest.raises(native.MppiError) as e:
            f()
        return e.value.code

    EINVAL = native.C["MPPI_EINVAL"]
    assert code(lambda: pool.results(0)) == EINVAL                       # nothing enqueued
    assert code(lambda: pool.tick([0, 0], st[[0, 0]], slot=0)) == EINVAL  # duplicate id
    assert code(lambda: pool.tick([7], st[[0]], slot=0)) == EINVAL        # id out of range
    assert code(lambda: pool.tick([0], st[[0]], slot=2)) == EINVAL        # slot out of range
    pool.tick([0, 1], st[[0, 1]], slot=0)
    assert code(lambda: pool.tick([2], st[[2]], slot=0)) == EINVAL        # slot holds a tick
    assert code(lambda: pool.tick([1, 2], st[[1, 2]], slot=1)) == EINVAL  # 1 is in flight
    pool.tick([2], st[[2]], slot=1)
    torch.cuda.synchronize()
    assert code(lambda: pool.results(0, plant=True)) == EINVAL            # no plant ran
    ids, u0, _ = pool.results(0, plant=False)
    assert list(ids) == [0, 1]
    pool.tick([1, 0], st[[1, 0]], slot=0)                                 # reusable again
    torch.cuda.synchronize()
    pool.results(0, plant=False)
    pool.results(1, plant=False)
    with pytest.raises(native.MppiError):
        Pool(ctls, 17)
    # replacing a position: not while its controller is in flight, not with
    # another rollout schedule, not out of range
    spare = Controller(cset[0][0])
    pool.tick([0], st[[0]], slot=0)
    assert code(lambda: pool.replace(0, spare)) == EINVAL
    torch.cuda.synchronize()
    pool.results(0, plant=False)
    assert code(lambda: pool.replace(len(ctls), spare)) == EINVAL
    assert code(lambda: pool.replace(1, Controller(dict(cset[1][0], schedule=WS)))) == EINVAL
    pool.replace(0, spare)
    pool.tick([0, 2], st[[0, 2]], slot=1)
    torch.cuda.synchronize()
    assert list(pool.results(1, plant=False)[0]) == [0, 2]


def test_server_serves_every_request_with_both_back_ends():
    cset = _set(WS, n=12, seed=30)
    cfgs = [c for c, _ in cset]
    x0s = [x for _, x in cset]
    dist = _dists(cset, steps=64)
    t, ids = workloads.serving_arrivals(rate=3000.0, duration=0.25, count=len(cset), seed=3)
    counts = np.bincount(ids, minlength=len(cset))
    for backend in ("pool", "plain"):
        print("server back end", backend, len(t), "requests", flush=True)
        srv = serving.Server(cfgs, x0s, dist, max_inflight=3, backend=backend)
        r = srv.run(t, ids)
        assert r["requests"] == len(t)
        assert np.array_equal(srv.served, counts)
        assert r["latency_ms"]["p50"] > 0
        for i in range(len(cfgs)):
            assert srv.iteration(i) == cfgs[i]["start_iteration"] + counts[i]
        srv.close()


@pytest.mark.parametrize("backend", ["pool", "plain"])
def test_bounded_residency_gives_the_same_results(backend):
    """Under an HBM cap that holds two or three of the controllers, requests
    wait for admission and idle residents are evicted and later rebuilt from
    their saved control sequence and iteration counter: every request's u_0
    and every plant state are bitwise those of a server with every
    controller resident."""
    cset = _set(WS, n=9, seed=31)
    cfgs = [c for c, _ in cset]
    x0s = [x for _, x in cset]
    dist = _dists(cset, steps=16)
    need = sorted(serving.footprint_bytes(c) for c in cfgs)
    cap = need[-1] + need[len(need) // 2]
    t, ids = workloads.serving_arrivals(rate=1500.0, duration=0.12, count=len(cset), seed=4)
    print("bounded residency", backend, len(t), "requests, cap", cap, flush=True)
    ref = serving.Server(cfgs, x0s, dist, max_inflight=2, backend=backend)
    ref.run(t, ids, record=True)
    srv = serving.Server(cfgs, x0s, dist, hbm_cap_bytes=cap, max_inflight=2, backend=backend)
    r = srv.run(t, ids, record=True)
    assert r["requests"] == len(t) and srv.evictions > 0 and srv.resident_bytes <= cap
    assert np.array_equal(srv.served, np.bincount(ids, minlength=len(cset)))
    for c in range(len(cset)):
        assert len(srv.log[c]) == len(ref.log[c])
        for a, b in zip(srv.log[c], ref.log[c]):
            assert np.array_equal(a, b), c
        assert srv.iteration(c) == ref.iteration(c)
    assert np.array_equal(srv.state, ref.state)
    for s in (ref, srv):
        s.close()
