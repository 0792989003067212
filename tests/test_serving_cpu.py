"""The serving scheduler's residency logic on the host, with the controller
and the device back end replaced by deterministic stand-ins: a stand-in's
result depends on its whole state (control sequence, iteration counter) and
on the request, so a controller that loses state across an eviction, or is
served out of order or twice, changes the results."""

import numpy as np
import pytest
import torch

from paper_1807_06108_amd import serving, workloads


class FakeController:
    """State: U [T] and the iteration counter.  A request from state x
    rotates U, mixes in x and the iteration, and returns u_0 = U[0]."""

    order = []

    def __init__(self, cfg, U0=None):
        self.name = cfg.get("controller_id")
        self.T = int(cfg["T"])
        self.m = 1
        self.U = torch.tensor(np.zeros(self.T, np.float32) if U0 is None else np.asarray(U0))
        self.it = int(cfg["start_iteration"])
        self.closed = False

    def request(self, x, iters):
        assert not self.closed
        FakeController.order.append(self.name)
        U = self.U.numpy()
        for _ in range(iters):
            U = np.roll(U, -1) * np.float32(0.9) + np.float32(0.01) * x[0] + np.float32(1e-3 * self.it)
            self.it += 1
        self.U = torch.tensor(U)
        return U[0]

    def stats(self):
        return {"iteration": self.it}

    def close(self):
        self.closed = True


class FakeBackend:
    """Finishes a tick when finished() has been asked `lag` times."""

    def __init__(self, controllers, max_inflight, lag=2):
        self.controllers = list(controllers)
        self.out = [None] * max_inflight
        self.lag = lag

    def tick(self, ids, states, dist, iters, slot, stream):
        assert self.out[slot] is None and len(set(ids)) == len(ids)
        u0 = np.zeros((len(ids), 4), np.float32)
        xn = np.zeros((len(ids), 12), np.float32)
        for j, p in enumerate(ids):
            u0[j, 0] = self.controllers[p].request(states[j], iters)
            xn[j, 0] = states[j, 0] * np.float32(0.5) + u0[j, 0] + dist[j, 0]
        self.out[slot] = [self.lag, np.array(ids), u0, xn]

    def replace(self, pos, ctl):
        self.controllers[pos] = ctl

    def finished(self, slot):
        self.out[slot][0] -= 1
        return self.out[slot][0] <= 0

    def results(self, slot):
        _, ids, u0, xn = self.out[slot]
        self.out[slot] = None
        return ids, u0, xn


@pytest.fixture
def fakes(monkeypatch):
    monkeypatch.setattr(serving, "Controller", FakeController)
    monkeypatch.setattr(serving, "PoolBackend", FakeBackend)
    monkeypatch.setattr(serving, "footprint_bytes", lambda c: int(c["K"]) * 1000)
    monkeypatch.setattr(torch.cuda, "Stream", lambda: None)
    monkeypatch.setattr(torch.cuda, "synchronize", lambda: None)


def _setup(n, seed):
    g = np.random.default_rng(seed)
    cfgs = [dict(K=int(g.integers(1, 9)), T=int(g.integers(3, 12)), start_iteration=int(i * 7))
            for i in range(n)]
    x0s = [g.standard_normal(4).astype(np.float32) for _ in range(n)]
    dist = [g.standard_normal((5, 8)).astype(np.float32) for _ in range(n)]
    return cfgs, x0s, dist


@pytest.mark.parametrize("cap_k", [8, 12, 20])
def test_eviction_changes_no_result(fakes, cap_k):
    n = 24
    cfgs, x0s, dist = _setup(n, seed=cap_k)
    g = np.random.default_rng(5)
    total = 600
    t = np.sort(g.uniform(0, 0.05, total))
    ids = g.integers(0, n, total)
    # two bursts on a few controllers, so that residents have requests waiting
    ids[100:160] = g.integers(0, 3, 60)
    ref = serving.Server(cfgs, x0s, dist, hbm_cap_bytes=10 ** 9, max_inflight=3)
    r_ref = ref.run(t, ids, record=True)
    assert ref.evictions == 0 and r_ref["requests"] == total
    srv = serving.Server(cfgs, x0s, dist, hbm_cap_bytes=cap_k * 1000, max_inflight=3)
    r = srv.run(t, ids, record=True)
    assert r["requests"] == total and srv.evictions > 0 and srv.admissions > 0
    assert np.array_equal(srv.served, np.bincount(ids, minlength=n))
    assert srv.resident_bytes <= cap_k * 1000
    for c in range(n):
        assert len(srv.log[c]) == len(ref.log[c])
        assert all(np.array_equal(a, b) for a, b in zip(srv.log[c], ref.log[c])), c
        assert srv.iteration(c) == ref.iteration(c) == cfgs[c]["start_iteration"] + srv.served[c]
    assert np.array_equal(srv.state, ref.state)


def test_a_controller_larger_than_the_cap_is_refused(fakes):
    cfgs, x0s, dist = _setup(6, seed=1)
    cfgs[2]["K"] = 50
    srv = serving.Server(cfgs, x0s, dist, hbm_cap_bytes=20 * 1000)
    assert srv.refused == [2] and srv.admitted == [0, 1, 3, 4, 5]
    assert srv.resident_bytes <= 20 * 1000
    with pytest.raises(ValueError):
        serving.Server(cfgs[2:3], x0s[2:3], dist[2:3], hbm_cap_bytes=20 * 1000)


def test_hot_residents_do_not_starve_a_waiting_controller(fakes):
    """Controllers 0 and 1 fill the cap and hold 100 requests each, all
    waiting at the start; controller 2's one request, which arrived after
    their first ten, is served long before they run out."""
    cfgs = [dict(K=5, T=4, start_iteration=0, controller_id=i) for i in range(3)]
    x0s = [np.zeros(4, np.float32)] * 3
    dist = [np.zeros((1, 8), np.float32)] * 3
    t = np.linspace(-1.0, -0.5, 201)
    ids = np.array([0, 1] * 100 + [0])
    ids[20] = 2
    srv = serving.Server(cfgs, x0s, dist, hbm_cap_bytes=10 * 1000, max_inflight=1)
    FakeController.order = []
    r = srv.run(t, ids, warmup_s=-2.0, record=True)
    assert r["requests"] == 201 and srv.served[2] == 1 and srv.evictions >= 1
    assert FakeController.order.index(2) < 40
