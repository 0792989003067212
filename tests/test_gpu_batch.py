"""Batched form: many uneven controllers advanced by one launch per iteration
give the results of running each controller on its own (same kernels, same
per-controller noise streams and combines), also when the batched step is
captured in a HIP graph and replayed."""

import numpy as np
import pytest
import torch

from gpu_util import check_S
from oracle import mppi as omppi
from paper_1807_06108_amd import native, workloads
from paper_1807_06108_amd import autotune
from paper_1807_06108_amd.controller import Batch, Controller

pytestmark = pytest.mark.gpu

LANE = native.C["MPPI_SCHED_LANE"]
WS = native.C["MPPI_SCHED_WAVE_SPECIALISED"]
GRID = native.C["MPPI_BATCH_GRID"]
PERSISTENT = native.C["MPPI_BATCH_PERSISTENT"]


def _controller_set(schedule, n=12, seed=5):
    out = workloads.random_controllers(n, seed=seed)
    out.append((workloads.double_integrator(K=300, T=17, seed=77, controller_id=500), None))
    out.append((workloads.cartpole(K=700, T=41, nu=0.0, seed=78, controller_id=501), None))
    out.append((workloads.quadrotor(K=64, T=5, cost_form=1, seed=79, controller_id=502), None))
    res = []
    for cfg, x0 in out:
        cfg = dict(cfg, schedule=schedule)
        if x0 is None:
            x0 = workloads.x0_for(cfg)
        res.append((cfg, x0))
    return res


def _make(cset):
    ctls, xs = [], []
    for cfg, x0 in cset:
        U0 = workloads.U0_for(cfg, "random", seed=cfg["controller_id"] + 3)
        ctls.append(Controller(cfg, U0))
        xs.append(torch.tensor(x0, device="cuda"))
    return ctls, xs


@pytest.mark.parametrize("schedule,launch", [(LANE, GRID), (WS, GRID), (LANE, PERSISTENT),
                                             (WS, PERSISTENT)])
def test_batch_equals_individual_controllers(schedule, launch):
    """Both launches of both schedules; two control steps of two iterations
    each, so the persistent launch's work queue is reused four times."""
    cset = _controller_set(schedule)
    print("batch of", len(cset), "controllers, schedule", schedule, "launch", launch, flush=True)
    a_ctl, a_x = _make(cset)
    b_ctl, b_x = _make(cset)
    batch = Batch(a_ctl, a_x, launch=launch)
    u0_ind = []
    for step in range(2):
        batch.step(iters=2, shift=True)
        u0_ind.append([c.control_step(x, 2).cpu().numpy() for c, x in zip(b_ctl, b_x)])
        u0_b = batch.u0.cpu().numpy()
        for i, (ca, cb) in enumerate(zip(a_ctl, b_ctl)):
            m = ca.m
            assert np.array_equal(ca.S.cpu().numpy(), cb.S.cpu().numpy()), i
            np.testing.assert_array_max_ulp(ca.U.cpu().numpy(), cb.U.cpu().numpy(), maxulp=1)
            np.testing.assert_array_max_ulp(u0_b[i, :m], u0_ind[-1][i], maxulp=1)
            sa, sb = ca.stats(), cb.stats()
            assert sa["iteration"] == sb["iteration"] == 2 * (step + 1)
            assert sa["rho"] == sb["rho"]
            assert sa["n_finite"] == sb["n_finite"]


def test_batched_costs_match_the_oracle():
    cset = _controller_set(LANE, n=4, seed=11)
    ctls, xs = _make(cset)
    batch = Batch(ctls, xs)
    batch.step(iters=1, shift=False)
    for (cfg, x0), c in zip(cset, ctls):
        U0 = workloads.U0_for(cfg, "random", seed=cfg["controller_id"] + 3)
        ref = omppi.iteration(cfg, x0, U0.astype(np.float64), 0)
        check_S(c, ref, exclude=ref["margin"] < 1e-4)


def test_batched_step_replays_from_a_graph():
    cset = _controller_set(LANE, n=8, seed=21)
    a_ctl, a_x = _make(cset)
    b_ctl, b_x = _make(cset)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ga = Batch(a_ctl, a_x, stream=s)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            ga.step(iters=2, shift=True)
    eb = Batch(b_ctl, b_x)
    for rep in range(3):
        g.replay()
        s.synchronize()
        eb.step(iters=2, shift=True)
        torch.cuda.synchronize()
        # eager work between replays
        _ = (torch.ones(1024, device="cuda") * 2).sum().item()
        for ca, cb in zip(a_ctl, b_ctl):
            assert np.array_equal(ca.U.cpu().numpy(), cb.U.cpu().numpy())
            assert ca.stats() == cb.stats()
        assert np.array_equal(ga.u0.cpu().numpy(), eb.u0.cpu().numpy())
        assert not ga.u0.cpu().numpy()[[c.m == 1 for c in a_ctl]][:, 1:].any()


def test_batch_error_paths():
    lane = Controller(workloads.cartpole(K=256, schedule=LANE))
    ws = Controller(workloads.cartpole(K=256, schedule=WS))
    x = torch.tensor(workloads.x0_for(workloads.cartpole()), device="cuda")
    with pytest.raises(native.MppiError) as e:
        Batch([lane, ws], [x, x])
    assert e.value.code == native.C["MPPI_EINVAL"]
    dbg = Controller(workloads.cartpole(K=256, schedule=LANE, debug_dump=1))
    with pytest.raises(native.MppiError) as e:
        Batch([lane, dbg], [x, x])
    assert e.value.code == native.C["MPPI_EUNSUPPORTED"]
    # controllers whose own iteration is not fused: far above and just above
    # the limits (64 lane workgroups, 256 wave-specialised)
    for cfg in (workloads.cartpole(K=200_000, T=5, schedule=LANE),
                workloads.cartpole(K=16_385, T=5, schedule=LANE),
                workloads.cartpole(K=16_385, T=5, schedule=WS)):
        big = Controller(cfg)
        with pytest.raises(native.MppiError) as e:
            Batch([big], [x])
        assert e.value.code == native.C["MPPI_EUNSUPPORTED"]


@pytest.mark.parametrize("launch", [GRID, PERSISTENT])
def test_per_model_sub_batches_equal_individual_controllers(launch):
    """The autotuner's per-model layout: one sub-batch per model (each a
    kernel of that model's variants only) on its own stream, stepped
    together and replayed from one graph captured across the streams."""
    cset = [(cfg, x0) for cfg, x0 in _controller_set(LANE, n=10, seed=31)
            if cfg["dynamics"] != 0]
    cfgs = [c for c, _ in cset]
    states = [torch.tensor(x0, device="cuda") for _, x0 in cset]
    U0s = [workloads.U0_for(c, "random", seed=c["controller_id"] + 3) for c in cfgs]
    ctls, group = autotune.make_batch(cfgs, states, (LANE, launch, True), U0s)
    assert len(group.batches) == 2
    b_ctl, b_x = _make(cset)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        group.step(iters=1, shift=True)
    for rep in range(3):
        g.replay()
        torch.cuda.synchronize()
        for c, x in zip(b_ctl, b_x):
            c.control_step(x, 1)
        torch.cuda.synchronize()
        _ = (torch.ones(1024, device="cuda") * 2).sum().item()  # eager work between replays
        for i, (ca, cb) in enumerate(zip(ctls, b_ctl)):
            assert np.array_equal(ca.S.cpu().numpy(), cb.S.cpu().numpy()), (rep, i)
            np.testing.assert_array_max_ulp(ca.U.cpu().numpy(), cb.U.cpu().numpy(), maxulp=1)
            assert ca.stats()["iteration"] == cb.stats()["iteration"] == rep + 1


def test_autotuner_times_every_layout():
    cset = _controller_set(LANE, n=8, seed=41)
    cfgs = [c for c, _ in cset]
    states = [torch.tensor(x0, device="cuda") for _, x0 in cset]
    plan, report = autotune.choose_plan(cfgs, states, ticks=2, warmup=1)
    print("autotune", report, flush=True)
    assert len(report["timings_ms"]) == len(autotune.PLANS)
    assert report["plan"] == autotune.plan_name(plan)
    assert min(report["timings_ms"].values()) == report["timings_ms"][report["plan"]]
