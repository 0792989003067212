"""Closed-loop study harness: paired trials, deterministic outcomes, and the
special case where both algorithms coincide (no plant jumps to sample)."""

import numpy as np
import pytest

from paper_1807_06108_amd import study

pytestmark = pytest.mark.gpu


def test_study_is_deterministic_and_paired():
    print("study: 6 trials x 80 steps", flush=True)
    a = study.run_condition(2.5, 10.0, trials=6, steps=80, hold_steps=20)
    b = study.run_condition(2.5, 10.0, trials=6, steps=80, hold_steps=20)
    assert np.array_equal(a["new_ok"], b["new_ok"]) and np.array_equal(a["old_ok"], b["old_ok"])
    assert 0.0 <= a["new"] <= 1.0 and 0.0 <= a["old"] <= 1.0


def test_without_plant_jumps_both_algorithms_are_the_same_controller():
    # nu = 0: the "new" controller samples no jumps either, so both columns
    # run identical controllers on identical disturbances
    r = study.run_condition(0.0, 10.0, trials=6, steps=80, hold_steps=20)
    assert np.array_equal(r["new_ok"], r["old_ok"])


def _euler(cfg, x, v, gust):
    """The oracle's explicit Euler step of the trial's model (fp32 inputs)."""
    from oracle import models
    from oracle import mppi as omppi
    return models.euler_step(cfg["dynamics"], omppi.f32(x)[None], np.asarray(v, np.float64)[None],
                             np.asarray(gust, np.float64)[None], float(omppi.f32(cfg["dt"])),
                             omppi.f32(cfg["params"]))[0]


def _control_jacobian_norm(cfg, x, v, gust, h=1e-4):
    """max over state entries of sum_j |d x_next / d v_j| (central
    differences of the oracle's Euler step): the sensitivity of the plant
    step to its applied control."""
    m = len(v)
    J = np.zeros((len(x), m))
    for j in range(m):
        e = np.zeros(m)
        e[j] = h
        J[:, j] = (_euler(cfg, x, v + e, gust) - _euler(cfg, x, v - e, gust)) / (2 * h)
    return float(np.abs(J).sum(axis=1).max())


@pytest.mark.parametrize("model", ["cartpole", "quadrotor"])
def test_trial_steps_match_the_oracle(model):
    """The study's closed loop, step by step against the oracle: one trial of
    each algorithm ("new" samples the plant's jumps, "old" does not) runs in
    one pool, one tick per control step, with the plant disturbances of the
    study (quadrotor: thrust noise plus world-frame gusts in disturbance
    words 4-6).  The oracle runs the loop; before each tick every controller
    is given the oracle's control sequence, and the tick starts from the
    oracle's state.  Per step: every path cost (1e-4 relative), u_0 within
    the first-order bound of the cost error, and the plant's next state
    against the oracle's Euler step under u_0 + disturbance and the gust."""
    from gpu_util import U_ATOL, s_err_ratio
    from oracle import mppi as omppi
    from paper_1807_06108_amd.controller import Controller, Pool
    from test_gpu_full_parity import first_order_bound
    import torch
    steps = 8
    if model == "cartpole":
        nu_p, sJ_p = 2.5, 10.0
        cfgs = [study.cartpole_trial_config(nu_p, sJ_p, 0, sigma=study.SIGMA),
                study.cartpole_trial_config(0.0, sJ_p, 0, sigma=study.SIGMA)]
        d = np.zeros((steps, 8), dtype=np.float32)
        d[:, 0] = study.workloads.plant_disturbance(steps, cfgs[0]["dt"], study.SIGMA, nu_p,
                                                    sJ_p, seed=7 * 100003)
    else:
        # a gust rate at which most of the steps carry a gust
        nu_p, sJ_p = 60.0, 100.0
        cfgs = [study.quadrotor_trial_config(nu_p, sJ_p, 0),
                study.quadrotor_trial_config(0.0, sJ_p, 0)]
        d = study.quadrotor_disturbances(steps, cfgs[0]["dt"], cfgs[0]["sigma"][0], nu_p, sJ_p,
                                         seed=11 * 100003)
        assert (np.abs(d[:, 4:7]).sum(axis=1) > 0).sum() >= steps // 4
    n, m = (4, 1) if model == "cartpole" else (12, 4)
    ctls = [Controller(c) for c in cfgs]
    pool = Pool(ctls, 1)
    x = [study.workloads.x0_for(c).astype(np.float64) for c in cfgs]
    U = [study.workloads.U0_for(c).astype(np.float64) for c in cfgs]
    ids = np.arange(2, dtype=np.int32)
    for s in range(steps):
        print("%s trial: control step %d" % (model, s), flush=True)
        states = np.zeros((2, 12), dtype=np.float32)
        for j in range(2):
            U[j] = omppi.f32(U[j])
            ctls[j].set_U(U[j])
            states[j, :n] = x[j]
        torch.cuda.synchronize()
        pool.tick(ids, states, np.repeat(d[s][None], 2, axis=0), iters=1, slot=0)
        torch.cuda.synchronize()
        rid, u0, xn = pool.results(0)
        assert list(rid) == [0, 1]
        for j, cfg in enumerate(cfgs):
            ref = omppi.iteration(cfg, x[j], U[j], s)
            S = ctls[j].S.cpu().numpy()
            excl = ref["margin"] < 1e-4
            assert s_err_ratio(S, ref)[~excl].max() <= 1.0
            flip = excl & ((S > 1e4) != (ref["S"] > 1e4))
            assert (ref["w"][flip] < 1e-30).all()
            dS = np.where(flip, 0.0, S - ref["S"])
            bound = U_ATOL + first_order_bound(ref["w"], ref["eps"], dS,
                                               float(omppi.f32(cfg["lambda"])))
            u0_ref, U_next = omppi.shift(ref["U"], omppi.f32(cfg["u_init"][:m]))
            du = np.abs(u0[j, :m] - u0_ref)
            assert (du <= bound[0]).all(), (du, bound[0])
            gust = d[s, 4:7] if model == "quadrotor" else np.zeros(3)
            v_ref = np.float32(u0_ref) + d[s, :m]
            x_ref = _euler(cfg, states[j, :n], v_ref, gust)
            tol = 1e-5 * (1.0 + np.abs(x_ref).max()) + \
                _control_jacobian_norm(cfg, states[j, :n], v_ref, gust) * du.max()
            assert np.abs(xn[j, :n] - x_ref).max() <= tol
            x[j] = x_ref
            U[j] = U_next
    pool.close()


def test_pool_plant_applies_the_gust():
    """A pool tick that leaves u_0 exact (no noise: U is unchanged, so u_0 is
    the first entry of the sequence) with a world-frame body force in
    disturbance words 4-6: the quadrotor plant's next state equals the
    oracle's Euler step with that gust."""
    from oracle import mppi as omppi
    from paper_1807_06108_amd.controller import Controller, Pool
    import torch
    cfg = study.workloads.quadrotor(K=64, T=10, sigma=[0.0] * 4, nu=0.0)
    U0 = study.workloads.U0_for(cfg, "random")
    ctl = Controller(cfg, U0)
    pool = Pool([ctl], 1)
    g = np.random.default_rng(5)
    x = study.workloads.x0_for(cfg) + 0.05 * g.standard_normal(12).astype(np.float32)
    dist = np.zeros((1, 8), dtype=np.float32)
    dist[0, :4] = 0.3 * g.standard_normal(4)
    dist[0, 4:7] = [40.0, -25.0, 60.0]
    states = np.zeros((1, 12), dtype=np.float32)
    states[0] = x
    pool.tick(np.zeros(1, np.int32), states, dist, iters=1, slot=0)
    torch.cuda.synchronize()
    _, u0, xn = pool.results(0)
    assert np.array_equal(u0[0], U0[0])
    ref = _euler(cfg, x, np.float32(U0[0]) + dist[0, :4], dist[0, 4:7])
    no_gust = _euler(cfg, x, np.float32(U0[0]) + dist[0, :4], np.zeros(3))
    assert np.abs(ref - no_gust).max() > 1e-2  # the gust matters at this size
    assert np.abs(xn[0] - ref).max() < 1e-5 * (1.0 + np.abs(ref).max())
    pool.close()
