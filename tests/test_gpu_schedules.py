"""The rollout schedules (one sample per lane; wave-specialised producer /
consumer) and the fused / staged update paths compute the same iteration:
the same draws from the same counters and the same fp32 arithmetic, so their
outputs agree bitwise.  Also checked against the oracle on ragged shapes."""

import numpy as np
import pytest

from gpu_util import check_S, run_rollout, staged_update
from paper_1807_06108_amd import native, workloads
from paper_1807_06108_amd.controller import Controller

pytestmark = pytest.mark.gpu

LANE = native.C["MPPI_SCHED_LANE"]
WS = native.C["MPPI_SCHED_WAVE_SPECIALISED"]


def _run(cfg, U0, x0, iters, staged=False):
    """(S, U, eps, W, stats) after `iters` iterations; eps is None where the
    iterations kept the perturbations on chip (fused wave-specialised form)
    and stored none."""
    ctl = Controller(cfg, U0)
    if staged:
        for _ in range(iters):
            ctl.rollout(x0)
            ctl.update()
    else:
        ctl.step(x0, iters)
    try:
        eps = ctl.eps.cpu().numpy()
    except native.MppiError as e:
        # only a fused wave-specialised iteration keeps them on chip
        assert e.code == native.C["MPPI_EUNSUPPORTED"] and not staged
        assert cfg.get("schedule", 0) != LANE
        eps = None
    return (ctl.S.cpu().numpy(), ctl.U.cpu().numpy(), eps, ctl.W.cpu().numpy(), ctl.stats())


@pytest.mark.parametrize("preset,K,T", [
    ("cartpole_single", 1000, 37), ("cartpole_single", 65, 16), ("cartpole_single", 1, 5),
    ("quadrotor_hover", 700, 33), ("quadrotor_hover", 64, 3), ("double_integrator", 300, 100),
    ("cartpole_mpc", 4096, 100),
    # wave-specialised fused updates with many partials per row
    ("quadrotor_hover", 8192, 100), ("cartpole_mpc", 16384, 100), ("quadrotor_hover", 1100, 60),
])
def test_schedules_and_update_paths_agree(preset, K, T):
    """Costs and perturbations agree bitwise.  The weights and the update sum
    the same fp64 terms grouped by workgroup (64 or 256 samples), so they
    agree to fp64 rounding: W to 1e-12 relative, U to one fp32 ulp."""
    cfg = workloads.PRESETS[preset](K=K, T=T)
    U0 = workloads.U0_for(cfg, "random")
    x0 = workloads.x0_for(cfg)
    print("case", preset, K, T, flush=True)
    ref = _run(dict(cfg, schedule=LANE), U0, x0, 1)
    for sched, staged in ((WS, False), (LANE, True), (WS, True)):
        S, U, eps, W, st = _run(dict(cfg, schedule=sched), U0, x0, 1, staged)
        assert np.array_equal(S, ref[0]), (sched, staged)
        # fused wave-specialised iterations keep eps on chip when the tile
        # fits: T <= 496 for the one-channel models, T <= 108 for the quadrotor
        assert (eps is None) == (sched == WS and not staged
                                 and T <= (108 if cfg["dynamics"] == 2 else 496)), (sched, staged)
        assert eps is None or np.array_equal(eps, ref[2]), (sched, staged)
        np.testing.assert_array_max_ulp(U, ref[1], maxulp=1)
        assert np.allclose(W, ref[3], rtol=1e-12, atol=1e-300)
        assert st["rho"] == ref[4]["rho"] and st["n_finite"] == ref[4]["n_finite"]
        assert abs(st["eta"] - ref[4]["eta"]) <= 1e-12 * ref[4]["eta"]


@pytest.mark.parametrize("sched", [LANE, WS])
@pytest.mark.parametrize("over", [dict(cost_form=1), dict(nu=0.0), dict(count_law=1, nu=30.0),
                                  dict(c=0.5, alpha=0.7)])
def test_schedules_match_the_oracle(sched, over):
    cfg = workloads.quadrotor(K=333, T=41, schedule=sched, **over)
    U0 = workloads.U0_for(cfg, "random")
    ctl, ref, _, _ = run_rollout(cfg, U0=U0)
    check_S(ctl, ref, exclude=ref["margin"] < 1e-4)
    staged_update(ctl, ref)


def test_large_K_uses_lane_schedule_and_deferred_update():
    # above the AUTO schedule's wave-specialised limit and the fused limit of
    # 512 workgroups: both schedules defer the update to the partials'
    # kernel; the lane schedule stores its perturbations, the wave-specialised
    # one keeps its tiles on chip (T = 20) and stores none
    K = 200_000
    cfg = workloads.cartpole(K=K, T=20)
    U0 = workloads.U0_for(cfg, "random")
    x0 = workloads.x0_for(cfg)
    a = _run(cfg, U0, x0, 1)
    b = _run(dict(cfg, schedule=WS), U0, x0, 1)
    assert a[2] is not None and b[2] is None
    assert np.array_equal(a[0], b[0])
    np.testing.assert_array_max_ulp(a[1], b[1], maxulp=1)
    W = a[3]
    assert abs(W.sum() - 1) < 1e-12


@pytest.mark.parametrize("preset,K,T,iters", [
    ("cartpole_mpc", 4096, 100, 5), ("quadrotor_hover", 1000, 37, 2),
    ("cartpole_single", 300, 1500, 2), ("double_integrator", 64, 1, 1),
    ("cartpole_single", 150_000, 8, 2), ("quadrotor_hover", 8192, 100, 2),
])
def test_control_step_equals_step_then_shift(preset, K, T, iters):
    """The fused control step (shift and u_0 folded into the last
    iteration's kernel) gives exactly the sequence and u_0 of step + shift."""
    cfg = workloads.PRESETS[preset](K=K, T=T)
    U0 = workloads.U0_for(cfg, "random")
    x0 = workloads.x0_for(cfg)
    print("case", preset, K, T, iters, flush=True)
    a = Controller(cfg, U0)
    a.step(x0, iters)
    u0_a = a.shift().cpu().numpy()
    b = Controller(cfg, U0)
    u0_b = b.control_step(x0, iters).cpu().numpy()
    assert np.array_equal(u0_a, u0_b)
    assert np.array_equal(a.U.cpu().numpy(), b.U.cpu().numpy())
    assert a.stats() == b.stats()
    # a second control step continues from the shifted sequence
    a.step(x0, 1)
    u1_a = a.shift().cpu().numpy()
    u1_b = b.control_step(x0, 1).cpu().numpy()
    assert np.array_equal(u1_a, u1_b)

