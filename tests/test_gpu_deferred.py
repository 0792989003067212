"""The deferred-update form of the rollout, used when a controller has more
workgroups than the fused epilogue combines (either schedule): every
workgroup publishes its weighted perturbation sums P[wg][r] of eq. (37), the
last one to arrive forms the statistics and the rescales, and a separate
kernel applies eq. (36) from the partials.  The wave-specialised form keeps
its 64-sample tiles on chip when they fit and then stores no perturbations.

  * against the staged form (rollout, then the update kernel over the stored
    perturbations) on the same seeded inputs, over two iterations (arrival
    counters reset, iteration counter advanced): costs and perturbations
    bitwise, weights to fp64 rounding, U to one fp32 ulp;
  * against eq. (36) formed by the oracle (its weights() and update(), fp64)
    from the device's own costs and perturbations: U to one fp32 ulp;
  * all costs non-finite: U unchanged, the status reported, the iteration
    counted."""

import numpy as np
import pytest

from oracle import mppi as omppi
from paper_1807_06108_amd import native, workloads
from paper_1807_06108_amd.controller import Controller

pytestmark = pytest.mark.gpu

LANE = native.C["MPPI_SCHED_LANE"]
WS = native.C["MPPI_SCHED_WAVE_SPECIALISED"]

# (preset, K, T, schedule, tile on chip): one-sample-per-lane controllers
# just above the fused limit of 64 workgroups of 256 samples (a ragged last
# workgroup) and above 512; one row block (R = 48); two row blocks, the
# second ragged (R = 70); many partials per chunk; the wave-specialised
# schedule just above its fused limit of 256 workgroups of 64 samples and
# far above it, its tile on chip where two workgroups still fit a compute
# unit's LDS (T = 20; the quadrotor's T = 12 and 20) and in HBM otherwise
# (T = 600; the quadrotor's T = 100)
CASES = [
    ("cartpole_single", 16_385, 30, LANE, False),
    ("quadrotor_hover", 16_385, 20, WS, True),
    ("double_integrator", 131_329, 9, LANE, False),
    ("cartpole_single", 140_000, 20, LANE, False),
    ("quadrotor_hover", 140_000, 12, LANE, False),
    ("cartpole_single", 300_000, 70, LANE, False),
    ("cartpole_single", 40_001, 20, WS, True),
    ("quadrotor_hover", 40_000, 12, WS, True),
    ("cartpole_single", 33_000, 600, WS, False),
    ("quadrotor_hover", 33_000, 100, WS, False),
]


def _ulps(a, b):
    """|a - b| in units of the fp32 spacing at b (at least 1e-12: the fp64
    rounding of the sums, for a value that happens to lie near zero)."""
    b32 = np.abs(np.asarray(b, dtype=np.float32))
    unit = np.maximum(np.spacing(b32).astype(np.float64), 1e-12)
    return np.abs(np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)) / unit


def _eps_or_none(ctl):
    try:
        return ctl.eps.cpu().numpy()
    except native.MppiError as e:
        assert e.code == native.C["MPPI_EUNSUPPORTED"]
        return None


@pytest.mark.parametrize("preset,K,T,sched,on_chip", CASES)
def test_deferred_matches_staged_and_eq36(preset, K, T, sched, on_chip):
    cfg = workloads.PRESETS[preset](K=K, T=T, schedule=sched)
    U0 = workloads.U0_for(cfg, "random")
    x0 = workloads.x0_for(cfg)
    print("case", preset, K, T, sched, flush=True)
    a = Controller(cfg, U0)  # deferred (step)
    b = Controller(cfg, U0)  # staged (rollout + update)
    for it in range(2):
        U_in = a.U.cpu().numpy().astype(np.float64)
        a.step(x0, 1)
        b.rollout(x0)
        b.update()
        S, Sb = a.S.cpu().numpy(), b.S.cpu().numpy()
        eps, epsb = _eps_or_none(a), b.eps.cpu().numpy()
        assert np.array_equal(S, Sb)
        assert (eps is None) == on_chip
        assert eps is None or np.array_equal(eps, epsb)
        eps = epsb
        W = a.W.cpu().numpy()
        assert np.allclose(W, b.W.cpu().numpy(), rtol=1e-12, atol=1e-300)
        sa, sb = a.stats(), b.stats()
        assert sa["status"] == 0 and sa["iteration"] == sb["iteration"] == it + 1
        assert sa["rho"] == sb["rho"] and sa["n_finite"] == sb["n_finite"] == K
        U, Ub = a.U.cpu().numpy(), b.U.cpu().numpy()
        np.testing.assert_array_max_ulp(U, Ub, maxulp=1)
        # eq. (36) with the oracle's weights of the device costs
        w, rho, eta, status = omppi.weights(S, float(omppi.f32(cfg["lambda"])))
        assert status == omppi.STATUS_OK and sa["rho"] == rho
        assert abs(sa["eta"] - eta) <= 1e-12 * eta
        ref = omppi.update(U_in.reshape(T, -1), w, np.transpose(eps, (2, 0, 1)).astype(np.float64),
                           float(omppi.f32(cfg["alpha"])))
        err = _ulps(U, ref).max()
        print("  iteration %d: U vs eq. (36) %.2f ulp" % (it, err), flush=True)
        assert err <= 1.0
        # the next iteration starts both from the same sequence
        b.set_U(U)


@pytest.mark.parametrize("K,sched", [(140_000, LANE), (40_001, WS)])
def test_deferred_all_nonfinite_leaves_U_unchanged(K, sched):
    cfg = workloads.cartpole(K=K, T=20, schedule=sched)
    U0 = workloads.U0_for(cfg, "random")
    ctl = Controller(cfg, U0)
    ctl.step(np.full(4, np.nan, dtype=np.float32), 1)
    st = ctl.stats()
    assert st["status"] == native.C["MPPI_ENONFINITE"] and st["n_finite"] == 0
    assert st["iteration"] == 1
    assert np.array_equal(ctl.U.cpu().numpy(), U0)
    ctl.step(workloads.x0_for(cfg), 1)
    st = ctl.stats()
    assert st["status"] == 0 and st["iteration"] == 2 and st["n_finite"] == cfg["K"]


# the kernel variants of the deferred form: the quadrotor's full noise
# covariance (Sigma_D = L L^T), the SO cost form, no jumps; each just above
# its schedule's fused limit, deferred step against the staged pair
VARIANTS = [
    ("quadrotor_hover", dict(full_sigma=1, sigma_L=workloads.random_cholesky(4, 0.6, seed=12))),
    ("quadrotor_hover", dict(cost_form=1)),
    ("cartpole_single", dict(cost_form=1)),
    ("cartpole_single", dict(nu=0.0)),
    ("double_integrator", dict(count_law=1, nu=5.0)),
]


@pytest.mark.parametrize("sched,K", [(LANE, 16_385), (WS, 16_448)])
@pytest.mark.parametrize("preset,over", VARIANTS)
def test_deferred_variants_match_staged(preset, over, sched, K):
    cfg = workloads.PRESETS[preset](K=K, T=12, schedule=sched, **over)
    U0 = workloads.U0_for(cfg, "random")
    x0 = workloads.x0_for(cfg)
    print("case", preset, sorted(over), sched, K, flush=True)
    a = Controller(cfg, U0)
    b = Controller(cfg, U0)
    a.step(x0, 1)
    b.rollout(x0)
    b.update()
    assert np.array_equal(a.S.cpu().numpy(), b.S.cpu().numpy())
    eps = _eps_or_none(a)
    assert eps is None or np.array_equal(eps, b.eps.cpu().numpy())
    sa, sb = a.stats(), b.stats()
    assert sa["iteration"] == sb["iteration"] == 1 and sa["rho"] == sb["rho"]
    assert sa["n_finite"] == sb["n_finite"] and abs(sa["eta"] - sb["eta"]) <= 1e-12 * sb["eta"]
    np.testing.assert_array_max_ulp(a.U.cpu().numpy(), b.U.cpu().numpy(), maxulp=1)
