"""Full Gaussian covariance Sigma_D = L L^T (Sec. IV-B eps_D ~ N(0, Sigma_D)):
the library's draws, costs and update against the oracle in both schedules
and both cost forms, and the diagonal factor against the diagonal form."""

import numpy as np
import pytest

from gpu_util import check_S, near_crash, run_rollout, staged_update
from oracle import noise as onoise
from paper_1807_06108_amd import native, workloads
from paper_1807_06108_amd.controller import Batch, Controller

pytestmark = pytest.mark.gpu

LANE = native.C["MPPI_SCHED_LANE"]
WS = native.C["MPPI_SCHED_WAVE_SPECIALISED"]


def _cfg(**over):
    L16 = workloads.random_cholesky(4, 0.6, seed=12)
    base = dict(K=700, T=33, full_sigma=1, sigma_L=L16)
    base.update(over)
    return workloads.quadrotor(**base)


@pytest.mark.parametrize("sched", [LANE, WS])
def test_full_covariance_draws_match_the_oracle(sched):
    cfg = _cfg(schedule=sched, debug_dump=1, K=300, T=20)
    ctl, ref, _, _ = run_rollout(cfg)
    zD, N, zJ = [t.cpu().numpy() for t in ctl.debug_draws()]
    assert np.array_equal(N, ref["N"])
    assert np.abs(zD - ref["z_D"]).max() < 1e-5
    eps = ctl.eps.cpu().numpy().transpose(2, 0, 1)
    assert np.abs(eps - ref["eps"]).max() < 2e-5


@pytest.mark.parametrize("sched", [LANE, WS])
@pytest.mark.parametrize("over", [dict(), dict(c=0.5), dict(c=2.0, nu=0.0), dict(cost_form=1)])
def test_full_covariance_costs_and_update_match_the_oracle(sched, over):
    cfg = _cfg(schedule=sched, **over)
    U0 = workloads.U0_for(cfg, "random", seed=6)
    ctl, ref, _, _ = run_rollout(cfg, U0=U0)
    check_S(ctl, ref, exclude=near_crash(ref))
    staged_update(ctl, ref)


def test_diagonal_factor_equals_the_diagonal_form():
    sig = [0.5, 0.3, 0.7, 0.4]
    L16 = [0.0] * 16
    for j in range(4):
        L16[5 * j] = sig[j]
    a = workloads.quadrotor(K=500, T=30, sigma=sig, c=0.7)
    b = dict(a, full_sigma=1, sigma_L=L16)
    x0 = workloads.x0_for(a)
    U0 = workloads.U0_for(a, "random", seed=8)
    ca, cb = Controller(a, U0), Controller(b, U0)
    ca.rollout(x0)
    cb.rollout(x0)
    Sa, Sb = ca.S.cpu().numpy(), cb.S.cpu().numpy()
    e = ca.eps.cpu().numpy().astype(np.float64)  # [T, m, K]
    assert np.array_equal(e, cb.eps.cpu().numpy())
    # with eps bitwise equal the trajectories are equal, and S differs only
    # by the rounding of the importance-sampling terms of eq. (35), whose
    # Sigma^-1 is 1/sigma^2 in one form and L^-T L^-1 in the other: a few
    # fp32 ulps of each term.  S itself can cancel to ~0 while its terms sum
    # to ~100 in magnitude, so the bound scales with the terms, not with S.
    U = np.asarray(U0, dtype=np.float64).reshape(a["T"], 4)
    iv = 1.0 / np.square(np.asarray(sig))[None, :, None]
    lam = a["lambda"]
    terms = (np.abs(lam * 0.7 * U[:, :, None] * e * iv).sum(axis=(0, 1))
             + np.abs(0.5 * lam * 0.3 * e * e * iv).sum(axis=(0, 1)))
    tol = 1e-6 * np.abs(Sb) + 8 * 2.0**-24 * terms + 1e-6
    assert np.all(np.abs(Sa - Sb) <= tol)


def test_one_channel_covariance_is_the_diagonal_form():
    a = workloads.cartpole(K=512, T=40, sigma=[1.3, 0, 0, 0])
    L16 = [1.3] + [0.0] * 15
    b = dict(a, full_sigma=1, sigma_L=L16, sigma=[0.0] * 4)
    x0 = workloads.x0_for(a)
    ca, cb = Controller(a), Controller(b)
    ca.step(x0, 2)
    cb.step(x0, 2)
    assert np.array_equal(ca.S.cpu().numpy(), cb.S.cpu().numpy())
    assert np.array_equal(ca.U.cpu().numpy(), cb.U.cpu().numpy())


def test_batches_refuse_a_full_covariance():
    import torch
    ctl = Controller(_cfg(K=256, T=10))
    x = torch.tensor(workloads.x0_for(ctl.cfg), device="cuda")
    with pytest.raises(native.MppiError) as e:
        Batch([ctl], [x])
    assert e.value.code == native.C["MPPI_EUNSUPPORTED"]
