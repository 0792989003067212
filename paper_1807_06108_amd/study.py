"""Closed-loop robustness study: MPPI that samples the jumps ("new", the
controller's jump rate and amplitude equal the plant's) against MPPI that
samples Gaussian noise only ("old", jump rate 0), on the cartpole swing-up
and balance task under plant disturbances with Gaussian noise and
compound-Poisson jumps (Sec. VI, Table 1: success rates of both algorithms as
the plant's jump amplitude and rate vary).

Every trial is one resident controller; all trials of one condition (both
algorithms) advance together, one pool tick per control step, with the
plant stepped on the device from each controller's own state.  Trial i of
both algorithms sees the same plant disturbance sequence (paired
comparison).  Success: the pole stays within `upright_tol` rad of upright
(cos theta >= cos upright_tol) over the last `hold_steps` control steps.

The paper does not give its time step, horizon, units of the jump rate and
amplitude, or success criterion, so only the trend is comparable.

Run:  python -m paper_1807_06108_amd.study [--trials 100] [--steps 500]
"""

import argparse
import json
import math
import time

import numpy as np
import torch

from . import workloads
from .controller import Controller, Pool

# plant jump conditions (rate /s, amplitude N) at Gaussian noise SIGMA (N):
# an amplitude sweep of 1, 1.5, 2 and 3 times SIGMA at a fixed rate and a
# rate sweep at twice SIGMA, the structure of Table 1
SIGMA = 5.0
CARTPOLE_CONDITIONS = ((2.5, 5.0), (2.5, 7.5), (2.5, 10.0), (2.5, 15.0),
                       (1.0, 10.0), (5.0, 10.0))


def cartpole_trial_config(nu, sigma_J, trial, K=1000, T=75, sigma=1.0, cost_form=0):
    """Controller of one cartpole trial; nu = 0 gives the Gaussian-only one."""
    return workloads.cartpole(K=K, T=T, nu=float(nu), sigma=[float(sigma), 0, 0, 0],
                              sigma_J=[float(sigma_J), 0, 0, 0], cost_form=int(cost_form),
                              seed=0x5EED0000 + trial, controller_id=trial)


def swing_up_success(theta, hold_steps, upright_tol):
    """theta [trials, steps] -> bool [trials]: upright over the last hold_steps."""
    tail = np.asarray(theta)[:, -hold_steps:]
    return np.all(np.cos(tail) >= math.cos(upright_tol), axis=1)


def run_condition(nu_p, sJ_p, trials=100, steps=500, iters=1, sigma_p=SIGMA, K=1000, T=75,
                  hold_steps=100, upright_tol=0.25, plant_seed=7, cost_form=0):
    """Success rates (new, old) and per-trial outcomes under plant jumps at
    rate nu_p /s with N(0, sJ_p^2) amplitudes plus N(0, sigma_p^2) noise;
    both controllers sample Gaussian noise of the plant's sigma_p."""
    cfgs = ([cartpole_trial_config(nu_p, sJ_p, i, K, T, sigma_p, cost_form) for i in range(trials)]
            + [cartpole_trial_config(0.0, sJ_p, i, K, T, sigma_p, cost_form) for i in range(trials)])
    ctls = [Controller(c) for c in cfgs]
    pool = Pool(ctls, 1)
    dt = cfgs[0]["dt"]
    n = len(ctls)
    dist = np.zeros((n, steps, 4), dtype=np.float32)
    for i in range(trials):
        d = workloads.plant_disturbance(steps, dt, sigma_p, nu_p, sJ_p, seed=plant_seed * 100003 + i)
        dist[i, :, 0] = d
        dist[trials + i, :, 0] = d
    x = np.zeros((n, 12), dtype=np.float32)
    x[:, :4] = workloads.x0_for(cfgs[0])
    ids = np.arange(n, dtype=np.int32)
    theta = np.zeros((n, steps), dtype=np.float64)
    for s in range(steps):
        pool.tick(ids, x, dist[:, s], iters=iters, slot=0)
        torch.cuda.current_stream().synchronize()
        rid, u0, xn = pool.results(0)
        x[rid] = xn
        theta[rid, s] = xn[:, 2]
    ok = swing_up_success(theta, hold_steps, upright_tol)
    pool.close()
    for c in ctls:
        c.close()
    return {"plant_nu": nu_p, "plant_sigma_J": sJ_p, "trials": trials,
            "new": float(ok[:trials].mean()), "old": float(ok[trials:].mean()),
            "new_ok": ok[:trials], "old_ok": ok[trials:]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trials", type=int, default=100)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--iters", type=int, default=1)
    ap.add_argument("--K", type=int, default=1000)
    ap.add_argument("--T", type=int, default=75)
    ap.add_argument("--cost-forms", default="0,1", help="0 IT (eqs. 34-35), 1 SO (eq. 49)")
    args = ap.parse_args()
    torch.cuda.set_device(0)
    rows = []
    for form in [int(f) for f in args.cost_forms.split(",")]:
        for nu_p, sJ_p in CARTPOLE_CONDITIONS:
            t0 = time.perf_counter()
            r = run_condition(nu_p, sJ_p, args.trials, args.steps, args.iters, K=args.K, T=args.T,
                              cost_form=form)
            r.pop("new_ok")
            r.pop("old_ok")
            r["cost_form"] = form
            r["seconds"] = round(time.perf_counter() - t0, 2)
            rows.append(r)
            print(json.dumps(r), flush=True)
    print("cost form | plant jumps (rate /s, amplitude N) | new MPPI | old MPPI")
    for r in rows:
        print("%s | nu=%g, sigma_J=%g | %3.0f%% | %3.0f%%" % (
            "IT" if r["cost_form"] == 0 else "SO", r["plant_nu"], r["plant_sigma_J"],
            100 * r["new"], 100 * r["old"]))


if __name__ == "__main__":
    main()
