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

The quadrotor task of Table 2 (fly from (0, 0, 1) to (1, -1, 2) under
thrust noise and world-frame gusts, success = no crash and within 0.5 m of
the target at the end) runs the same way with --model quadrotor.

Run:  python -m paper_1807_06108_amd.study [--model cartpole|quadrotor]
      [--trials 100] [--steps 500]
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


# quadrotor (Table 2): gust conditions (rate /s, amplitude N per axis), an
# amplitude sweep at a fixed rate and a rate sweep at a fixed amplitude
QUAD_CONDITIONS = ((2.0, 25.0), (2.0, 50.0), (2.0, 100.0), (2.0, 200.0),
                   (1.0, 100.0), (4.0, 100.0))


def quadrotor_trial_config(nu, sigma_J, trial, K=3000, T=100, cost_form=1):
    """Controller of one quadrotor trial: gusts sampled at the plant's rate
    and amplitude ("new"), or none (nu = 0, "old").  The SO cost form: with
    the hover thrust as nominal control, the IT form's cross term
    lambda c U^T Sigma^-1 eps (U ~ 2.45 N against sigma = 0.5 N, summed over
    100 steps and 4 rotors) has a spread of ~100 in the exponent and swamps
    the task cost in the weights, so the IT controller never settles."""
    return workloads.quadrotor(K=K, T=T, nu=float(nu), sigma_J=[float(sigma_J)] * 3 + [0.0],
                               cost_form=int(cost_form), seed=0x5EED8000 + trial,
                               controller_id=trial)


def quadrotor_disturbances(steps, dt, sigma, nu, sigma_J, seed):
    """[steps, 8]: N(0, sigma^2) thrust noise per rotor and a world-frame gust
    sqrt(N) N(0, sigma_J^2) per axis, N ~ Poisson(nu dt), held for one step."""
    g = np.random.default_rng(seed)
    d = np.zeros((steps, 8), dtype=np.float64)
    d[:, :4] = sigma * g.standard_normal((steps, 4))
    n = g.poisson(nu * dt, size=steps)
    d[:, 4:7] = sigma_J * np.sqrt(n)[:, None] * g.standard_normal((steps, 3))
    return d.astype(np.float32)


def quadrotor_success(traj, goal, params, tol=0.5):
    """traj [trials, steps, 12] -> bool [trials]: never crashed (the model's
    rule: below z_min, or roll or pitch beyond the tilt limit) and within
    tol m of the goal position at the end."""
    tilt, zmin = params[7], params[8]
    crashed = np.any((traj[:, :, 2] < zmin) | (np.abs(traj[:, :, 6]) > tilt)
                     | (np.abs(traj[:, :, 7]) > tilt), axis=1)
    dist = np.linalg.norm(traj[:, -1, :3] - np.asarray(goal[:3]), axis=1)
    return ~crashed & (dist <= tol)


def run_quadrotor_condition(nu_p, sJ_p, trials=100, steps=500, iters=1, K=3000, T=100,
                            plant_seed=11):
    """Success rates (new, old) of the fly-to-target task under gusts at rate
    nu_p /s with N(0, sJ_p^2) amplitudes per axis and thrust noise of the
    controllers' sigma."""
    cfgs = ([quadrotor_trial_config(nu_p, sJ_p, i, K, T) for i in range(trials)]
            + [quadrotor_trial_config(0.0, sJ_p, i, K, T) for i in range(trials)])
    ctls = [Controller(c) for c in cfgs]
    pool = Pool(ctls, 1)
    dt, sigma = cfgs[0]["dt"], cfgs[0]["sigma"][0]
    n = len(ctls)
    dist = np.zeros((n, steps, 8), dtype=np.float32)
    for i in range(trials):
        d = quadrotor_disturbances(steps, dt, sigma, nu_p, sJ_p, seed=plant_seed * 100003 + i)
        dist[i] = d
        dist[trials + i] = d
    x = np.zeros((n, 12), dtype=np.float32)
    x[:] = workloads.x0_for(cfgs[0])
    ids = np.arange(n, dtype=np.int32)
    traj = np.zeros((n, steps, 12), dtype=np.float32)
    for s in range(steps):
        pool.tick(ids, x, dist[:, s], iters=iters, slot=0)
        torch.cuda.current_stream().synchronize()
        rid, u0, xn = pool.results(0)
        x[rid] = xn
        traj[rid, s] = xn
    ok = quadrotor_success(traj, cfgs[0]["x_goal"], cfgs[0]["params"])
    pool.close()
    for c in ctls:
        c.close()
    return {"model": "quadrotor", "plant_nu": nu_p, "plant_sigma_J": sJ_p, "trials": trials,
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
    ap.add_argument("--model", default="cartpole", choices=["cartpole", "quadrotor"])
    args = ap.parse_args()
    torch.cuda.set_device(0)
    rows = []
    if args.model == "quadrotor":
        for nu_p, sJ_p in QUAD_CONDITIONS:
            t0 = time.perf_counter()
            r = run_quadrotor_condition(nu_p, sJ_p, args.trials, args.steps, args.iters)
            r.pop("new_ok")
            r.pop("old_ok")
            r["seconds"] = round(time.perf_counter() - t0, 2)
            rows.append(r)
            print(json.dumps(r), flush=True)
        print("gusts (rate /s, amplitude N per axis) | new MPPI | old MPPI")
        for r in rows:
            print("nu=%g, sigma_J=%g | %3.0f%% | %3.0f%%" % (r["plant_nu"], r["plant_sigma_J"],
                                                          100 * r["new"], 100 * r["old"]))
        return
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
