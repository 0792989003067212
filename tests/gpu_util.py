"""Shared helpers of the GPU tests: run the library and the oracle on the same
seeded inputs and compare them."""

import numpy as np
import torch

from oracle import mppi as omppi
from paper_1807_06108_amd import workloads
from paper_1807_06108_amd.controller import Controller

S_RTOL = 1e-4   # relative to max(|S|, 1)
U_ATOL = 1e-5


def s_rel_err(S_gpu, S_ref):
    return np.abs(S_gpu - S_ref) / np.maximum(np.abs(S_ref), 1.0)


def run_rollout(cfg, x0=None, U0=None, it=0):
    """GPU rollout and oracle iteration on the same inputs."""
    x0 = workloads.x0_for(cfg) if x0 is None else x0
    U0 = workloads.U0_for(cfg) if U0 is None else U0
    print("case: dyn=%d K=%d T=%d nu=%g it=%d" % (cfg["dynamics"], cfg["K"], cfg["T"],
                                                   cfg["nu"], it), flush=True)
    ctl = Controller(cfg, U0)
    ctl.rollout(x0)
    ref = omppi.iteration(cfg, x0, U0.astype(np.float64), cfg.get("start_iteration", 0) + it)
    return ctl, ref, x0, U0


def check_S(ctl, ref, exclude=None):
    S = ctl.S.cpu().numpy()
    err = s_rel_err(S, ref["S"])
    if exclude is not None:
        err = err[~exclude]
    assert err.max() < S_RTOL, "max rel S err %.3e" % err.max()
    return S, err.max()


def near_crash(ref, tol=1e-4):
    return ref["margin"] < tol


def staged_update(ctl, ref):
    """Feed the oracle's S to the GPU update; compare U with the oracle's."""
    ctl.set_S(ref["S"])
    ctl.update()
    U = ctl.U.cpu().numpy().astype(np.float64)
    err = np.abs(U - ref["U"]).max()
    assert err < U_ATOL, "staged U err %.3e" % err
    return U, err


def sync():
    torch.cuda.synchronize()
