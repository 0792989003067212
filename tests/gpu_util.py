"""Shared helpers of the GPU tests: run the library and the oracle on the same
seeded inputs and compare them."""

import numpy as np
import torch

from oracle import mppi as omppi
from paper_1807_06108_amd import workloads
from paper_1807_06108_amd.controller import Controller

S_RTOL = 1e-4   # relative to max(|S|, 1)
U_ATOL = 1e-5
# Rounding allowance of a signed sum: 16 fp32 ulps of the summed magnitudes
# of the terms of S~ (the IS cross term of eq. (35) is signed, and with a
# large nominal sequence S~ can cancel to near zero while its terms sum to
# thousands; no fp32 evaluation meets 1e-4 of such a sum, while its error
# stays at the ulp level of the terms)
S_ABS_EPS = 2.0 ** -19


def s_rel_err(S_gpu, S_ref):
    return np.abs(S_gpu - S_ref) / np.maximum(np.abs(S_ref), 1.0)


def s_err_ratio(S_gpu, ref):
    """|S_gpu - S_oracle| over its tolerance S_RTOL max(|S|, 1) + S_ABS_EPS
    S_abs (S_abs: the oracle's summed magnitudes of the terms of each S~);
    at most 1 passes."""
    tol = S_RTOL * np.maximum(np.abs(ref["S"]), 1.0) + S_ABS_EPS * ref["S_abs"]
    return np.abs(S_gpu - ref["S"]) / tol


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
    ratio = s_err_ratio(S, ref)
    if exclude is not None:
        err, ratio = err[~exclude], ratio[~exclude]
    assert ratio.max() <= 1.0, "max rel S err %.3e, err/tol %.3f" % (err.max(), ratio.max())
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
