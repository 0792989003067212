"""The no-allocation control step (library-owned static scratch) against the
context control step: same kernels, same noise stream, so u_0 and the
shifted sequence agree bitwise.  Two calls in a row on the one array, the
second with a smaller configuration; a configuration above the array's size
is refused."""

import ctypes

import numpy as np
import pytest
import torch

from paper_1807_06108_amd import native, workloads
from paper_1807_06108_amd.controller import Controller

pytestmark = pytest.mark.gpu


def _static_step(cfg, U, x0, iters, stream=None):
    """One call of mppi_jump_control_step_static; returns (rc, u0, U')."""
    n, m, q = native.dims(cfg["dynamics"])
    c = native.make_config(cfg)
    Ud = torch.tensor(np.asarray(U, np.float32).reshape(cfg["T"], m), device="cuda")
    xd = torch.tensor(np.asarray(x0, np.float32), device="cuda")
    u0 = torch.full((m,), np.nan, dtype=torch.float32, device="cuda")
    s = stream if stream is not None else torch.cuda.current_stream()
    rc = native.lib().mppi_jump_control_step_static(
        ctypes.byref(c), ctypes.c_void_p(Ud.data_ptr()), ctypes.c_void_p(xd.data_ptr()),
        int(iters), ctypes.c_void_p(u0.data_ptr()), ctypes.c_void_p(s.cuda_stream))
    torch.cuda.synchronize()
    return rc, u0.cpu().numpy(), Ud.cpu().numpy()


def _context_step(cfg, U, x0, iters):
    ctl = Controller(cfg, U)
    u0 = ctl.control_step(x0, iters).cpu().numpy()
    return u0, ctl.U.cpu().numpy()


@pytest.mark.parametrize("first,second", [
    # quadrotor hover shape (13.9 MB of scratch: its largest use here), then
    # the cartpole MPC shape
    (("quadrotor_hover", {}, 1), ("cartpole_mpc", {}, 5)),
    # the cartpole MPC shape, then a ragged smaller one (lane schedule and
    # the deferred update: above 64 rollout workgroups)
    (("cartpole_mpc", {}, 5), ("cartpole_single", dict(K=150_000, T=6), 2)),
    # the wave-specialised schedule's deferred update (above 256 rollout
    # workgroups, the tile on chip), cartpole then quadrotor
    (("cartpole_single", dict(K=40_001, T=30), 2), ("quadrotor_hover", dict(K=20_000, T=25), 1)),
])
def test_static_scratch_matches_the_context_step(first, second):
    for preset, over, iters in (first, second):
        cfg = workloads.PRESETS[preset](**over)
        assert native.workspace_bytes(cfg) <= native.C["MPPI_JUMP_STATIC_SCRATCH_BYTES"]
        print("no-alloc case: %s K=%d T=%d iters=%d" % (preset, cfg["K"], cfg["T"], iters),
              flush=True)
        U0 = workloads.U0_for(cfg, "random")
        x0 = workloads.x0_for(cfg)
        u0_ref, U_ref = _context_step(cfg, U0, x0, iters)
        rc, u0, U = _static_step(cfg, U0, x0, iters)
        assert rc == native.MPPI_OK, native.lib().mppi_jump_last_error()
        assert np.array_equal(u0, u0_ref), (u0, u0_ref)
        assert np.array_equal(U, U_ref)
        # a controller continues with the next iteration indices
        cfg2 = dict(cfg, start_iteration=iters)
        ctl = Controller(cfg, U0)
        ctl.control_step(x0, iters)
        u1_ref = ctl.control_step(x0, 1).cpu().numpy()
        rc, u1, _ = _static_step(cfg2, U, x0, 1)
        assert rc == native.MPPI_OK and np.array_equal(u1, u1_ref)


def test_static_scratch_refuses_oversized_configurations():
    cfg = workloads.cartpole(K=1 << 20, T=100)
    assert native.workspace_bytes(cfg) > native.C["MPPI_JUMP_STATIC_SCRATCH_BYTES"]
    rc, u0, U = _static_step(cfg, workloads.U0_for(cfg), workloads.x0_for(cfg), 1)
    assert rc == native.C["MPPI_EWORKSPACE"]
    assert b"static maximum" in native.lib().mppi_jump_last_error()
    assert np.isnan(u0).all()  # nothing was enqueued
    bad = workloads.cartpole(debug_dump=1)
    rc, _, _ = _static_step(bad, workloads.U0_for(bad), workloads.x0_for(bad), 1)
    assert rc == native.C["MPPI_EUNSUPPORTED"]
