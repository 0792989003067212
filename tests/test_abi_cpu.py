"""C-ABI checks that need no GPU: the library loads and exports every entry
point the header declares, the ctypes structures match the C layout, and the
pure host functions (dimensions, workspace sizing, validation, count tables,
status strings) behave as documented."""

import os
import re
import subprocess

import numpy as np
import pytest

from oracle import noise
from paper_1807_06108_amd import native, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(native.HEADER).read()
    return sorted(set(re.findall(r"^(?:int|const char\*)\s+(mppi_jump_\w+)\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    names = _declared_functions()
    assert len(names) >= 18
    lib = native.lib()
    for n in names:
        assert hasattr(lib, n), n
    # every binding prototype is declared in the header
    assert set(native._PROTOS) <= set(names)
    out = subprocess.run(["nm", "-D", "--defined-only", native.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (mppi_jump_\w+)$", out, re.M))
    assert set(names) <= exported


def test_struct_layout_matches_c(tmp_path):
    fields = [f for f, _ in native.Config._fields_]
    cfields = [("lambda" if f == "lambda_" else f) for f in fields]
    src = ["#include <stdio.h>", "#include <stddef.h>", '#include "mppi_jump.h"', "int main(void){",
           'printf("%zu %zu\\n", sizeof(mppi_jump_config), sizeof(mppi_jump_stats));']
    src += ['printf("%%zu\\n", offsetof(mppi_jump_config, %s));' % f for f in cfields]
    src += ['printf("%%zu\\n", offsetof(mppi_jump_stats, %s));' % f for f, _ in native.Stats._fields_]
    src += ["return 0;}"]
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(c)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                           check=True).stdout.split()]
    import ctypes
    assert vals[0] == ctypes.sizeof(native.Config) and vals[1] == ctypes.sizeof(native.Stats)
    offs = [getattr(native.Config, f).offset for f in fields]
    offs += [getattr(native.Stats, f).offset for f, _ in native.Stats._fields_]
    assert vals[2:] == offs


def test_version_dims_strerror():
    assert native.lib().mppi_jump_abi_version() == native.C["MPPI_JUMP_ABI_VERSION"]
    assert native.dims(0) == (2, 1, 1)
    assert native.dims(1) == (4, 1, 1)
    assert native.dims(2) == (12, 4, 3)
    with pytest.raises(native.MppiError) as e:
        native.dims(7)
    assert e.value.code == native.C["MPPI_EINVAL"] and "unknown dynamics" in str(e.value)
    for code in (0, -1, -2, -3, -4, -5, 99):
        assert native.strerror(code)


def test_workspace_bytes_scales_with_the_problem():
    small = native.workspace_bytes(workloads.cartpole())
    big = native.workspace_bytes(workloads.cartpole_mpc())
    quad = native.workspace_bytes(workloads.quadrotor())
    assert small > 256 * 50 * 4
    assert big >= 4096 * 100 * 4 + 4096 * 16
    assert quad >= 8192 * 100 * 4 * 4
    # the debug dumps (compared on the lane schedule, whose partials are laid
    # out alike with and without them)
    lane = native.workspace_bytes(dict(workloads.cartpole(), schedule=1))
    dbg = native.workspace_bytes(dict(workloads.cartpole(), schedule=1, debug_dump=1))
    assert dbg >= lane + 256 * 50 * 12


def test_auto_schedule_limits():
    # AUTO takes the wave-specialised schedule up to MPPI_JUMP_WS_MAX_K
    # samples, MPPI_JUMP_WS_MAX_K_MULTI for the multi-channel quadrotor; the
    # two schedules' workspaces differ (per-workgroup partials of 64 or 256
    # samples), which shows the choice
    LANE, WS = native.C["MPPI_SCHED_LANE"], native.C["MPPI_SCHED_WAVE_SPECIALISED"]
    for mk, limit in ((workloads.cartpole, native.C["MPPI_JUMP_WS_MAX_K"]),
                      (workloads.quadrotor, native.C["MPPI_JUMP_WS_MAX_K_MULTI"])):
        for K, sched in ((limit, WS), (limit + 1, LANE)):
            auto = native.workspace_bytes(mk(K=K, T=20))
            assert auto == native.workspace_bytes(mk(K=K, T=20, schedule=sched)), (K, sched)
            other = LANE if sched == WS else WS
            assert auto != native.workspace_bytes(mk(K=K, T=20, schedule=other)), (K, sched)
    assert native.C["MPPI_JUMP_WS_MAX_K_MULTI"] < native.C["MPPI_JUMP_WS_MAX_K"]


BAD = [
    ("dynamics", 3), ("K", 0), ("K", 2**24 + 1), ("T", 0), ("T", 4097), ("dt", 0.0),
    ("dt", float("nan")), ("lambda", 0.0), ("lambda", -1.0), ("c", 0.0), ("nu", -0.1),
    ("nu", float("inf")), ("alpha", float("nan")), ("count_law", 2), ("cost_form", 5),
    ("debug_dump", 3), ("schedule", 3), ("sigma", [-1.0, 0, 0, 0]),
    ("sigma_J", [float("nan"), 0, 0, 0]), ("controller_id", 2**24),
    ("start_iteration", 2**32), ("params", [0.0] * 12),
]


@pytest.mark.parametrize("field,value", BAD)
def test_invalid_config_is_rejected(field, value):
    cfg = workloads.cartpole()
    cfg[field] = value
    with pytest.raises(native.MppiError) as e:
        native.workspace_bytes(cfg)
    assert e.value.code == native.C["MPPI_EINVAL"]


def test_abi_version_mismatch_and_jump_table_overflow():
    c = native.make_config(workloads.cartpole())
    c.abi_version = 99
    import ctypes
    b = ctypes.c_size_t()
    assert native.lib().mppi_jump_workspace_bytes(ctypes.byref(c), ctypes.byref(b)) == native.C["MPPI_EINVAL"]
    with pytest.raises(native.MppiError):
        native.workspace_bytes(workloads.cartpole(nu=2000.0))        # nu dt = 40
    with pytest.raises(native.MppiError):
        native.workspace_bytes(workloads.cartpole(nu=60.0, count_law=1))  # zero-one needs nu dt <= 1
    q = workloads.quadrotor()
    q["params"] = list(q["params"])
    q["params"][7] = 1.6
    with pytest.raises(native.MppiError):
        native.workspace_bytes(q)
    # the jump marks are normal (the only law the configuration names)
    with pytest.raises(native.MppiError) as e:
        native.workspace_bytes(workloads.cartpole(mark_law=1))
    assert e.value.code == native.C["MPPI_EINVAL"] and "mark_law" in str(e.value)
    assert native.C["MPPI_MARK_NORMAL"] == 0


@pytest.mark.parametrize("nu,law,dt", [(0.0, 0, 0.02), (2.0, 0, 0.02), (5.0, 0, 0.02),
                                       (3.0, 0, 0.01), (10.0, 0, 0.02), (10.0, 1, 0.02),
                                       (50.0, 0, 0.05), (0.5, 1, 0.1), (49.0, 1, 0.02)])
def test_count_tables_equal_the_oracle(nu, law, dt):
    cfg = workloads.cartpole(nu=nu, count_law=law, dt=dt)
    lib_th = native.count_thresholds(cfg)
    a = float(np.float32(nu)) * float(np.float32(dt))
    ref = noise.count_thresholds(a, law)
    assert lib_th[:len(ref)] == ref
    assert all(v == 2**32 for v in lib_th[len(ref):])


def test_pool_and_batch_entry_points_reject_null_arguments():
    import ctypes
    L = native.lib()
    EINVAL = native.C["MPPI_EINVAL"]
    d, h = ctypes.c_size_t(), ctypes.c_size_t()
    assert L.mppi_jump_pool_bytes(None, 0, 1, ctypes.byref(d), ctypes.byref(h)) == EINVAL
    assert L.mppi_jump_pool_bytes(None, 1, 0, ctypes.byref(d), ctypes.byref(h)) == EINVAL
    assert L.mppi_jump_pool_tick(None, None, None, None, 1, 1, 0, None) == EINVAL
    f = ctypes.c_int32()
    assert L.mppi_jump_pool_query(None, 0, ctypes.byref(f)) == EINVAL
    assert L.mppi_jump_pool_results(None, 0, None, None, None, ctypes.byref(f)) == EINVAL
    assert L.mppi_jump_batch_scratch_bytes(None, 1, ctypes.byref(d)) == EINVAL


def test_serving_workload_recipe():
    cs = workloads.serving_controllers(1024)
    kinds = [c["dynamics"] for c, _ in cs]
    assert kinds.count(1) == kinds.count(2) == 512
    assert {c["K"] for c, _ in cs} == {1024, 2048, 4096, 8192}
    assert min(c["T"] for c, _ in cs) >= 50 and max(c["T"] for c, _ in cs) <= 150
    assert len({c["controller_id"] for c, _ in cs}) == 1024
    t, ids = workloads.serving_arrivals(20000.0, 2.0, 1024, seed=9)
    gaps = np.diff(t)
    assert abs(gaps.mean() - 5e-5) < 2e-6 and abs(gaps.std() / gaps.mean() - 1.0) < 0.03
    assert t.max() < 2.0 and ids.min() >= 0 and ids.max() < 1024
    d = workloads.serving_disturbances(workloads.quadrotor(), 20000, seed=1)
    assert d.shape == (20000, 8) and abs(d[:, :4].std() - 0.5) < 0.01 and not d[:, 7].any()
    # the gust: per axis variance nu dt sigma_J^2 = 0.03 * 9
    assert np.allclose(d[:, 4:7].var(axis=0) / 0.27, 1.0, atol=0.1)
    d = workloads.serving_disturbances(workloads.cartpole_mpc(), 20000, seed=1)
    assert d.shape == (20000, 8) and not d[:, 1:].any()
    # variance 1 + nu dt sigma_J^2 = 1 + 0.1 * 100
    assert abs(d[:, 0].var() / 11.0 - 1.0) < 0.1


def test_admission_by_footprint():
    from paper_1807_06108_amd import serving
    cfgs = [c for c, _ in workloads.serving_controllers(64)]
    need = [serving.footprint_bytes(c) for c in cfgs]
    assert need == [native.workspace_bytes(c) for c in cfgs]
    ok, rest, used = serving.admit(cfgs, sum(need))
    assert ok == list(range(64)) and not rest and used == sum(need)
    cap = sum(need[:10]) + 1
    ok, rest, used = serving.admit(cfgs, cap)
    assert ok[:10] == list(range(10)) and used <= cap
    assert sorted(ok + rest) == list(range(64))


def test_study_success_criterion():
    from paper_1807_06108_amd import study
    t = np.zeros((3, 10))
    t[1, -1] = 0.3           # leaves the 0.25 rad band at the last step
    t[2, :5] = 3.0           # down early, upright over the last 5 steps
    t[0] = 2 * np.pi         # a full turn is upright again
    assert list(study.swing_up_success(t, 5, 0.25)) == [True, False, True]
    assert list(study.swing_up_success(t, 6, 0.25)) == [True, False, False]


def test_study_quadrotor_disturbances_and_success():
    from paper_1807_06108_amd import study
    d = study.quadrotor_disturbances(20000, 0.01, 0.5, 2.0, 100.0, seed=3)
    assert d.shape == (20000, 8) and not d[:, 7].any()
    assert abs(d[:, :4].std() - 0.5) < 0.02
    # gust variance nu dt sigma_J^2 per axis
    assert abs(d[:, 4:7].var() / (0.02 * 100.0 ** 2) - 1.0) < 0.15
    params = workloads.QUAD_PARAMS
    goal = [1.0, -1.0, 2.0]
    t = np.zeros((3, 4, 12), dtype=np.float32)
    t[:, :, 2] = 1.0
    t[:, -1, :3] = goal
    t[1, 2, 2] = -0.1            # below the ground once
    t[2, -1, 0] = 1.6            # 0.6 m short of the target at the end
    assert list(study.quadrotor_success(t, goal, params)) == [True, False, False]


def test_full_covariance_validation():
    good = workloads.quadrotor(full_sigma=1, sigma_L=workloads.random_cholesky(4, 0.5, seed=1))
    assert native.workspace_bytes(good) > 0
    upper = list(good["sigma_L"])
    upper[1] = 0.1                     # above the diagonal
    zero_diag = list(good["sigma_L"])
    zero_diag[5] = 0.0
    for bad in (dict(good, sigma_L=upper), dict(good, sigma_L=zero_diag),
                dict(good, full_sigma=2)):
        with pytest.raises(native.MppiError) as e:
            native.workspace_bytes(bad)
        assert e.value.code == native.C["MPPI_EINVAL"]
    # a one-channel model: only L00 is read
    cp = workloads.cartpole(full_sigma=1, sigma_L=[1.5] + [0.0] * 15, sigma=[0.0] * 4)
    assert native.workspace_bytes(cp) > 0


def test_sample_offset_validation():
    assert native.workspace_bytes(workloads.cartpole(K=1000, sample_offset=5000)) > 0
    for bad in (workloads.cartpole(K=1000, sample_offset=2**31 - 10),
                workloads.cartpole(sample_offset=-1)):
        with pytest.raises(native.MppiError) as e:
            native.workspace_bytes(bad)
        assert e.value.code == native.C["MPPI_EINVAL"]
