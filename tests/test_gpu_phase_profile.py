"""The phase-profiling build (timestamps compiled into the same kernels) and
its reader: one short run per mode, in a process of its own (the library is
loaded once per process).  The timeline must be ordered and account for the
launch."""

import os
import re
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    r = subprocess.run([sys.executable, "-m", "paper_1807_06108_amd.phase_profile", *args],
                       cwd=ROOT, capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    return r.stdout


def _last_row(text):
    rows = [ln for ln in text.splitlines() if re.match(r"^\| [0-9]", ln)]
    return [float(x) for x in rows[-1].strip("|").split("|")]


def test_launch_phases_are_ordered_and_account_for_the_launch():
    out = _run("--workload", "cartpole_single", "--reps", "5", "--warmup", "5")
    print(out)
    launches = [ln for ln in out.splitlines() if re.match(r"^\| [0-2] \|", ln)]
    assert len(launches) == 3
    for ln in launches:
        cells = [c.strip() for c in ln.strip("|").split("|")]
        start_hi = float(cells[1].split("..")[1])
        t = [float(c) for c in cells[2:]]  # first chunk .. end
        assert start_hi <= t[0] <= t[1] <= t[2] <= t[3] <= t[4] <= t[5] <= t[6]
    phases = _last_row(out)  # to first chunk .. per launch
    assert all(x >= 0 for x in phases)
    assert abs(sum(phases[:8]) - phases[8]) < 0.25 * phases[8]


def test_batched_tile_timeline():
    out = _run("--batched", "32", "--reps", "3")
    print(out)
    span, peak, mean, ideal, tail, cart, quad = _last_row(out)
    assert 0 < mean <= peak and ideal <= span and 0 <= tail <= span
    assert cart > 0 and quad > cart
