"""Closed-loop study harness: paired trials, deterministic outcomes, and the
special case where both algorithms coincide (no plant jumps to sample)."""

import numpy as np
import pytest

from paper_1807_06108_amd import study

pytestmark = pytest.mark.gpu


def test_study_is_deterministic_and_paired():
    print("study: 6 trials x 80 steps", flush=True)
    a = study.run_condition(2.5, 10.0, trials=6, steps=80, hold_steps=20)
    b = study.run_condition(2.5, 10.0, trials=6, steps=80, hold_steps=20)
    assert np.array_equal(a["new_ok"], b["new_ok"]) and np.array_equal(a["old_ok"], b["old_ok"])
    assert 0.0 <= a["new"] <= 1.0 and 0.0 <= a["old"] <= 1.0


def test_without_plant_jumps_both_algorithms_are_the_same_controller():
    # nu = 0: the "new" controller samples no jumps either, so both columns
    # run identical controllers on identical disturbances
    r = study.run_condition(0.0, 10.0, trials=6, steps=80, hold_steps=20)
    assert np.array_equal(r["new_ok"], r["old_ok"])
