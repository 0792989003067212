"""Pins of the oracle's Philox block function (CPU only).

The round structure is shared by the 64-bit and 32-bit instances; the 64-bit
instance is checked against numpy.random.Philox (a library Philox4x64-10),
which fixes the structure.  The Weyl constants are checked against their
closed form, the 32-bit multiply against python integers."""

from decimal import Decimal, getcontext

import numpy as np
import pytest

from oracle import philox


def test_structure_matches_numpy_philox4x64():
    rng = np.random.default_rng(123)
    for _ in range(40):
        ctr = [int(v) for v in rng.integers(1, 2**63, size=4, dtype=np.uint64)]
        key = [int(v) for v in rng.integers(0, 2**63, size=2, dtype=np.uint64)]
        # numpy increments the counter before producing a block
        bg = np.random.Philox(counter=[ctr[0] - 1] + ctr[1:], key=key)
        got = [int(v) for v in bg.random_raw(4)]
        assert got == list(philox.philox4x64(ctr, key))


@pytest.mark.parametrize("rounds", [1, 7, 10])
def test_structure_rounds_numpy(rounds):
    # numpy only exposes 10 rounds; other round counts must at least differ
    ctr, key = [5, 6, 7, 8], [11, 12]
    out = philox.philox4x64(ctr, key, rounds)
    ref = [int(v) for v in np.random.Philox(counter=[4, 6, 7, 8], key=key).random_raw(4)]
    assert (list(out) == ref) == (rounds == 10)


def test_weyl_constants_closed_form():
    getcontext().prec = 80
    frac_phi = (Decimal(5).sqrt() - 1) / 2
    frac_s3 = Decimal(3).sqrt() - 1
    for W, consts in ((32, philox.W4x32), (64, philox.W4x64)):
        assert consts[0] == int(frac_phi * 2**W)
        assert consts[1] == int(frac_s3 * 2**W)


def test_mulhilo32_against_python_ints():
    rng = np.random.default_rng(5)
    b = rng.integers(0, 2**32, size=1000, dtype=np.uint64)
    for M in philox.M4x32:
        hi, lo = philox._mulhilo32(M, b)
        for bi, h, l in zip(b[:200], hi[:200], lo[:200]):
            p = M * int(bi)
            assert int(h) == p >> 32 and int(l) == p & 0xFFFFFFFF


def _philox4x32_pyint(ctr, key, rounds=10):
    return philox._round_structure(
        tuple(ctr), tuple(key), rounds,
        lambda a, b: ((a * b) >> 32, (a * b) & 0xFFFFFFFF),
        philox.M4x32, philox.W4x32, lambda k, w: (k + w) & 0xFFFFFFFF)


def test_vectorised_4x32_equals_scalar():
    rng = np.random.default_rng(9)
    ctr = rng.integers(0, 2**32, size=(64, 4), dtype=np.uint64)
    key = (0x89ABCDEF, 0x01234567)
    vec = philox.philox4x32(ctr, key)
    assert vec.dtype == np.uint32
    for i in range(64):
        assert tuple(int(v) for v in vec[i]) == _philox4x32_pyint(
            [int(v) for v in ctr[i]], key)


def test_4x32_avalanche_and_balance():
    # flipping one counter bit flips about half of the 128 output bits
    rng = np.random.default_rng(11)
    ctr = rng.integers(0, 2**32, size=(2000, 4), dtype=np.uint64)
    key = (1, 2)
    base = philox.philox4x32(ctr, key)
    flips = []
    for word in range(4):
        c2 = ctr.copy()
        c2[:, word] ^= np.uint64(1 << (word * 7 % 32))
        diff = base ^ philox.philox4x32(c2, key)
        flips.append(np.unpackbits(diff.view(np.uint8)).reshape(2000, -1).sum(1).mean())
    assert all(abs(f - 64.0) < 1.0 for f in flips)
    bits = np.unpackbits(base.view(np.uint8)).mean()
    assert abs(bits - 0.5) < 0.005


def test_philox4x32_against_rocrand_host_build(tmp_path):
    """Known-answer check of the 32-bit instance itself (multipliers, Weyl
    constants, round order) against rocRAND's Philox4x32-10 engine, an
    independent implementation whose header ships with ROCm, compiled for the
    host: random counters and keys plus the all-zero and all-ones inputs."""
    import os
    import shutil
    import subprocess
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    header = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"
    if not (os.path.exists(hipcc) and os.path.exists(header)):
        pytest.skip("hipcc or the rocRAND header is not installed")
    src = os.path.join(os.path.dirname(__file__), "rocrand_philox_kat.cpp")
    exe = str(tmp_path / "kat")
    subprocess.run([hipcc, "-x", "hip", "--cuda-host-only", "-O1", "-o", exe, src], check=True,
                   capture_output=True)
    rng = np.random.default_rng(2024)
    rows = rng.integers(0, 2**32, size=(2000, 6), dtype=np.uint64)
    rows[0] = 0
    rows[1] = 2**32 - 1
    text = "\n".join(" ".join("%x" % v for v in r) for r in rows) + "\n"
    out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(w, 16) for w in ln.split()] for ln in out.splitlines()], dtype=np.uint64)
    got = np.stack([philox.philox4x32(r[:4], (int(r[4]), int(r[5]))) for r in rows])
    assert ref.shape == (2000, 4)
    assert np.array_equal(np.asarray(got, dtype=np.uint64), ref)
