"""Philox-4xW-R counter-based block function, written from its published definition.

Source: J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11, Sec. 3.3 (the Philox S-box: one
multiply-hi/lo per pair of words, XOR of the high half into the other word of
the pair together with a round key, followed by a fixed word permutation) and
Sec. 4 (key schedule: the key is bumped by the Weyl constants -- the
fractional parts of the golden ratio and of sqrt(3), scaled to W bits -- before
every round after the first).

One generic round structure is used for both word widths:
  W = 64 instance - pinned against numpy.random.Philox (a library
                    implementation of Philox4x64-10) in the CPU tests, which
                    fixes the structure: which words are multiplied, where the
                    high halves and the keys are XORed, the permutation and the
                    key schedule;
  W = 32 instance - the one the method uses (four 32-bit words per block);
                    it differs from the W = 64 instance only in the constants
                    and in the width of the multiply.

Parity: pinned (structure by the numpy library routine; Weyl constants by
their closed form; the 32-bit multiply by Python integers).  The two 32-bit
multipliers have no independent source here beyond the SC'11 paper.
"""

import numpy as np

# Multipliers (SC'11, Table 2 of the Philox parameters) and Weyl key increments.
M4x32 = (0xD2511F53, 0xCD9E8D57)
W4x32 = (0x9E3779B9, 0xBB67AE85)
M4x64 = (0xD2E7470EE14C6C93, 0xCA5A826395121157)
W4x64 = (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)


def _round_structure(x, key, rounds, mulhilo, M, Wk, add_key):
    """R Philox rounds over four words x[0..3] with key (k0, k1).

    Each round: (hi0, lo0) = M0 * x0, (hi1, lo1) = M1 * x2, then the new block
    is (hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0).  The key is bumped by the Weyl
    increments before every round but the first.
    """
    x0, x1, x2, x3 = x
    k0, k1 = key
    for r in range(rounds):
        if r > 0:
            k0 = add_key(k0, Wk[0])
            k1 = add_key(k1, Wk[1])
        hi0, lo0 = mulhilo(M[0], x0)
        hi1, lo1 = mulhilo(M[1], x2)
        x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
    return x0, x1, x2, x3


def _mulhilo32(a, b):
    # a: python int constant, b: uint64 array holding 32-bit values.
    p = np.uint64(a) * b  # < 2^64, exact in uint64
    return p >> np.uint64(32), p & np.uint64(0xFFFFFFFF)


def _add32(k, w):
    return (k + w) & 0xFFFFFFFF


def philox4x32(counter, key, rounds=10):
    """Philox4x32-R.  counter: integer array [..., 4] (values < 2^32);
    key: (k0, k1) python ints < 2^32.  Returns uint32 array [..., 4]."""
    c = np.asarray(counter, dtype=np.uint64)
    words = [c[..., i] for i in range(4)]
    out = _round_structure(words, (int(key[0]), int(key[1])), rounds,
                           _mulhilo32, M4x32, W4x32, _add32)
    # key words are python ints; XOR with uint64 arrays keeps uint64
    return np.stack([np.asarray(o, dtype=np.uint64) & np.uint64(0xFFFFFFFF)
                     for o in out], axis=-1).astype(np.uint32)


_MASK64 = (1 << 64) - 1


def _mulhilo64(a, b):
    p = a * b  # python big int
    return p >> 64, p & _MASK64


def _add64(k, w):
    return (k + w) & _MASK64


def philox4x64(counter, key, rounds=10):
    """Philox4x64-R on python ints (slow; used to pin the shared round
    structure against numpy.random.Philox)."""
    return _round_structure(tuple(int(v) for v in counter),
                            (int(key[0]), int(key[1])), rounds,
                            _mulhilo64, M4x64, W4x64, _add64)
