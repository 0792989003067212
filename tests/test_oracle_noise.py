"""Pins of the oracle's noise transform (CPU only): Box-Muller closed forms and
distribution, count thresholds against scipy and exact arithmetic, count and
perturbation moments (Sec. II mark law, Sec. IV-B jump law), the zero-one
mixture density of eq. (42), and the word-stream layout."""

import math
from decimal import Decimal, getcontext

import numpy as np
import pytest
from scipy import stats

from oracle import noise
from paper_1807_06108_amd import workloads


def test_box_muller_closed_forms():
    u1 = np.array([0xFFFFFFFF], dtype=np.uint32)          # u = 1 -> radius 0
    half = np.array([(2**23 - 1) << 8], dtype=np.uint32)  # u = 1/2
    z0, z1 = noise.box_muller(u1, np.array([12345 << 8], dtype=np.uint32))
    assert z0[0] == 0.0 and z1[0] == 0.0
    r = math.sqrt(2.0 * math.log(2.0))
    for ang, (c, s) in {0: (1, 0), 1 << 30: (0, 1), 2 << 30: (-1, 0),
                        3 << 30: (0, -1)}.items():
        z0, z1 = noise.box_muller(half, np.array([ang], dtype=np.uint32))
        assert abs(z0[0] - r * c) < 1e-15 and abs(z1[0] - r * s) < 1e-15
    # low 8 bits are ignored
    a = noise.box_muller(half | np.uint32(0xFF), np.array([77 << 8 | 0x5A], dtype=np.uint32))
    b = noise.box_muller(half, np.array([77 << 8], dtype=np.uint32))
    assert a == b


def test_box_muller_is_standard_normal():
    cfg = workloads.cartpole(K=2048, T=100)
    z_D, N, z_J = noise.sample(cfg, 0)
    for z in (z_D.ravel(), z_J.ravel()):
        assert stats.kstest(z, "norm").pvalue > 1e-3
        assert abs(z.mean()) < 5 / math.sqrt(z.size)
        assert abs(z.var() - 1) < 6 * math.sqrt(2 / z.size)
    # the two outputs of a pair are uncorrelated
    assert abs(np.corrcoef(z_D.ravel(), z_J.ravel())[0, 1]) < 5 / math.sqrt(z_D.size)
    # 24-bit radius: |z| never exceeds sqrt(-2 ln 2^-24)
    assert np.abs(z_D).max() <= math.sqrt(-2 * math.log(2.0**-24)) + 1e-12


@pytest.mark.parametrize("a", [0.0, 0.02, 0.04, 0.1, 0.2, 1.0, 3.0])
def test_poisson_thresholds_match_scipy(a):
    th = noise.count_thresholds(a, 0)
    assert th[-1] == 2**32 and all(x <= y for x, y in zip(th, th[1:]))
    cdf = stats.poisson.cdf(np.arange(len(th)), a)
    for j, t in enumerate(th[:-1]):
        assert abs(t - math.floor(cdf[j] * 2**32)) <= 1
    # closing level: the remaining tail mass is below 2^-32
    assert stats.poisson.sf(len(th) - 1, a) * 2**32 < 2.0


@pytest.mark.parametrize("a", [0.04, 0.1, 0.25, 2.0])
def test_poisson_thresholds_exact_arithmetic(a):
    getcontext().prec = 60
    A = Decimal(a)           # the exact binary value of the double
    F = Decimal(0)
    term = (-A).exp()
    th = noise.count_thresholds(a, 0)
    for j, t in enumerate(th[:-1]):
        if j > 0:
            term = term * A / j
        F += term
        exact = F * 2**32
        if abs(exact - exact.to_integral_value()) > Decimal("1e-5"):
            assert t == int(exact)


def test_zero_one_thresholds():
    assert noise.count_thresholds(0.0, 1) == [2**32]
    assert noise.count_thresholds(1.0, 1) == [0, 2**32]
    th = noise.count_thresholds(0.25, 1)
    assert th == [3 * 2**30, 2**32]
    with pytest.raises(ValueError):
        noise.count_thresholds(1.5, 1)
    with pytest.raises(ValueError):
        noise.count_thresholds(40.0, 0)


def test_counts_by_inversion():
    th = [10, 20, 2**32]
    w = np.array([0, 9, 10, 19, 20, 2**32 - 1], dtype=np.uint32)
    assert list(noise.counts(w, th)) == [0, 0, 1, 1, 2, 2]


@pytest.mark.parametrize("law", [0, 1])
def test_count_moments(law):
    cfg = workloads.cartpole(K=4096, T=100, nu=5.0, count_law=law)
    _, N, _ = noise.sample(cfg, 3)
    a = float(np.float32(5.0)) * float(np.float32(0.02))
    n = N.size
    var = a if law == 0 else a * (1 - a)
    assert abs(N.mean() - a) < 5 * math.sqrt(var / n)
    p0 = math.exp(-a) if law == 0 else 1 - a
    assert abs((N == 0).mean() - p0) < 5 * math.sqrt(p0 * (1 - p0) / n)
    assert abs(N.var() - var) < 6 * math.sqrt((var + 3 * var * var) / n) + 1e-3
    if law == 1:
        assert N.max() <= 1


def test_perturbation_variance():
    # Var eps = sigma^2 + nu dt sigma_J^2 for a control-channel jump
    cfg = workloads.cartpole(K=4096, T=100, nu=5.0, sigma_J=[10.0, 0, 0, 0])
    eps, gust = noise.compose(cfg, *noise.sample(cfg, 0))
    e = eps.ravel()
    a = float(np.float32(5.0)) * float(np.float32(0.02))
    target = 1.0 + a * 100.0
    se = math.sqrt(((e**4).mean() - e.var()**2) / e.size)
    assert abs(e.var() - target) < 5 * se
    assert abs(e.mean()) < 5 * math.sqrt(target / e.size)
    assert not gust.any()


def test_zero_one_mixture_density_eq42():
    # Under the zero-one law the perturbation is the two-component normal
    # mixture of eq. (42): N(0, sD^2) w.p. 1 - a, N(0, sD^2 + sJ^2) w.p. a.
    cfg = workloads.cartpole(K=4096, T=100, nu=10.0, count_law=1,
                             sigma_J=[3.0, 0, 0, 0])
    eps, _ = noise.compose(cfg, *noise.sample(cfg, 1))
    a = float(np.float32(10.0)) * float(np.float32(0.02))
    s_big = math.sqrt(1.0 + 9.0)

    def cdf(x):
        return (1 - a) * stats.norm.cdf(x) + a * stats.norm.cdf(x / s_big)
    assert stats.kstest(eps.ravel(), cdf).pvalue > 1e-3
    # and it is not the single normal of the same variance
    assert stats.kstest(eps.ravel(), "norm", args=(0, math.sqrt(1 + a * 9))).pvalue < 1e-6


def test_quadrotor_layout_and_gust():
    assert noise.layout(2) == (12, 4, 3, None, 2)
    assert noise.layout(1) == (4, 1, 1, 2, 1)
    cfg = workloads.quadrotor(K=512, T=40)
    z_D, N, z_J = noise.sample(cfg, 0)
    assert z_D.shape == (512, 40, 4) and z_J.shape == (512, 40, 3) and N.shape == (512, 40)
    eps, gust = noise.compose(cfg, z_D, N, z_J)
    assert np.array_equal(eps, z_D * np.float32(0.5))
    assert np.array_equal(gust == 0, np.broadcast_to((N == 0)[..., None], gust.shape) | (z_J == 0))


def test_stream_properties():
    cfg = workloads.cartpole(K=128, T=20)
    zD, N, zJ = noise.sample(cfg, 4)
    # changing the jump rate leaves the Gaussian draws bitwise unchanged
    zD2, N2, _ = noise.sample(dict(cfg, nu=0.0), 4)
    assert np.array_equal(zD, zD2) and not N2.any()
    # a subset of samples reproduces the same rows
    idx = np.array([0, 5, 127, 64])
    zs, Ns, zJs = noise.sample(cfg, 4, idx)
    assert np.array_equal(zs, zD[idx]) and np.array_equal(Ns, N[idx])
    # iteration, controller id and seed all select a different stream
    for over in (dict(controller_id=1), dict(seed=cfg["seed"] + 1)):
        assert not np.array_equal(noise.sample(dict(cfg, **over), 4)[0], zD)
    assert not np.array_equal(noise.sample(cfg, 5)[0], zD)


def test_low_byte_count_word_is_poisson_and_independent():
    # quadrotor: the count word comes from the low bytes of words 0-3, the
    # same words whose top 24 bits give z_D.  The counts must still follow
    # the count law (chi-square against scipy's Poisson pmf) and carry no
    # dependence on the Gaussian draws of their step.
    cfg = workloads.quadrotor(K=4096, T=50, nu=40.0)
    z_D, N, _ = noise.sample(cfg, 2)
    a = float(np.float32(40.0)) * float(np.float32(cfg["dt"]))
    n = N.ravel()
    top = 5
    obs = np.array([np.sum(n == j) for j in range(top)] + [np.sum(n >= top)], dtype=np.float64)
    pmf = stats.poisson.pmf(np.arange(top), a)
    exp = n.size * np.append(pmf, 1.0 - pmf.sum())
    assert stats.chisquare(obs, exp).pvalue > 1e-4
    # mean and variance a; no correlation with z_D or z_D^2
    assert abs(n.mean() - a) < 5 * math.sqrt(a / n.size)
    for j in range(4):
        for f in (z_D[..., j], z_D[..., j] ** 2):
            r = np.corrcoef(n, f.ravel())[0, 1]
            assert abs(r) < 5 / math.sqrt(n.size)
    # the assembled word is uniform over 32 bits: its byte lanes are
    # the low bytes of four different words
    w = noise.words(cfg["seed"], cfg["controller_id"], 2, np.arange(256), 50, 2)
    wc = noise.low_byte_word(w)
    for sh in (0, 8, 16, 24):
        b = ((wc >> sh) & 255).ravel()
        assert np.array_equal(b, (w[..., sh // 8] & 255).ravel())
        hist = np.bincount(b, minlength=256).astype(np.float64)
        assert stats.chisquare(hist).pvalue > 1e-4
