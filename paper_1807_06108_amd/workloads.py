"""Seeded synthetic workloads: configurations, initial states, initial control
sequences and plant disturbance sequences.

This module holds none of the method's arithmetic; it only produces inputs,
and it is the one module that the tests, the benchmark and the CPU reference
share.  The shapes and parameters follow the paper's two systems (Sec. VI:
cartpole swing-up with 1000 samples, quadrotor fly-to-target with 3000-6000
samples) at the sizes this library is measured on:

  cartpole_single   K=256,  T=50,  dt=0.02, sigma=1, nu=2 /s, sigma_J=5
  cartpole_mpc      K=4096, T=100, dt=0.02, 5 iterations per control step,
                    500 control steps; controller and plant nu=5 /s,
                    sigma_J=10, sigma=1
  quadrotor_hover   K=8192, T=100, dt=0.01, sigma=0.5 N, gust nu=3 /s,
                    N(0, 3^2) per axis, crash penalty 1e4, lambda=0.5
  double_integrator small closed-form test system

The paper publishes no dataset, so there is nothing these stand in for
beyond its described tasks.
"""

import math

import numpy as np

DYN_ID = {"linear": 0, "cartpole": 1, "quadrotor": 2}
DIMS = {0: (2, 1, 1), 1: (4, 1, 1), 2: (12, 4, 3)}

DEFAULT_SEED = 0x1807061080000001

CARTPOLE_PARAMS = [1.0, 0.1, 0.5, 9.81]                       # m_cart, m_pole, half length, g
QUAD_PARAMS = [1.0, 0.01, 0.01, 0.02, 0.2, 0.02, 9.81, 1.2, 0.0]  # mass, Jx, Jy, Jz, arm, k_yaw, g, tilt, z_min
QUAD_HOVER = QUAD_PARAMS[0] * QUAD_PARAMS[6] / 4.0


def _pad(v, n):
    v = list(v)
    return v + [0.0] * (n - len(v))


def base_config(dynamics):
    """All fields of the C configuration structure, zero/neutral filled."""
    return dict(dynamics=dynamics, K=256, T=50, dt=0.02, **{"lambda": 1.0},
                alpha=1.0, c=1.0, nu=0.0, count_law=0, cost_form=0,
                debug_dump=0, sigma=[0.0] * 4, sigma_J=[0.0] * 4,
                u_init=[0.0] * 4, R=[0.0] * 4, Q=[0.0] * 12, Qf=[0.0] * 12,
                x_goal=[0.0] * 12, params=[0.0] * 12, crash_penalty=0.0, schedule=0,
                seed=DEFAULT_SEED, controller_id=0, start_iteration=0,
                full_sigma=0, sigma_L=[0.0] * 16, sample_offset=0, mark_law=0)


def random_cholesky(m, scale, seed):
    """A seeded lower-triangular factor L (positive diagonal) of a full
    Gaussian covariance L L^T of the m control channels, as the 16 row-major
    entries of a 4 x 4 block."""
    g = np.random.default_rng(seed)
    L = np.tril(g.uniform(-0.5, 0.5, size=(m, m))) * scale
    L[np.diag_indices(m)] = scale * g.uniform(0.6, 1.4, size=m)
    out = np.zeros((4, 4))
    out[:m, :m] = L
    return [float(v) for v in out.reshape(-1)]


def cartpole(**over):
    cfg = base_config(1)
    Q = [1.0, 0.1, 10.0, 0.1]
    cfg.update(K=256, T=50, dt=0.02, sigma=_pad([1.0], 4), nu=2.0,
               sigma_J=_pad([5.0], 4), Q=_pad(Q, 12),
               Qf=_pad([10 * q for q in Q], 12), R=_pad([0.01], 4),
               params=_pad(CARTPOLE_PARAMS, 12))
    cfg["lambda"] = 1.0
    cfg.update(over)
    return cfg


def cartpole_mpc(**over):
    cfg = cartpole(K=4096, T=100, nu=5.0, sigma_J=_pad([10.0], 4))
    cfg.update(over)
    return cfg


def quadrotor(**over):
    cfg = base_config(2)
    Q = [1.0] * 3 + [0.1] * 3 + [1.0] * 3 + [0.1] * 3
    goal = [1.0, -1.0, 2.0] + [0.0] * 9
    cfg.update(K=8192, T=100, dt=0.01, sigma=[0.5] * 4, nu=3.0,
               sigma_J=_pad([3.0] * 3, 4), Q=Q, Qf=[10 * q for q in Q],
               R=[0.01] * 4, x_goal=goal, params=_pad(QUAD_PARAMS, 12),
               crash_penalty=1e4, u_init=[QUAD_HOVER] * 4)
    cfg["lambda"] = 0.5
    cfg.update(over)
    return cfg


def double_integrator(**over):
    cfg = base_config(0)
    cfg.update(K=64, T=20, dt=0.1, sigma=_pad([1.0], 4), nu=1.0,
               sigma_J=_pad([2.0], 4), Q=_pad([1.0, 0.1], 12),
               Qf=_pad([10.0, 1.0], 12), R=_pad([0.1], 4))
    cfg["lambda"] = 1.0
    cfg.update(over)
    return cfg


PRESETS = {"cartpole_single": cartpole, "cartpole_mpc": cartpole_mpc,
           "quadrotor_hover": quadrotor, "double_integrator": double_integrator}


def x0_for(cfg):
    """Initial state of the preset tasks."""
    d = cfg["dynamics"]
    if d == 1:
        return np.array([0.0, 0.0, math.pi - 0.2, 0.0], dtype=np.float32)
    if d == 2:
        x = np.zeros(12, dtype=np.float32)
        x[2] = 1.0
        return x
    return np.array([1.0, 0.0], dtype=np.float32)


def U0_for(cfg, kind="nominal", seed=1):
    """Initial control sequence [T, m] (fp32): "nominal" = u_init everywhere
    (zero force / hover thrust), "random" = nominal + N(0, 1) draws."""
    n, m, q = DIMS[cfg["dynamics"]]
    U = np.tile(np.asarray(cfg["u_init"][:m], dtype=np.float32), (cfg["T"], 1))
    if kind == "random":
        U = U + np.random.default_rng(seed).standard_normal(U.shape).astype(np.float32)
    return U.astype(np.float32)


def plant_disturbance(steps, dt, sigma, nu, sigma_J, seed=7):
    """Force disturbances of the simulated plant, one per control step:
    N(0, sigma^2) plus a Poisson(nu dt) number of N(0, sigma_J^2) jumps."""
    g = np.random.default_rng(seed)
    n = g.poisson(nu * dt, size=steps)
    d = sigma * g.standard_normal(steps) + sigma_J * np.sqrt(n) * g.standard_normal(steps)
    return d.astype(np.float32)


def random_controllers(count, seed=42):
    """Mixed cartpole / quadrotor controller set of the batched and serving
    forms: an exact half/half split, K from {512..8192}, T from [30, 150],
    nu from [0, 10] /s, random initial states, per-controller seed."""
    g = np.random.default_rng(seed)
    kinds = np.array([1] * (count // 2) + [2] * (count - count // 2))
    g.shuffle(kinds)
    out = []
    for i, d in enumerate(kinds):
        K = int(g.choice([512, 1024, 2048, 4096, 8192]))
        T = int(g.integers(30, 151))
        nu = float(g.uniform(0.0, 10.0))
        if d == 1:
            cfg = cartpole(K=K, T=T, nu=nu)
            x0 = np.array([g.uniform(-1, 1), 0.0, g.uniform(-math.pi, math.pi), 0.0],
                          dtype=np.float32)
        else:
            cfg = quadrotor(K=K, T=T, nu=nu)
            x0 = np.zeros(12, dtype=np.float32)
            x0[0:2] = g.uniform(-1, 1, size=2)
            x0[2] = g.uniform(0.5, 1.5)
            x0[6:9] = g.uniform(-0.1, 0.1, size=3)
        cfg.update(seed=42 + i, controller_id=i)
        out.append((cfg, x0))
    return out


def serving_controllers(count=1024, seed=4):
    """Resident controller set of the serving form: an exact half/half
    cartpole / quadrotor split in shuffled order, K from {1024..8192}, T from
    [50, 150], nu from [0, 10] /s, random initial states, per-controller
    seed and controller id."""
    g = np.random.default_rng(seed)
    kinds = np.array([1] * (count // 2) + [2] * (count - count // 2))
    g.shuffle(kinds)
    out = []
    for i, d in enumerate(kinds):
        K = int(g.choice([1024, 2048, 4096, 8192]))
        T = int(g.integers(50, 151))
        nu = float(g.uniform(0.0, 10.0))
        if d == 1:
            cfg = cartpole(K=K, T=T, nu=nu)
            x0 = np.array([g.uniform(-1, 1), 0.0, g.uniform(-math.pi, math.pi), 0.0],
                          dtype=np.float32)
        else:
            cfg = quadrotor(K=K, T=T, nu=nu)
            x0 = np.zeros(12, dtype=np.float32)
            x0[0:2] = g.uniform(-1, 1, size=2)
            x0[2] = g.uniform(0.5, 1.5)
            x0[6:9] = g.uniform(-0.1, 0.1, size=3)
        cfg.update(seed=1000 + i, controller_id=i)
        out.append((cfg, x0))
    return out


def serving_arrivals(rate, duration, count, seed=9):
    """Poisson request stream: arrival times (s, exponential gaps of mean
    1/rate) over [0, duration) and, for each, a uniformly chosen controller."""
    g = np.random.default_rng(seed)
    n = int(rate * duration * 1.2) + 64
    t = np.cumsum(g.exponential(1.0 / rate, size=n))
    while t[-1] < duration:
        t = np.concatenate([t, t[-1] + np.cumsum(g.exponential(1.0 / rate, size=n))])
    t = t[t < duration]
    return t, g.integers(0, count, size=len(t)).astype(np.int32)


def serving_disturbances(cfg, steps, seed):
    """Plant disturbances of one served controller, [steps, 8] fp32: words
    0..3 added to its control channels, N(0, sigma_j^2) per channel plus,
    where the model's jumps enter the control channels, a Poisson(nu dt)
    number of N(0, sigma_J^2) jumps (one count per step); words 4..6 the
    quadrotor's world-frame gust, sqrt(N) N(0, sigma_J^2) per axis with
    N ~ Poisson(nu dt), held for one step (the plant step applies it as a
    body force); word 7 unused."""
    n, m, q = DIMS[cfg["dynamics"]]
    g = np.random.default_rng(seed)
    sig = np.asarray(cfg["sigma"][:m], dtype=np.float64)
    d = np.zeros((steps, 8))
    d[:, :m] = sig * g.standard_normal((steps, m))
    cnt = g.poisson(cfg["nu"] * cfg["dt"], size=steps)
    if cfg["dynamics"] != 2:
        sj = np.asarray(cfg["sigma_J"][:m], dtype=np.float64)
        d[:, :m] += sj * np.sqrt(cnt)[:, None] * g.standard_normal((steps, m))
    else:
        sj = np.asarray(cfg["sigma_J"][:3], dtype=np.float64)
        d[:, 4:7] = sj * np.sqrt(cnt)[:, None] * g.standard_normal((steps, 3))
    return d.astype(np.float32)
