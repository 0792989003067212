"""Sampling of the control perturbations: Gaussian part plus compound-Poisson jumps.

What is sampled (paper, Sec. IV-B and Algorithm 1): at every time step j each
sampled control is the nominal one plus a diffusion term eps_D ~ N(0, Sigma_D)
and a jump term whose count follows the jump law with mean nu*dt and whose
mark is N(0, Sigma_J) (Sec. II: zero-mean normal mark distribution).  Readings
fixed here (also listed in the design notes):
  * all noise parameters are per-step control-space values (sigma, sigma_J);
  * one jump count per (sample, step) shared by the channels, with a vector
    mark; the sum of N i.i.d. N(0, diag sigma_J^2) marks is drawn as
    sqrt(N) * sigma_J * z_J, which has exactly that distribution;
  * count law: Poisson(nu*dt) (default) or the zero-one law of Sec. IV-B /
    Algorithm 1 (Bernoulli(nu*dt));
  * where the jump enters: through the control channel (cartpole, double
    integrator; part of eps) or as a world-frame force on the body
    (quadrotor; a rollout disturbance only, not part of eps).

Random words come from Philox4x32-10 (oracle.philox), with
  key     = (seed mod 2^32, seed >> 32)
  counter = (t, k, iteration mod 2^32, block | controller_id << 8)
Per (k, t) the blocks are concatenated into a word stream w[0], w[1], ...
Normal number i comes from the Box-Muller pair i // 2 (words 2p, 2p+1):
  u = ((w[2p] >> 8) + 1) / 2^24 in (0, 1]     (radius: -2 ln u finite)
  v =  (w[2p+1] >> 8)     / 2^24 in [0, 1)    (angle: 2 pi v)
  normal 2p = sqrt(-2 ln u) cos(2 pi v), normal 2p+1 = sqrt(-2 ln u) sin(2 pi v)
(Box & Muller 1958).  The first m normals are z_D, the next q are z_J.  The
jump-count word is the word after the last pair when that word lies in a
block the pairs already use (one- and two-channel models: word 2); when the
pairs fill whole blocks (the quadrotor: 4 pairs, words 0-7, two blocks) it is
assembled from the low bytes of words 0-3, which Box-Muller leaves unused:
  w_count = (w[0] & 255) | (w[1] & 255) << 8 | (w[2] & 255) << 16 | (w[3] & 255) << 24
so that no block is drawn for one word.  The count is the number of integer
thresholds theta_0 <= theta_1 <= ... that the 32-bit word reaches,
theta_j = floor(F(j) * 2^32) with F the CDF of the count law (inversion; the
decision is taken in integers, so both implementations agree exactly).

Parity: pinned.  Box-Muller by its closed form at special angles/radii and by
a Kolmogorov-Smirnov test; thresholds against scipy.stats.poisson.cdf and
exact rational arithmetic; counts and marginals by their moments; the
zero-one marginal by the mixture density of eq. (42).
"""

import math

import numpy as np

from .philox import philox4x32

MAX_LEVELS = 32          # most thresholds a count law may need
TWO32 = 1 << 32

DIMS = {0: (2, 1, 1),    # double integrator: n, m, q
        1: (4, 1, 1),    # cartpole
        2: (12, 4, 3)}   # quadrotor
JUMP_IN_CONTROL = {0: True, 1: True, 2: False}


def layout(dynamics):
    """(n, m, q, count_word, n_blocks) of the per-(k, t) word stream;
    count_word is None when the count word is assembled from low bytes."""
    n, m, q = DIMS[dynamics]
    pairs = (m + q + 1) // 2
    if (2 * pairs) % 4 == 0:
        return n, m, q, None, 2 * pairs // 4
    count_word = 2 * pairs
    n_blocks = count_word // 4 + 1
    return n, m, q, count_word, n_blocks


def low_byte_word(w):
    """Count word from the low bytes of words 0-3 of the stream (uint32)."""
    w = w.astype(np.uint64)
    out = (w[..., 0] & 255) | ((w[..., 1] & 255) << 8) | ((w[..., 2] & 255) << 16) \
        | ((w[..., 3] & 255) << 24)
    return out.astype(np.uint32)


def words(seed, controller_id, iteration, k_index, T, n_blocks):
    """Philox word stream, uint32 [len(k_index), T, 4 * n_blocks]."""
    k = np.asarray(k_index, dtype=np.uint64)
    K = k.shape[0]
    key = (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    out = np.empty((K, T, 4 * n_blocks), dtype=np.uint32)
    t = np.arange(T, dtype=np.uint64)
    for b in range(n_blocks):
        ctr = np.empty((K, T, 4), dtype=np.uint64)
        ctr[..., 0] = t[None, :]
        ctr[..., 1] = k[:, None]
        ctr[..., 2] = iteration & 0xFFFFFFFF
        ctr[..., 3] = b | (controller_id << 8)
        out[..., 4 * b:4 * b + 4] = philox4x32(ctr, key)
    return out


def box_muller(w_radius, w_angle):
    """Two standard normals from two 32-bit words (fp64)."""
    u = ((w_radius.astype(np.int64) >> 8) + 1) / float(1 << 24)
    v = (w_angle.astype(np.int64) >> 8) / float(1 << 24)
    r = np.sqrt(-2.0 * np.log(u))
    return r * np.cos(2.0 * math.pi * v), r * np.sin(2.0 * math.pi * v)


def count_thresholds(a, count_law):
    """Integer inversion thresholds of the count law with mean a = nu*dt.

    Poisson: F(j) = exp(-a) sum_{i<=j} a^i / i!, built by the recurrence
    p_j = p_{j-1} a / j.  Zero-one law (Sec. IV-B): F(0) = 1 - a, F(1) = 1.
    theta_j = floor(F(j) 2^32); the first level whose threshold reaches
    2^32 - 1 (remaining tail mass below 2^-32) is closed at 2^32.
    Raises ValueError when the law does not fit in MAX_LEVELS levels.
    """
    if not (a >= 0.0) or math.isinf(a):
        raise ValueError("jump mean nu*dt must be finite and >= 0")
    if count_law == 1:
        if a > 1.0:
            raise ValueError("zero-one law needs nu*dt <= 1")
        th0 = min(int(math.floor((1.0 - a) * TWO32)), TWO32)
        return [th0, TWO32] if th0 < TWO32 else [TWO32]
    if count_law != 0:
        raise ValueError("unknown count law")
    th = []
    p = math.exp(-a)
    F = p
    for j in range(MAX_LEVELS):
        if j > 0:
            p = p * a / j
            F = F + p
        tj = int(math.floor(F * TWO32))
        if tj >= TWO32 - 1:
            th.append(TWO32)
            return th
        th.append(tj)
    raise ValueError("nu*dt too large for %d count levels" % MAX_LEVELS)


def counts(w, thresholds):
    """Count = number of thresholds the word reaches."""
    w = w.astype(np.int64)
    N = np.zeros(w.shape, dtype=np.int32)
    for th in thresholds:
        N += (w >= th).astype(np.int32)
    return N


def sample(cfg, iteration, k_index=None):
    """Standard-normal and count draws of one iteration.

    Returns z_D [K', T, m], N [K', T] (int32), z_J [K', T, q] for the samples
    k_index (default: all K).  Sample k draws the stream of global sample
    index sample_offset + k (a shard of a larger sample set)."""
    dyn = cfg["dynamics"]
    n, m, q, cw, nb = layout(dyn)
    K, T = cfg["K"], cfg["T"]
    if k_index is None:
        k_index = np.arange(K)
    k_glob = int(cfg.get("sample_offset", 0)) + np.asarray(k_index, dtype=np.int64)
    w = words(cfg["seed"], cfg["controller_id"], iteration, k_glob, T, nb)
    normals = []
    for p in range((m + q + 1) // 2):
        z0, z1 = box_muller(w[..., 2 * p], w[..., 2 * p + 1])
        normals += [z0, z1]
    z_D = np.stack(normals[:m], axis=-1)
    z_J = np.stack(normals[m:m + q], axis=-1)
    a = float(np.float32(cfg["nu"])) * float(np.float32(cfg["dt"]))
    wc = low_byte_word(w) if cw is None else w[..., cw]
    N = counts(wc, count_thresholds(a, cfg.get("count_law", 0)))
    return z_D, N, z_J


def cholesky_factor(cfg):
    """The m x m Gaussian covariance factor L (Sigma_D = L L^T) of a
    configuration with a full covariance, as fp64 of its fp32 entries, or
    None for the diagonal form (Sigma_D = diag sigma^2)."""
    if not int(cfg.get("full_sigma", 0)):
        return None
    m = DIMS[cfg["dynamics"]][1]
    L = np.asarray(cfg["sigma_L"], dtype=np.float32).astype(np.float64).reshape(4, 4)
    return L[:m, :m]


def compose(cfg, z_D, N, z_J):
    """Control perturbation eps [K', T, m] and body-force disturbance
    gust [K', T, 3] from the standard draws (readings in the module header).
    The Gaussian part is sigma * z_D, or L z_D for a full covariance
    Sigma_D = L L^T (Sec. IV-B: eps_D ~ N(0, Sigma_D))."""
    dyn = cfg["dynamics"]
    n, m, q = DIMS[dyn]
    sigma = np.asarray(cfg["sigma"][:m], dtype=np.float32).astype(np.float64)
    sigJ = np.asarray(cfg["sigma_J"][:q], dtype=np.float32).astype(np.float64)
    L = cholesky_factor(cfg)
    eps_D = z_D * sigma if L is None else z_D @ L.T
    J = np.sqrt(N.astype(np.float64))[..., None] * z_J * sigJ
    if JUMP_IN_CONTROL[dyn]:
        return eps_D + J, np.zeros(J.shape[:-1] + (3,))
    return eps_D, J
