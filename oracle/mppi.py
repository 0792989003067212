"""One MPPI iteration on a jump-diffusion process, step by step, in FP64.

Follows the paper's Algorithm 1 ("MPPI Control on Jump Diffusion") and the
equations it rests on:
  sampling      - Sec. IV-B noise model, Algorithm 1 jump timer (oracle.noise);
  rollout       - explicit Euler propagation of the sampled controls;
  path cost     - the modified cost S~ of eqs. (34)-(35): state cost and
                  nominal control cost times dt, plus the importance-sampling
                  terms;
  weights       - exp(-S~/lambda) normalised, eq. (37); the minimum is
                  subtracted first, which leaves the normalised weights
                  unchanged;
  update        - U_j += alpha * sum_k w_k eps_{k,j}, eq. (36) with the
                  control-channel simplification stated after eq. (49)
                  (G^-1 B = identity), step size alpha of eq. (49);
  shift         - execute u_0, shift left, append u_init (Algorithm 1, Sec. V).

Readings of passages the paper leaves open (listed again in the design notes):
  * eps is a per-step control-space perturbation, so the paper's
    eps/sqrt(dt) is eps here and the update is U += sum w eps;
  * IS terms per step, from the Gaussian likelihood ratio behind eq. (35)
    with sampling covariance Sigma_s = diag(sigma^2), or Sigma_s = L L^T
    for a full covariance given by its Cholesky factor L:
        lambda * c * U_t^T Sigma_s^-1 eps_t + 0.5 lambda (c - 1) eps_t^T Sigma_s^-1 eps_t
    (channels with sigma = 0 contribute nothing); the IS term uses the full
    perturbation including a control-channel jump, as Algorithm 1 adds the
    jump to eps before the cost;
  * the running cost is taken on the pre-step states x_0..x_{T-1} and the
    terminal cost on x_T (eq. (34));
  * "SO" cost form (Sec. IV): J = phi + sum (q + 0.5 v^T R v) dt on the
    applied control v = U + eps, with no IS term;
  * quadrotor crash: sticky; the state freezes; the penalty is added inside
    q (so times dt) for every crashed step and once to the terminal cost;
  * non-finite S_k get zero weight and are ignored by the minimum; when no
    S_k is finite the update is skipped (status "non-finite").

Parity: pinned by the CPU tests (closed-form double integrator, equilibria,
weight invariants, zero noise, lambda -> 0 against brute_force_argmin,
lambda -> infinity, nu = 0 against gaussian_only_iteration, IT = SO when the
IS and control-cost terms vanish, exact shift, permutation invariance).
"""

import math

import numpy as np

from . import models, noise

STATUS_OK = 0
STATUS_NONFINITE = -4


def f32(v):
    """The fp32 value a config field holds, as fp64."""
    return np.asarray(v, dtype=np.float32).astype(np.float64)


def params(cfg):
    """Config floats as the fp32 values the configuration carries."""
    n, m, q = noise.DIMS[cfg["dynamics"]]
    sig = f32(cfg["sigma"][:m])
    iv = np.where(sig > 0, 1.0 / np.where(sig > 0, sig * sig, 1.0), 0.0)
    L = noise.cholesky_factor(cfg)
    # inverse sampling covariance: L^-T L^-1 from the factor, or diagonal
    Pinv = None if L is None else np.linalg.inv(L @ L.T)
    return dict(Pinv=Pinv,
        n=n, m=m, q=q,
        dt=float(f32(cfg["dt"])), lam=float(f32(cfg["lambda"])),
        alpha=float(f32(cfg.get("alpha", 1.0))), c=float(f32(cfg.get("c", 1.0))),
        inv_var=iv, R=f32(cfg["R"][:m]), Q=f32(cfg["Q"][:n]),
        Qf=f32(cfg["Qf"][:n]), goal=f32(cfg["x_goal"][:n]),
        P=f32(cfg.get("params", [0.0] * 12)),
        pen=float(f32(cfg.get("crash_penalty", 0.0))),
        cost_form=int(cfg.get("cost_form", 0)),
        u_init=f32(cfg["u_init"][:m]))


def rollout(cfg, x0, U, eps, gust, with_magnitude=False):
    """Path costs S~_k of eq. (34) for the perturbations eps [K', T, m] and
    body-force disturbances gust [K', T, 3].

    Returns (S [K'], crash_margin [K']); the margin is the smallest distance
    of any visited quadrotor state to the crash boundary (inf otherwise).
    with_magnitude: also the sum of the magnitudes of the terms that make up
    each S~_k (every running-cost, control-cost and importance-sampling term
    and the terminal cost), the scale against which the rounding of a sum of
    signed terms is measured: the IS cross term of eq. (35) is signed, so S~
    can be far smaller than its terms."""
    p = params(cfg)
    dyn = cfg["dynamics"]
    Kp, T, m = eps.shape
    dt, lam, c = p["dt"], p["lam"], p["c"]
    x = np.repeat(f32(x0)[None, :p["n"]], Kp, axis=0)
    U = np.asarray(U, dtype=np.float64).reshape(T, m)
    S = np.zeros(Kp)
    Sabs = np.zeros(Kp)
    crashed = np.zeros(Kp, dtype=bool)
    margin = np.full(Kp, np.inf)
    if dyn == 2:
        margin = models.quadrotor_margin(x, p["P"])
        crashed = models.quadrotor_crashed(x, p["P"])
    for t in range(T):
        e = eps[:, t, :]
        v = U[t][None, :] + e
        qx = models.state_cost(x, p["Q"], p["goal"]) + p["pen"] * crashed
        if p["cost_form"] == 0:
            ctrl = 0.5 * float((p["R"] * U[t] * U[t]).sum())
            if p["Pinv"] is None:
                is_cross = lam * c * (U[t][None, :] * e * p["inv_var"]).sum(axis=1)
                is_var = 0.5 * lam * (c - 1.0) * (e * e * p["inv_var"]).sum(axis=1)
            else:
                is_cross = lam * c * (e @ (p["Pinv"] @ U[t]))
                is_var = 0.5 * lam * (c - 1.0) * np.einsum("ki,ij,kj->k", e, p["Pinv"], e)
            S = S + (qx + ctrl) * dt + is_cross + is_var
            Sabs = Sabs + (np.abs(qx) + abs(ctrl)) * dt + np.abs(is_cross) + np.abs(is_var)
        else:
            S = S + (qx + 0.5 * (p["R"] * v * v).sum(axis=1)) * dt
            Sabs = Sabs + (np.abs(qx) + 0.5 * (np.abs(p["R"]) * v * v).sum(axis=1)) * dt
        xn = models.euler_step(dyn, x, v, gust[:, t, :], dt, p["P"])
        if dyn == 2:
            xn = np.where(crashed[:, None], x, xn)
            margin = np.minimum(margin, np.where(crashed, np.inf,
                                                 models.quadrotor_margin(xn, p["P"])))
            crashed = crashed | models.quadrotor_crashed(xn, p["P"])
        x = xn
    phi = models.state_cost(x, p["Qf"], p["goal"]) + p["pen"] * crashed
    S = S + phi
    if with_magnitude:
        return S, margin, Sabs + np.abs(phi)
    return S, margin


def weights(S, lam):
    """w_k = exp(-(S_k - rho)/lambda) / eta over the finite S_k (eq. (37)).

    Returns (w, rho, eta, status)."""
    S = np.asarray(S, dtype=np.float64)
    fin = np.isfinite(S)
    if not fin.any():
        return np.zeros_like(S), math.nan, 0.0, STATUS_NONFINITE
    rho = S[fin].min()
    e = np.where(fin, np.exp(-(np.where(fin, S, rho) - rho) / lam), 0.0)
    eta = e.sum()
    return e / eta, float(rho), float(eta), STATUS_OK


def update(U, w, eps, alpha=1.0):
    """U'[t, j] = U[t, j] + alpha * sum_k w_k eps[k, t, j]."""
    return np.asarray(U, dtype=np.float64) + alpha * np.einsum("k,ktj->tj", w, eps)


def iteration(cfg, x0, U, it, k_index=None):
    """One full iteration with the method's own noise draws (Philox)."""
    z_D, N, z_J = noise.sample(cfg, it, k_index)
    eps, gust = noise.compose(cfg, z_D, N, z_J)
    S, margin, S_abs = rollout(cfg, x0, U, eps, gust, with_magnitude=True)
    out = dict(z_D=z_D, N=N, z_J=z_J, eps=eps, gust=gust, S=S, margin=margin, S_abs=S_abs)
    if k_index is None:
        w, rho, eta, status = weights(S, float(f32(cfg["lambda"])))
        U = np.asarray(U, dtype=np.float64).reshape(cfg["T"], -1)
        out.update(w=w, rho=rho, eta=eta, status=status,
                   U=U if status != STATUS_OK else
                   update(U, w, eps, float(f32(cfg.get("alpha", 1.0)))))
    return out


def shift(U, u_init):
    """Execute u_0; U[t] <- U[t+1]; U[T-1] <- u_init (Algorithm 1)."""
    U = np.asarray(U, dtype=np.float64)
    u0 = U[0].copy()
    Us = np.empty_like(U)
    Us[:-1] = U[1:]
    Us[-1] = u_init
    return u0, Us


def control_step(cfg, x0, U, it0, iters):
    """iters iterations from the same x0 (fresh iteration index each), then
    the shift: one MPC control step."""
    for i in range(iters):
        U = iteration(cfg, x0, U, it0 + i)["U"]
    return shift(U, f32(cfg["u_init"][:U.shape[1]]))


# -------------------------------------------------------- reference forms
def scalar_path_cost(cfg, x0, U, e):
    """S~ of one sample by a plain loop over python floats (double integrator
    and cartpole), written separately from rollout(): e is that sample's
    perturbation [T] (single control channel)."""
    dyn = cfg["dynamics"]
    assert dyn in (0, 1)
    p = params(cfg)
    lam, dt, c = p["lam"], p["dt"], p["c"]
    Q, Qf, goal = [list(map(float, p[k])) for k in ("Q", "Qf", "goal")]
    R0, iv = float(p["R"][0]), float(p["inv_var"][0])
    x = [float(v) for v in f32(x0)[:p["n"]]]
    s = 0.0
    for t in range(len(e)):
        u, ek = float(U[t]), float(e[t])
        s += sum(Q[i] * (x[i] - goal[i]) ** 2 for i in range(len(x))) * dt
        if p["cost_form"] == 0:
            s += 0.5 * R0 * u * u * dt
            s += lam * c * u * ek * iv + 0.5 * lam * (c - 1.0) * ek * ek * iv
        else:
            s += 0.5 * R0 * (u + ek) ** 2 * dt
        F = u + ek
        if dyn == 0:
            x = [x[0] + x[1] * dt, x[1] + F * dt]
        else:
            m_c, m_p, l, g = [float(v) for v in p["P"][:4]]
            th, thd = x[2], x[3]
            tot = m_c + m_p
            tmp = (F + m_p * l * thd * thd * math.sin(th)) / tot
            thdd = (g * math.sin(th) - math.cos(th) * tmp) / (
                l * (4.0 / 3.0 - m_p * math.cos(th) ** 2 / tot))
            pdd = tmp - m_p * l * thdd * math.cos(th) / tot
            x = [x[0] + x[1] * dt, x[1] + pdd * dt,
                 x[2] + x[3] * dt, x[3] + thdd * dt]
    return s + sum(Qf[i] * (x[i] - goal[i]) ** 2 for i in range(len(x)))


def gaussian_only_iteration(cfg, x0, U, it):
    """MPPI without jumps (the "old MPPI" of Sec. VI; eqs. (36)-(37) with the
    diffusion perturbation only): per-sample scalar loops, Gaussian draws only,
    plain normalised exponential weights."""
    K, T = cfg["K"], cfg["T"]
    z_D = noise.sample(cfg, it)[0][:, :, 0]
    sigma = float(f32(cfg["sigma"][0]))
    lam = float(f32(cfg["lambda"]))
    alpha = float(f32(cfg.get("alpha", 1.0)))
    U = np.asarray(U, dtype=np.float64).reshape(T)
    S = np.array([scalar_path_cost(cfg, x0, U, sigma * z_D[k]) for k in range(K)])
    e = np.exp(-(S - S.min()) / lam)
    w = e / e.sum()
    dU = np.array([sum(w[k] * sigma * z_D[k, t] for k in range(K)) for t in range(T)])
    return S, U + alpha * dU


def brute_force_argmin(cfg, x0, U, eps):
    """U + eps of the lowest-cost sample, found by a plain per-sample scalar
    loop (the lambda -> 0 limit of eq. (37)); double integrator and cartpole."""
    K, T, m = eps.shape
    U = np.asarray(U, dtype=np.float64).reshape(T)
    costs = [scalar_path_cost(cfg, x0, U, eps[k, :, 0]) for k in range(K)]
    best_k = min(range(K), key=lambda k: costs[k])
    return (U + eps[best_k, :, 0])[:, None], best_k
