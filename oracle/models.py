"""Discrete-time dynamics and state costs of the three systems (FP64).

The paper's dynamics are the control-affine SDE of eqs. (2) and (4),
propagated by the explicit Euler step of Algorithm 1 (x_{i+1} = x_i + F dt,
noise entering through the sampled control).  The paper names the systems
(cartpole swing-up, quadrotor fly-to-target; Sec. VI) but not their
equations, constants or costs; the readings below are this implementation's
and are pinned only as stated.

  double integrator (dynamics id 0), n=2, m=1: x = [p, v]; p' = v, v' = u.
      Pinned by its closed-form linear propagation.
  cartpole (id 1), n=4, m=1: x = [p, p', theta, theta'], theta = 0 upright,
      force on the cart, frictionless pole of half-length l with the moment
      of inertia of a uniform rod (the classic Barto-Sutton-Anderson form):
        M = m_c + m_p,  tmp = (F + m_p l theta'^2 sin theta) / M
        theta'' = (g sin theta - cos theta tmp) / (l (4/3 - m_p cos^2 theta / M))
        p''     = tmp - m_p l theta'' cos theta / M
      Pinned against the Lagrangian equations of motion solved as a linear
      system, and by the upright equilibrium.
  quadrotor (id 2), n=12, m=4: x = [position(3), velocity(3), ZYX Euler
      angles (roll phi, pitch theta, yaw psi), body rates (p, q, r)], inputs
      are the four rotor thrusts of a "+" frame (rotor 1 on +x, 2 on +y, 3 on
      -x, 4 on -y), arm L, yaw reaction coefficient k:
        tau = (L (f2 - f4), L (f3 - f1), k (f1 - f2 + f3 - f4))
        v'  = R(phi, theta, psi) e3 sum(f) / mass - g e3 + gust / mass
        euler angle rates = W(phi, theta) omega
        omega' = J^-1 (tau - omega x J omega)
      Pinned by the hover equilibrium, R e3 against scipy's rotation, the
      Euler-rate map against a finite difference of the rotation, torques
      against r x F, and the gyroscopic term by conservation of rotational
      energy and angular-momentum magnitude.  The constants themselves (arm,
      yaw coefficient, crash rule) are readings: parity unpinned by the paper.

Costs: q(x) = (x - x*)^T diag(Q) (x - x*), phi(x) = (x - x*)^T diag(Qf) (x - x*)
(the paper leaves q and phi free, eqs. (1), (3), (5)); the quadrotor adds
the crash indicator times the crash penalty.
"""

import numpy as np


# ---------------------------------------------------------------- integrator
def linear_deriv(x, v):
    """Double integrator: (p', v') = (v, u)."""
    return np.stack([x[:, 1], v[:, 0]], axis=1)


# ---------------------------------------------------------------- cartpole
def cartpole_accel(x, F, P):
    """(p'', theta'') of the cartpole.  P = (m_cart, m_pole, half_length, g)."""
    m_c, m_p, l, g = P[0], P[1], P[2], P[3]
    th, thd = x[:, 2], x[:, 3]
    s, c = np.sin(th), np.cos(th)
    Mt = m_c + m_p
    tmp = (F + m_p * l * thd * thd * s) / Mt
    thdd = (g * s - c * tmp) / (l * (4.0 / 3.0 - m_p * c * c / Mt))
    pdd = tmp - m_p * l * thdd * c / Mt
    return pdd, thdd


def cartpole_deriv(x, v, P):
    pdd, thdd = cartpole_accel(x, v[:, 0], P)
    return np.stack([x[:, 1], pdd, x[:, 3], thdd], axis=1)


# ---------------------------------------------------------------- quadrotor
def rotor_torques(f, P):
    """Body torques of the "+" frame.  f: [K, 4] thrusts."""
    L, k = P[4], P[5]
    return np.stack([L * (f[:, 1] - f[:, 3]),
                     L * (f[:, 2] - f[:, 0]),
                     k * (f[:, 0] - f[:, 1] + f[:, 2] - f[:, 3])], axis=1)


def body_z_in_world(phi, th, psi):
    """Third column of R = Rz(psi) Ry(theta) Rx(phi)."""
    cph, sph = np.cos(phi), np.sin(phi)
    cth, sth = np.cos(th), np.sin(th)
    cps, sps = np.cos(psi), np.sin(psi)
    return np.stack([cps * sth * cph + sps * sph,
                     sps * sth * cph - cps * sph,
                     cth * cph], axis=1)


def euler_rates(phi, th, w):
    """ZYX Euler-angle rates from body rates w = (p, q, r)."""
    p, q, r = w[:, 0], w[:, 1], w[:, 2]
    sph, cph = np.sin(phi), np.cos(phi)
    tth, cth = np.tan(th), np.cos(th)
    return np.stack([p + (q * sph + r * cph) * tth,
                     q * cph - r * sph,
                     (q * sph + r * cph) / cth], axis=1)


def body_rate_accel(w, tau, P):
    """omega' = J^-1 (tau - omega x J omega), J = diag(Jx, Jy, Jz)."""
    Jx, Jy, Jz = P[1], P[2], P[3]
    p, q, r = w[:, 0], w[:, 1], w[:, 2]
    return np.stack([(tau[:, 0] - (Jz - Jy) * q * r) / Jx,
                     (tau[:, 1] - (Jx - Jz) * r * p) / Jy,
                     (tau[:, 2] - (Jy - Jx) * p * q) / Jz], axis=1)


def quadrotor_deriv(x, f, gust, P):
    """P = (mass, Jx, Jy, Jz, arm, k_yaw, g, tilt_max, z_min)."""
    mass, g = P[0], P[6]
    vel = x[:, 3:6]
    phi, th, psi = x[:, 6], x[:, 7], x[:, 8]
    w = x[:, 9:12]
    thrust = f.sum(axis=1)
    acc = body_z_in_world(phi, th, psi) * (thrust / mass)[:, None] + gust / mass
    acc[:, 2] -= g
    tau = rotor_torques(f, P)
    return np.concatenate([vel, acc, euler_rates(phi, th, w),
                           body_rate_accel(w, tau, P)], axis=1)


def quadrotor_crashed(x, P):
    """Crash rule: below z_min, or roll or pitch beyond tilt_max."""
    tilt, zmin = P[7], P[8]
    return (x[:, 2] < zmin) | (np.abs(x[:, 6]) > tilt) | (np.abs(x[:, 7]) > tilt)


def quadrotor_margin(x, P):
    """Distance of the state to the crash boundary (for parity screening)."""
    tilt, zmin = P[7], P[8]
    return np.minimum(np.abs(x[:, 2] - zmin),
                      np.minimum(np.abs(tilt - np.abs(x[:, 6])),
                                 np.abs(tilt - np.abs(x[:, 7]))))


# ---------------------------------------------------------------- dispatch
def deriv(dynamics, x, v, gust, P):
    if dynamics == 0:
        return linear_deriv(x, v)
    if dynamics == 1:
        return cartpole_deriv(x, v, P)
    if dynamics == 2:
        return quadrotor_deriv(x, v, gust, P)
    raise ValueError("unknown dynamics id %r" % (dynamics,))


def euler_step(dynamics, x, v, gust, dt, P):
    """One explicit Euler step (Algorithm 1): x + F(x, v) dt."""
    return x + deriv(dynamics, x, v, gust, P) * dt


def state_cost(x, Q, goal):
    d = x - goal
    return (d * d * Q).sum(axis=1)
