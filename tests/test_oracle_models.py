"""Pins of the oracle's dynamics (CPU only): the cartpole against its
Lagrangian equations of motion, the quadrotor against rotation, kinematic and
rigid-body identities computed independently, the double integrator against
its closed-form linear propagation, and the equilibria."""

import numpy as np
from scipy.linalg import expm
from scipy.spatial.transform import Rotation

from oracle import models
from paper_1807_06108_amd import workloads

CP = np.array(workloads.CARTPOLE_PARAMS, dtype=np.float64)
QP = np.array(workloads.QUAD_PARAMS, dtype=np.float64)


def test_cartpole_matches_lagrangian():
    # Generalised coordinates (p, theta); pole: uniform rod of length 2l
    # (moment of inertia m_p l^2 / 3 about its centre), theta = 0 upright.
    # Mass matrix and forcing from the Lagrangian, solved as a linear system.
    m_c, m_p, l, g = CP
    rng = np.random.default_rng(0)
    x = rng.uniform(-3, 3, size=(200, 4))
    F = rng.uniform(-20, 20, size=200)
    pdd, thdd = models.cartpole_accel(x, F, CP)
    for i in range(200):
        th, thd = x[i, 2], x[i, 3]
        Mq = np.array([[m_c + m_p, m_p * l * np.cos(th)],
                       [m_p * l * np.cos(th), m_p * l * l * (1 + 1 / 3)]])
        rhs = np.array([F[i] + m_p * l * np.sin(th) * thd**2,
                        m_p * g * l * np.sin(th)])
        sol = np.linalg.solve(Mq, rhs)
        assert np.allclose([pdd[i], thdd[i]], sol, rtol=1e-12, atol=1e-12)


def test_cartpole_upright_equilibrium_is_exact():
    x = np.zeros((3, 4))
    for _ in range(100):
        x = models.euler_step(1, x, np.zeros((3, 1)), np.zeros((3, 3)), 0.02, CP)
    assert not x.any()


def test_double_integrator_closed_form():
    rng = np.random.default_rng(1)
    T, dt = 30, 0.1
    v = rng.standard_normal((5, T))
    x = np.tile([1.0, -0.5], (5, 1))
    A = np.array([[1.0, dt], [0.0, 1.0]])
    B = np.array([0.0, dt])
    for t in range(T):
        x = models.euler_step(0, x, v[:, t:t + 1], None, dt, None)
    ref = np.array([np.linalg.matrix_power(A, T) @ [1.0, -0.5]
                    + sum(np.linalg.matrix_power(A, T - 1 - t) @ B * v[k, t]
                          for t in range(T)) for k in range(5)])
    assert np.allclose(x, ref, rtol=1e-12, atol=1e-12)


def test_quadrotor_hover_equilibrium():
    x = np.zeros((2, 12))
    x[:, 2] = 1.0
    f = np.full((2, 4), workloads.QUAD_HOVER)
    x1 = x
    for _ in range(100):
        x1 = models.euler_step(2, x1, f, np.zeros((2, 3)), 0.01, QP)
    assert np.abs(x1 - x).max() < 1e-12


def test_quadrotor_body_axis_matches_scipy_rotation():
    rng = np.random.default_rng(2)
    e = rng.uniform(-1.2, 1.2, size=(100, 3))
    z = models.body_z_in_world(e[:, 0], e[:, 1], e[:, 2])
    for i in range(100):
        R = Rotation.from_euler("ZYX", [e[i, 2], e[i, 1], e[i, 0]]).as_matrix()
        assert np.allclose(z[i], R[:, 2], atol=1e-13)


def test_quadrotor_euler_rates_match_rotation_kinematics():
    # R(eta + h * eta_dot) ~ R(eta) expm(h [omega]_x) to first order in h.
    rng = np.random.default_rng(3)
    h = 1e-6
    for _ in range(50):
        eta = rng.uniform(-1.0, 1.0, size=3)
        w = rng.uniform(-2, 2, size=3)
        rates = models.euler_rates(np.array([eta[0]]), np.array([eta[1]]), w[None, :])[0]

        def R(a):
            return Rotation.from_euler("ZYX", [a[2], a[1], a[0]]).as_matrix()
        W = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
        lhs = (R(eta + h * rates) - R(eta)) / h
        rhs = (R(eta) @ expm(h * W) - R(eta)) / h
        assert np.allclose(lhs, rhs, atol=1e-5)


def test_quadrotor_torques_are_r_cross_f():
    rng = np.random.default_rng(4)
    f = rng.uniform(0, 5, size=(20, 4))
    tau = models.rotor_torques(f, QP)
    L, k = QP[4], QP[5]
    pos = np.array([[L, 0, 0], [0, L, 0], [-L, 0, 0], [0, -L, 0]])
    spin = np.array([1, -1, 1, -1])  # reaction torque sign per rotor
    for i in range(20):
        ref = sum(np.cross(pos[j], [0, 0, f[i, j]]) for j in range(4))
        ref = ref + np.array([0, 0, k * (spin * f[i]).sum()])
        assert np.allclose(tau[i], ref, atol=1e-13)


def test_quadrotor_gyroscopic_term_conserves_energy_and_momentum():
    rng = np.random.default_rng(5)
    w = rng.uniform(-5, 5, size=(100, 3))
    J = QP[1:4]
    wd = models.body_rate_accel(w, np.zeros((100, 3)), QP)
    # d/dt (1/2 w^T J w) = w^T J w' = 0 and d/dt |J w|^2 = 2 (J w)^T J w' = 0
    assert np.abs((w * J * wd).sum(1)).max() < 1e-10
    assert np.abs(((J * w) * (J * wd)).sum(1)).max() < 1e-10
    tau = rng.uniform(-1, 1, size=(100, 3))
    wd = models.body_rate_accel(w, tau, QP)
    assert np.allclose((w * J * wd).sum(1), (w * tau).sum(1), atol=1e-10)


def test_quadrotor_translational_and_gust():
    x = np.zeros((1, 12))
    f = np.full((1, 4), 3.0)
    gust = np.array([[0.5, -1.0, 2.0]])
    d = models.quadrotor_deriv(x, f, gust, QP)
    m, g = QP[0], QP[6]
    assert np.allclose(d[0, 3:6], [0.5 / m, -1.0 / m, 12.0 / m - g + 2.0 / m])


def test_quadrotor_crash_rule():
    x = np.zeros((4, 12))
    x[:, 2] = 1.0
    x[1, 2] = -1e-3
    x[2, 6] = 1.21
    x[3, 7] = -1.21
    assert list(models.quadrotor_crashed(x, QP)) == [False, True, True, True]
