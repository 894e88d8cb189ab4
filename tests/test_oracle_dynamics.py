"""Pins of the oracle's cubic edge (Eq. 6) and torque model (Eqs. 4-5)
against closed forms, independent kinematics and invariants."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2609_22608_amd import workload as W
from tests import kin

RIGID_G = O.T_RIGID | O.T_GRAVITY


def rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return np.max(np.abs(a - b)) / max(1e-300, np.max(np.abs(b)))


# ---------------------------------------------------------------- cubic

@pytest.mark.parametrize("seed", range(5))
def test_cubic_reproduces_boundary_states(seed):
    rng = np.random.default_rng(seed)
    x0 = rng.uniform(-2, 2, 14)
    x1 = rng.uniform(-2, 2, 14)
    for T in (0.02, 0.137, 1.0, 3.7):
        s, sd, _ = O.cubic(x0, x1, T, 0.0)
        assert np.max(np.abs(s - x0[:7])) <= 1e-12
        assert np.max(np.abs(sd - x0[7:])) <= 1e-12
        s, sd, _ = O.cubic(x0, x1, T, T)
        assert np.max(np.abs(s - x1[:7])) <= 1e-12 * max(1.0, np.max(np.abs(x1)))
        assert np.max(np.abs(sd - x1[7:])) <= 1e-12 * max(1.0, np.max(np.abs(x1)) / T)


@pytest.mark.parametrize("seed", range(3))
def test_cubic_equals_hermite_basis(seed):
    """The monomial form of Eq. (6) equals the cubic Hermite interpolant."""
    rng = np.random.default_rng(100 + seed)
    x0 = rng.uniform(-2, 2, 14)
    x1 = rng.uniform(-2, 2, 14)
    T = 0.63
    for u in np.linspace(0, 1, 11):
        h00 = 2 * u**3 - 3 * u**2 + 1
        h10 = u**3 - 2 * u**2 + u
        h01 = -2 * u**3 + 3 * u**2
        h11 = u**3 - u**2
        ref = h00 * x0[:7] + h10 * T * x0[7:] + h01 * x1[:7] + h11 * T * x1[7:]
        dref = (6 * u**2 - 6 * u) / T * x0[:7] + (3 * u**2 - 4 * u + 1) * x0[7:] \
            + (-6 * u**2 + 6 * u) / T * x1[:7] + (3 * u**2 - 2 * u) * x1[7:]
        s, sd, _ = O.cubic(x0, x1, T, u * T)
        assert np.max(np.abs(s - ref)) <= 1e-12
        assert np.max(np.abs(sd - dref)) <= 1e-12


def test_cubic_initial_acceleration_is_controller_law():
    """sigma''(0) equals the controller's feed-forward of Eq. (9) before
    clipping: 6 (q_g - q)/T^2 - (4 qd + 2 qd_g)/T."""
    rng = np.random.default_rng(7)
    for _ in range(20):
        x0 = rng.uniform(-2, 2, 14)
        x1 = rng.uniform(-2, 2, 14)
        T = rng.uniform(0.05, 1.5)
        _, _, sdd = O.cubic(x0, x1, T, 0.0)
        law = 6 * (x1[:7] - x0[:7]) / T**2 - (4 * x0[7:] + 2 * x1[7:]) / T
        assert rel(sdd, law) <= 1e-12


# ---------------------------------------------------------------- friction

def test_friction_zero_at_rest_and_saturation():
    rng = np.random.default_rng(3)
    for _ in range(50):
        p1, p2, p3 = rng.uniform(0.1, 0.6), rng.uniform(5, 50), rng.uniform(-0.05, 0.05)
        assert O.friction(p1, p2, p3, 0.0) == pytest.approx(0.0, abs=1e-15)
        s = 1.0 / (1.0 + math.exp(-p2 * p3))
        assert O.friction(p1, p2, p3, 1e3) == pytest.approx(p1 * (1 - s), rel=1e-12)
        assert O.friction(p1, p2, p3, -1e3) == pytest.approx(-p1 * s, rel=1e-12)
        v = rng.uniform(-3, 3)
        direct = p1 / (1 + math.exp(-p2 * (v + p3))) - p1 / (1 + math.exp(-p2 * p3))
        assert O.friction(p1, p2, p3, v) == pytest.approx(direct, rel=1e-12, abs=1e-15)


# ---------------------------------------------------------------- RNEA

def planar_arm(l1, l2, lc1, lc2, m1, m2, I1, I2, g=9.81):
    """Two parallel z axes (DH alpha = 0), motion in the x-y plane, gravity
    along -y."""
    return dict(n=2, alpha=np.zeros(2), a=np.array([0.0, l1]), d=np.zeros(2),
                m=np.array([m1, m2]), rc=np.array([[lc1, 0, 0], [lc2, 0, 0.0]]),
                I=np.array([[0.01, 0.02, I1], [0.01, 0.02, I2]]), Im=np.zeros(2),
                psi1=np.zeros(2), psi2=np.ones(2), psi3=np.zeros(2),
                qmin=-np.ones(2) * 3, qmax=np.ones(2) * 3, qdmax=np.ones(2) * 3,
                taumax=np.ones(2) * 50, acc=np.ones(2) * 10, wmax=100.0,
                g=np.array([0.0, -g, 0.0]), tool=np.zeros(3),
                sph_link=np.zeros(0, np.int32), sph=np.zeros((0, 4)))


@pytest.mark.parametrize("seed", range(6))
def test_rnea_planar_two_link_closed_form(seed):
    """Textbook planar 2-link Lagrangian dynamics."""
    rng = np.random.default_rng(seed)
    l1, l2 = rng.uniform(0.2, 0.6, 2)
    lc1, lc2 = rng.uniform(0.05, 0.3, 2)
    m1, m2 = rng.uniform(0.5, 4, 2)
    I1, I2 = rng.uniform(0.005, 0.05, 2)
    g = 9.81
    A = O.make_oarm(planar_arm(l1, l2, lc1, lc2, m1, m2, I1, I2, g), RIGID_G)
    q, qd, qdd = rng.uniform(-2, 2, (3, 2))
    c2, s2 = math.cos(q[1]), math.sin(q[1])
    M11 = I1 + I2 + m1 * lc1**2 + m2 * (l1**2 + lc2**2 + 2 * l1 * lc2 * c2)
    M12 = I2 + m2 * (lc2**2 + l1 * lc2 * c2)
    M22 = I2 + m2 * lc2**2
    h = m2 * l1 * lc2 * s2
    cor = np.array([-h * (2 * qd[0] * qd[1] + qd[1] ** 2), h * qd[0] ** 2])
    grav = np.array([(m1 * lc1 + m2 * l1) * g * math.cos(q[0]) + m2 * lc2 * g * math.cos(q[0] + q[1]),
                     m2 * lc2 * g * math.cos(q[0] + q[1])])
    ref = np.array([M11 * qdd[0] + M12 * qdd[1], M12 * qdd[0] + M22 * qdd[1]]) + cor + grav
    tau = O.rnea(A, q, qd, qdd)
    assert rel(tau, ref) <= 1e-12


@pytest.mark.parametrize("n,seed", [(2, 0), (3, 1), (3, 2), (3, 3)])
def test_rnea_matches_lagrangian_spatial(n, seed):
    """M from link Jacobians, c from Christoffel symbols of a
    central-differenced M, g from the potential: M qdd + c + g."""
    arm = kin.random_arm(n, seed)
    A = O.make_oarm(arm, RIGID_G)
    rng = np.random.default_rng(seed + 10)
    for _ in range(3):
        q, qd, qdd = rng.uniform(-2, 2, (3, n))
        ref = kin.mass_matrix(arm, q) @ qdd + kin.coriolis_vector(arm, q, qd) + kin.gravity_vector(arm, q)
        assert rel(O.rnea(A, q, qd, qdd), ref) <= 2e-7


def test_rnea_at_rest_equals_gravity_torque_7dof():
    """qd = qdd = 0: every term but gravity vanishes (friction is zero at
    zero velocity), so tau = sum_j m_j J_vj^T (-g0)."""
    arm = W.make_arm(0)
    A = O.make_oarm(arm)  # all terms on
    rng = np.random.default_rng(11)
    for _ in range(10):
        q = rng.uniform(-2.8, 2.8, 7)
        tau = O.rnea(A, q, np.zeros(7), np.zeros(7))
        assert rel(tau, kin.gravity_vector(arm, q)) <= 1e-12


def test_rnea_mass_matrix_symmetric_positive_definite_7dof():
    arm = W.make_arm(0)
    A = O.make_oarm(arm, O.T_RIGID)
    rng = np.random.default_rng(12)
    for _ in range(5):
        q = rng.uniform(-2.8, 2.8, 7)
        M = np.stack([O.rnea(A, q, np.zeros(7), e) for e in np.eye(7)], axis=1)
        assert rel(M, M.T) <= 1e-12
        assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0
        assert rel(M, kin.mass_matrix(arm, q)) <= 1e-12


def test_rnea_power_identity_along_cubic():
    """Along any trajectory, qd . tau_rigid+gravity = d(kinetic + potential)/dt."""
    arm = W.make_arm(0)
    A = O.make_oarm(arm, RIGID_G)
    rng = np.random.default_rng(13)
    x0 = rng.uniform(-1.5, 1.5, 14)
    x1 = rng.uniform(-1.5, 1.5, 14)
    T = 0.8

    def energy(t):
        s, sd, _ = O.cubic(x0, x1, T, t)
        return 0.5 * sd @ kin.mass_matrix(arm, s) @ sd + kin.potential(arm, s)

    for t in (0.1, 0.3, 0.55, 0.7):
        s, sd, sdd = O.cubic(x0, x1, T, t)
        p = sd @ O.rnea(A, s, sd, sdd)
        h = 1e-5
        dE = (energy(t + h) - energy(t - h)) / (2 * h)
        assert p == pytest.approx(dE, rel=1e-6, abs=1e-6)


def test_armature_adds_exactly_Im_qdd():
    arm = W.make_arm(0)
    Aw = O.make_oarm(arm, O.T_RIGID | O.T_GRAVITY | O.T_ARMATURE)
    Ao = O.make_oarm(arm, O.T_RIGID | O.T_GRAVITY)
    rng = np.random.default_rng(14)
    for _ in range(5):
        q, qd, qdd = rng.uniform(-2, 2, (3, 7))
        d = O.rnea(Aw, q, qd, qdd) - O.rnea(Ao, q, qd, qdd)
        assert np.max(np.abs(d - arm["Im"] * qdd)) <= 1e-12 * max(1, np.max(np.abs(O.rnea(Ao, q, qd, qdd))))


def test_friction_term_in_torque():
    arm = W.make_arm(0)
    Aw = O.make_oarm(arm, O.T_RIGID | O.T_GRAVITY | O.T_FRICTION)
    Ao = O.make_oarm(arm, O.T_RIGID | O.T_GRAVITY)
    rng = np.random.default_rng(15)
    q, qd, qdd = rng.uniform(-2, 2, (3, 7))
    d = O.rnea(Aw, q, qd, qdd) - O.rnea(Ao, q, qd, qdd)
    ref = [arm["psi1"][i] / (1 + math.exp(-arm["psi2"][i] * (qd[i] + arm["psi3"][i])))
           - arm["psi1"][i] / (1 + math.exp(-arm["psi2"][i] * arm["psi3"][i])) for i in range(7)]
    assert np.max(np.abs(d - ref)) <= 1e-12
