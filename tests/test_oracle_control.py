"""Pins of the oracle's tracking-controller law (Sec. IV-F, Eq. (9)): the
desired acceleration against the Hermite-basis form of the refitted cubic,
the torque against a Lagrangian built from link Jacobians, and every clip
against closed forms on a one-joint arm."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2609_22608_amd import workload as W

from . import kin
from .test_oracle_search import one_dof_arm

BIG = 1e12


def hermite_qdd0(q, qd, qg, qdg, T):
    """Second derivative at t = 0 of the cubic Hermite interpolant through
    (q, qd) and (qg, qdg) over T: h00''(0) = -6, h10''(0) = -4, h01''(0) = 6,
    h11''(0) = -2 on the unit interval, divided by T^2."""
    return (-6 * q - 4 * T * qd + 6 * qg - 2 * T * qdg) / T**2


def friction(arm, qd):
    """Eq. (5), written out: psi1 (s(psi2 (qd + psi3)) - s(psi2 psi3)), s the logistic."""
    s = lambda x: 1.0 / (1.0 + np.exp(-x))  # noqa: E731
    return arm["psi1"] * (s(arm["psi2"] * (qd + arm["psi3"])) - s(arm["psi2"] * arm["psi3"]))


def unlimited(arm):
    a = dict(arm)
    a["taumax"] = np.full(arm["n"], BIG)
    a["wmax"] = BIG
    a["qdmax"] = np.full(arm["n"], BIG)
    a["acc"] = np.full(arm["n"], BIG)
    return a


def test_unclipped_torque_is_eq4_at_the_refit_cubics_initial_acceleration():
    base = W.make_arm(0)
    arm = unlimited(base)
    A = O.make_oarm(arm)
    rng = np.random.default_rng(7)
    for _ in range(20):
        x = W.uniform_states(base, 2, rng)
        q, qd, qg, qdg = x[0, :7], x[0, 7:], x[1, :7], x[1, 7:]
        T = rng.uniform(0.1, 0.8)
        tau, qdd, st = O.control(A, q, qd, np.zeros(7), qg, qdg, T, 1e-3, np.full(7, BIG))
        assert st[0] == 0
        assert np.allclose(qdd[0], hermite_qdd0(q, qd, qg, qdg, T), rtol=1e-12, atol=1e-12)
        a = qdd[0]
        ref = (kin.mass_matrix(arm, q) @ a + kin.coriolis_vector(arm, q, qd)
               + kin.gravity_vector(arm, q) + arm["Im"] * a + friction(arm, qd))
        assert np.allclose(tau[0], ref, rtol=2e-6, atol=2e-6 * np.abs(ref).max())


def test_at_rest_on_the_rendezvous_the_torque_is_gravity():
    base = W.make_arm(0)
    arm = unlimited(base)
    A = O.make_oarm(arm)
    rng = np.random.default_rng(8)
    for _ in range(10):
        q = W.uniform_states(base, 1, rng)[0, :7]
        tau, qdd, st = O.control(A, q, np.zeros(7), np.zeros(7), q, np.zeros(7), 0.5, 1e-3,
                                 np.full(7, BIG))
        assert st[0] == 0 and np.all(qdd[0] == 0)
        g = kin.gravity_vector(arm, q)
        assert np.allclose(tau[0], g, rtol=1e-12, atol=1e-12 * np.abs(g).max())


I1 = 0.05 + 2.0 * 0.3**2  # the one-joint arm's inertia about its axis


def one(q, qd, qg, qdg, T, dt=1e-3, tau_prev=0.0, slew=BIG, **kw):
    A = O.make_oarm(one_dof_arm(**kw), O.T_RIGID)
    tau, qdd, st = O.control(A, [q], [qd], [tau_prev], [qg], [qdg], T, dt, [slew])
    return tau[0, 0], qdd[0, 0], int(st[0])


def test_velocity_taper_clip_near_the_limit():
    # q = 2.79 moving up at 0.4 rad/s: the taper allows sqrt(2 * 10 * 0.01)
    # rad/s, so u = (0.4472... - 0.4) / dt; Eq. (9) asks for
    # 6 * 0.01 / 1e-4 - (1.6 + 0.6) / 0.01 = 380 rad/s^2
    tau, qdd, st = one(2.79, 0.4, 2.8, 0.3, 0.01, taumax=BIG, wmax=BIG)
    u = (math.sqrt(2 * 10.0 * 0.01) - 0.4) / 1e-3
    assert st == O.C_ACC and qdd == pytest.approx(u, rel=1e-12)
    assert tau == pytest.approx(I1 * u, rel=1e-12)
    # the lower bound, moving down toward -2.8
    tau, qdd, st = one(-2.78, -0.5, -2.9, 0.0, 0.05, taumax=BIG, wmax=BIG)
    lo = (-math.sqrt(2 * 10.0 * 0.02) + 0.5) / 1e-3
    assert st == O.C_ACC and qdd == pytest.approx(lo, rel=1e-12)
    # away from the limits and within the speed limit: no clip
    tau, qdd, st = one(0.0, 0.1, 0.05, 0.0, 0.5, taumax=BIG, wmax=BIG)
    assert st == 0 and qdd == pytest.approx(6 * 0.05 / 0.25 - 0.4 / 0.5, rel=1e-12)


def test_slew_torque_and_power_clips():
    # slew: wanted I * qdd, allowed tau_prev +- slew dt
    tau, qdd, st = one(0.0, 0.0, 0.3, 0.0, 0.5, tau_prev=0.2, slew=50.0, taumax=BIG, wmax=BIG)
    want = I1 * 6 * 0.3 / 0.25
    assert want > 0.25 and st == O.C_SLEW and tau == pytest.approx(0.2 + 50.0 * 1e-3, rel=1e-12)
    # torque limit after the slew clip
    tau, qdd, st = one(0.0, 0.0, 1.0, 0.0, 0.1, tau_prev=19.99, slew=1e6, taumax=20.0, wmax=BIG)
    assert st == O.C_TORQUE and tau == 20.0
    # power: tau qd = 2 * 15 = 30 W > 10 W, so tau is scaled by 1 / 3
    qdd_want = 15.0 / I1
    T = 0.5
    qg = (qdd_want + (4 * 2.0) / T) * T * T / 6.0  # gives qdd_des = 15 / I1 at qd = 2, qdg = 0
    tau, qdd, st = one(0.0, 2.0, qg, 0.0, T, taumax=20.0, wmax=10.0)
    assert st == O.C_POWER and qdd == pytest.approx(qdd_want, rel=1e-12)
    assert tau == pytest.approx(15.0 * 10.0 / 30.0, rel=1e-12)


def test_bad_inputs_give_zero_torque():
    A = O.make_oarm(one_dof_arm(), O.T_RIGID)
    tau, qdd, st = O.control(A, [[0.0], [0.0], [np.nan]], [[0.0], [0.0], [0.0]],
                             [[0.0]] * 3, [[0.1]] * 3, [[0.0]] * 3, [0.0, -0.1, 0.5], 1e-3, [1.0])
    assert (st == O.C_BAD).all() and (tau == 0).all() and (qdd == 0).all()
