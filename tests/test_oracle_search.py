"""Pins of the oracle's limit ratios (Def. 6 / Eq. 7), minimum-time search
(Def. 7) and post-checks against closed forms and brute force."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2609_22608_amd import workload as W


def one_dof_arm(m=2.0, r=0.3, izz=0.05, taumax=20.0, wmax=40.0, qdmax=2.5, acc=10.0):
    """One revolute joint about z, no gravity: tau = (Izz + m r^2) qdd."""
    return dict(n=1, alpha=np.zeros(1), a=np.zeros(1), d=np.zeros(1), m=np.array([m]),
                rc=np.array([[r, 0, 0.0]]), I=np.array([[0.02, 0.03, izz]]), Im=np.zeros(1),
                psi1=np.zeros(1), psi2=np.ones(1), psi3=np.zeros(1), qmin=np.array([-2.8]),
                qmax=np.array([2.8]), qdmax=np.array([qdmax]), taumax=np.array([taumax]),
                acc=np.array([acc]), wmax=wmax, g=np.zeros(3), tool=np.zeros(3),
                sph_link=np.zeros(0, np.int32), sph=np.zeros((0, 4)))


def test_one_dof_rest_to_rest_closed_form():
    """Rest-to-rest: sigma'' = 6 dq (1 - 2u)/T^2, so the peak torque
    6 I |dq| / T^2 sits at the (sampled) endpoints, and the power is
    36 I dq^2 (1-2u)(u-u^2)/T^3.  Expected j* from these closed forms."""
    arm = one_dof_arm()
    A = O.make_oarm(arm, O.T_RIGID)
    I = 0.05 + 2.0 * 0.3**2
    S = 16
    grid = W.t_grid(32, 0.02, 1.0)
    u = np.arange(S) / (S - 1)
    kappa = np.max(np.abs((1 - 2 * u) * (u - u * u)))
    checked = 0
    for dq in np.linspace(0.05, 2.5, 40):
        rho_t = 6 * I * dq / grid**2 / 20.0
        rho_p = 36 * I * dq * dq * kappa / grid**3 / 40.0
        rho = np.maximum(rho_t, rho_p)
        if np.min(np.abs(rho - 1)) < 1e-6:
            continue  # keep away from slot boundaries
        feas = np.nonzero(rho <= 1)[0]
        expect = feas[0] if len(feas) else -1
        x0 = np.array([0.1, 0.0])
        x1 = np.array([0.1 + dq, 0.0])
        r = O.edge_time(A, x0[None], x1[None], grid, S, scan=0)
        assert r["j"][0] == expect
        if expect >= 0:
            assert r["rho"][0, 0] == pytest.approx(rho[expect], rel=1e-12)
            T = grid[expect]
            # peak speed 1.5 dq / T at u = 1/2, where sigma = q0 + dq/2
            qm = 0.1 + dq / 2
            lim = min(2.5, math.sqrt(2 * 10.0 * (2.8 - qm)))
            assert r["rho"][0, 1] == pytest.approx(1.5 * dq / T / lim, rel=1e-12)
            # monotone path: extrema at the endpoints
            assert r["rho"][0, 2] == pytest.approx((0.1 + dq) / 2.8, rel=1e-12)
            checked += 1
        else:
            assert r["status"][0] & O.S_NONE
        # margin = min |rho_j - 1| over slots up to j*
        upto = rho[: (expect + 1 if expect >= 0 else len(rho))]
        m_exp = np.min(np.abs(upto - 1))
        if expect >= 0:
            m_exp = min(m_exp, abs(r["rho"][0, 1] - 1), abs(r["rho"][0, 2] - 1), 1.0)
        assert r["margin"][0] == pytest.approx(m_exp, rel=1e-9)
    assert checked > 10


def test_position_overshoot_closed_form():
    """q0 = q1 = 0, qd0 = v, qd1 = -v: sigma = v t - v t^2 / T, maximum v T / 4."""
    A = O.make_oarm(one_dof_arm(), O.T_RIGID)
    for v, T in ((1.0, 0.5), (2.0, 1.2), (-1.5, 0.8)):
        x0 = np.array([0.0, v])
        x1 = np.array([0.0, -v])
        assert O.rho_q(A, x0, x1, T) == pytest.approx(abs(v) * T / 4 / 2.8, rel=1e-12)


def test_velocity_peak_against_brute_force():
    """rho_v at the exact extremum equals a fine sampling of |sigma'|/taper
    wherever the peak ratio sits at a peak of |sigma'| (taper flat there)."""
    arm = W.make_arm(0)
    A = O.make_oarm(arm)
    rng = np.random.default_rng(5)
    checked = 0
    for _ in range(200):
        x0 = W.uniform_states(arm, 1, rng)[0]
        x1 = W.uniform_states(arm, 1, rng)[0]
        T = rng.uniform(0.3, 1.5)
        ts = np.linspace(0, T, 2001)
        s_all = np.stack([O.cubic(x0, x1, T, t)[1] for t in ts])
        peak_samp = np.max(np.abs(s_all), axis=0)
        # exact peaks of |sd| per joint are at 0, T or the vertex
        for i in range(7):
            c2 = 3 * (x1[i] - x0[i] - x0[7 + i] * T) / T**2 - (x1[7 + i] - x0[7 + i]) / T
            c3 = (x1[7 + i] - x0[7 + i]) / T**2 - 2 * (x1[i] - x0[i] - x0[7 + i] * T) / T**3
            cand = [abs(x0[7 + i]), abs(x1[7 + i])]
            if c3 != 0 and 0 < -c2 / (3 * c3) < T:
                tv = -c2 / (3 * c3)
                cand.append(abs(x0[7 + i] + 2 * c2 * tv + 3 * c3 * tv * tv))
            assert max(cand) >= peak_samp[i] - 1e-12
            assert max(cand) == pytest.approx(peak_samp[i], rel=1e-4, abs=1e-9)
            checked += 1
    assert checked == 1400


def test_taper_braking_law():
    """Moving toward a limit the allowed speed is sqrt(2 a dist) (capped)."""
    A = O.make_oarm(one_dof_arm(qdmax=2.5, acc=10.0), O.T_RIGID)
    # stationary cubic at position q with velocity v: x0 = x1 = (q, v) gives a
    # path whose velocity at t = 0 is v
    for q, v in ((2.7, 1.0), (2.7, -1.0), (-2.75, -0.5), (0.0, 2.0), (2.8, 0.1)):
        x0 = np.array([q, v])
        x1 = np.array([q + v * 1e-9, v])
        dist = (2.8 - q) if v >= 0 else (q + 2.8)
        lim = min(2.5, math.sqrt(2 * 10 * max(0.0, dist)))
        expect = abs(v) / lim if lim > 0 else math.inf
        got = O.rho_v(A, x0, x1, 1e-9)
        assert got == pytest.approx(expect, rel=1e-6)


def test_dense_equals_scan_tiny_workload():
    """The ascending scan with early exit equals the dense definition."""
    sh = W.CONFIGS["tiny"]
    wl = W.make_workload(sh, seed=1)
    A = O.make_oarm(wl["arm"])
    idx, _ = O.plan_knn(wl["tree_x"], wl["cand"]["x"], sh.k)
    x0, x1, ok = O.edges_of(wl["tree_x"], wl["cand"]["x"], idx)
    a = O.edge_time(A, x0, x1, wl["grid"], sh.samples, scan=0)
    b = O.edge_time(A, x0, x1, wl["grid"], sh.samples, scan=1)
    for key in ("j", "status", "margin", "rho"):
        # rho_c is NaN where the limit checks fail (the clearance is not evaluated)
        assert np.array_equal(a[key], b[key], equal_nan=key == "rho"), key
    assert b["nslots"].sum() <= a["nslots"].sum()
    # first-feasible definition against the dense rho table
    dense = O.edge_dense(A, x0, x1, wl["grid"], sh.samples).max(axis=2)
    for e in range(len(x0)):
        f = np.nonzero(dense[e] <= 1.0)[0]
        assert a["j"][e] == (f[0] if len(f) else -1)


def test_nary_equals_dense_on_monotone_edges():
    sh = W.CONFIGS["tiny"]
    wl = W.make_workload(sh, seed=2)
    A = O.make_oarm(wl["arm"])
    idx, _ = O.plan_knn(wl["tree_x"], wl["cand"]["x"][:32], sh.k)
    x0, x1, _ = O.edges_of(wl["tree_x"], wl["cand"]["x"][:32], idx)
    dense = O.edge_dense(A, x0, x1, wl["grid"], sh.samples).max(axis=2) <= 1.0
    ref = O.edge_time(A, x0, x1, wl["grid"], sh.samples, scan=0)["j"]
    for N in (4, 8):
        nary = O.edge_nary(A, x0, x1, wl["grid"], sh.samples, N)
        mono = np.array([not (np.diff(d.astype(int)) < 0).any() for d in dense])
        assert mono.sum() > 0.9 * len(mono)
        assert np.array_equal(nary[mono], ref[mono])


def test_jmax_bound_and_bad_input():
    sh = W.CONFIGS["tiny"]
    wl = W.make_workload(sh, seed=1)
    A = O.make_oarm(wl["arm"])
    idx, _ = O.plan_knn(wl["tree_x"], wl["cand"]["x"], sh.k)
    x0, x1, _ = O.edges_of(wl["tree_x"], wl["cand"]["x"], idx)
    r = O.edge_time(A, x0, x1, wl["grid"], sh.samples)
    e = int(np.nonzero(r["j"] > 0)[0][0])
    j = int(r["j"][e])
    rj = O.edge_time(A, x0[e:e + 1], x1[e:e + 1], wl["grid"], sh.samples, jmax=[j])
    assert rj["j"][0] == j
    rj = O.edge_time(A, x0[e:e + 1], x1[e:e + 1], wl["grid"], sh.samples, jmax=[j - 1])
    assert rj["j"][0] == -1 and rj["status"][0] & O.S_NONE
    bad = x1[:2].copy()
    bad[0, 3] = np.nan
    rb = O.edge_time(A, x0[:2], bad, wl["grid"], sh.samples)
    assert rb["status"][0] == O.S_BAD and rb["j"][0] == -1
    assert rb["status"][1] == r["status"][1] and rb["j"][1] == r["j"][1]
    rp = O.edge_time(A, x0[:2], x1[:2], wl["grid"], sh.samples, parent_ok=[0, 1])
    assert rp["status"][0] == O.S_NOPARENT and rp["j"][0] == -1


def test_edge_check_matches_slot_and_post_checks():
    sh = W.CONFIGS["iteration"]
    wl = W.make_workload(sh, seed=3)
    A = O.make_oarm(wl["arm"])
    idx, _ = O.plan_knn(wl["tree_x"], wl["cand"]["x"][:8], sh.k)
    x0, x1, _ = O.edges_of(wl["tree_x"], wl["cand"]["x"][:8], idx)
    T = np.linspace(0.3, 1.0, len(x0))
    T[0] = -0.1
    r = O.edge_check(A, x0, x1, T, sh.samples, wl["obs"], want_tau=True)
    assert r["status"][0] == O.S_NONE
    for e in range(1, len(x0)):
        rt, rp, tau = O.slot_rho(A, x0[e], x1[e], T[e], sh.samples, want_tau=True)
        assert r["rho"][e, 0] == rt and r["rho"][e, 1] == rp
        assert np.array_equal(r["tau"][e], tau)
        assert r["rho"][e, 2] == O.rho_v(A, x0[e], x1[e], T[e])
        # clearance only after every limit check passed (Alg. 1), else NaN
        if np.all(r["rho"][e, :4] <= 1.0):
            assert r["rho"][e, 4] == O.rho_c(A, x0[e], x1[e], T[e], sh.samples, wl["obs"])
        else:
            assert np.isnan(r["rho"][e, 4]) and not r["status"][e] & O.S_COLL
        # the stored torques are the samples of Eq. (4) along the cubic
        u = 7 / (sh.samples - 1)
        s, sd, sdd = O.cubic(x0[e], x1[e], T[e], u * T[e])
        assert np.array_equal(tau[7], O.rnea(A, s, sd, sdd))
