"""Pins of the oracle's clearance check (Sec. IV-E), nearest-node scan
(Alg. 1 Parents) and risk objective (Eqs. 2-3)."""
import math

import numpy as np
import pytest
import scipy.special

import oracle as O
from paper_2609_22608_amd import workload as W


def planar_with_spheres(l1, l2, sph):
    return dict(n=2, alpha=np.zeros(2), a=np.array([0.0, l1]), d=np.zeros(2),
                m=np.ones(2), rc=np.zeros((2, 3)), I=np.full((2, 3), 0.01), Im=np.zeros(2),
                psi1=np.zeros(2), psi2=np.ones(2), psi3=np.zeros(2), qmin=-np.ones(2) * 3,
                qmax=np.ones(2) * 3, qdmax=np.ones(2) * 3, taumax=np.ones(2) * 50,
                acc=np.ones(2) * 10, wmax=100.0, g=np.zeros(3), tool=np.zeros(3),
                sph_link=np.array([s[0] for s in sph], np.int32),
                sph=np.array([s[1:] for s in sph], float))


def test_sphere_fk_planar_closed_form():
    l1, l2 = 0.4, 0.3
    arm = planar_with_spheres(l1, l2, [(1, 0.2, 0, 0, 0.05), (2, 0.25, 0, 0, 0.05)])
    A = O.make_oarm(arm)
    rng = np.random.default_rng(0)
    for _ in range(10):
        q = rng.uniform(-3, 3, 2)
        c = O.fk_spheres(A, q)
        assert np.allclose(c[0], [0.2 * math.cos(q[0]), 0.2 * math.sin(q[0]), 0], atol=1e-14)
        assert np.allclose(c[1], [l1 * math.cos(q[0]) + 0.25 * math.cos(q[0] + q[1]),
                                  l1 * math.sin(q[0]) + 0.25 * math.sin(q[0] + q[1]), 0], atol=1e-14)


@pytest.mark.parametrize("delta,inside", [(1e-6, False), (-1e-6, True), (0.05, False), (-0.02, True)])
def test_clearance_hand_placed(delta, inside):
    """A resting arm and one obstacle at distance r_a + r_o + margin + delta
    from an arm sphere: rho_c = (r_a + r_o + margin) / distance."""
    arm = planar_with_spheres(0.4, 0.3, [(2, 0.25, 0, 0, 0.05)])
    A = O.make_oarm(arm)
    q = np.array([0.3, -0.4])
    c = O.fk_spheres(A, q)[0]
    ro, margin = 0.07, 0.01
    need = 0.05 + ro + margin
    obs = np.array([[c[0], c[1] + need + delta, c[2], ro]])
    x = np.array([q[0], q[1], 0.0, 0.0])
    r = O.rho_c(A, x, x, 0.5, 8, obs, margin)
    assert r == pytest.approx(need / (need + delta), rel=1e-9)
    assert (r > 1.0) == inside


def test_clearance_brute_force_7dof():
    sh = W.CONFIGS["iteration"]
    wl = W.make_workload(sh, seed=4)
    A = O.make_oarm(wl["arm"])
    arm = wl["arm"]
    rng = np.random.default_rng(1)
    for _ in range(4):
        x0 = W.uniform_states(arm, 1, rng)[0]
        x1 = W.uniform_states(arm, 1, rng)[0]
        T, S = 0.7, 9
        best = 0.0
        for s in range(S):
            q = O.cubic(x0, x1, T, T * s / (S - 1))[0]
            cen = O.fk_spheres(A, q)
            for a in range(len(cen)):
                for o in wl["obs"]:
                    dist = np.linalg.norm(cen[a] - o[:3])
                    best = max(best, (arm["sph"][a][3] + o[3]) / dist)
        assert O.rho_c(A, x0, x1, T, S, wl["obs"]) == pytest.approx(best, rel=1e-14)


def _seq_d2(x, Y):
    d = np.zeros(len(Y))
    for j in range(Y.shape[1]):
        t = x[j] - Y[:, j]
        d = d + t * t
    return d


@pytest.mark.parametrize("seed", range(3))
def test_knn_against_lexsort(seed):
    rng = np.random.default_rng(seed)
    nodes = W._f32(rng.uniform(-2, 2, (300, 14)))
    qs = W._f32(rng.uniform(-2, 2, (20, 14)))
    # exact ties: duplicated nodes and a query equal to a node
    nodes[17] = nodes[3]
    nodes[250] = nodes[3]
    qs[5] = nodes[3]
    qs[6] = nodes[40] + 1e-3
    nodes[41] = nodes[40]
    idx, d2 = O.plan_knn(nodes, qs, 8)
    for b in range(len(qs)):
        d = _seq_d2(qs[b], nodes)
        order = np.lexsort((np.arange(len(nodes)), d))[:8]
        assert np.array_equal(idx[b], order)
        assert np.array_equal(d2[b], d[order])
    assert list(idx[5][:3]) == [3, 17, 250] and d2[5][0] == 0.0


def test_knn_pads_when_fewer_nodes():
    nodes = np.arange(3 * 14, dtype=float).reshape(3, 14)
    idx, d2 = O.plan_knn(nodes, nodes[:1], 5)
    assert list(idx[0]) == [0, 1, 2, -1, -1]
    assert np.isinf(d2[0][3:]).all()


def _risk_py(T, v_rel, nu, vz0, t_fall, sigma, gz=-9.81, w=O.PAPER_RISK):
    sg = sigma(T)
    lpo = math.log(math.erf(w["r"] / (sg * math.sqrt(2))))
    st = sg / abs(vz0 + gz * t_fall)
    lpr = float(scipy.special.log_ndtr((t_fall - T) / st))
    lpa = -w["lam"] * (nu - w["nu0"]) * T * (1 - w["nu0"] / nu) if nu > w["nu0"] else 0.0
    return w["wv"] * min(v_rel, w["vtarget"]) + w["wp"] * lpo + w["wr"] * lpr + w["wx"] * lpa


@pytest.mark.parametrize("mode", [0, 1])
def test_risk_against_independent_evaluation(mode):
    R = O.make_orisk(sigma_mode=mode, sp=0.0054, sv=0.0406, sa=0.20, s0=0.01, s1=0.05)
    if mode == 0:
        sigma = lambda t: math.sqrt(0.0054**2 + (0.0406 * t) ** 2 + (0.5 * 0.2 * t * t) ** 2)
    else:
        sigma = lambda t: 0.01 + 0.05 * t
    rng = np.random.default_rng(mode)
    n = 200
    T = rng.uniform(0.1, 1.0, n)
    t_fall = T + rng.uniform(-0.3, 0.5, n)
    v_rel = rng.uniform(0, 12, n)
    nu = rng.uniform(0.5, 1.3, n)
    vz0 = rng.uniform(1, 6, n)
    J = O.risk_score(R, T, v_rel, nu, vz0, t_fall)
    ref = [_risk_py(T[i], v_rel[i], nu[i], vz0[i], t_fall[i], sigma) for i in range(n)]
    assert np.allclose(J, ref, rtol=1e-10, atol=1e-9)


def test_risk_special_cases():
    R = O.make_orisk(sigma_mode=1, s0=0.01, s1=0.05)
    # T = t_fall: P_inrange = 1/2; nu <= nu0: no arm penalty; tiny sigma: P_object -> 1
    J = O.risk_score(R, [0.5], [3.0], [0.8], [4.0], [0.5])[0]
    lpo = math.log(math.erf(0.09 / (0.035 * math.sqrt(2))))
    assert J == pytest.approx(0.2 * 3.0 + 8 * lpo + 8 * math.log(0.5), rel=1e-12)
    R0 = O.make_orisk(sigma_mode=1, s0=1e-6, s1=0.0)
    J0 = O.risk_score(R0, [0.5], [20.0], [0.9], [4.0], [5.0])[0]
    assert J0 == pytest.approx(0.2 * 9.0, abs=1e-9)


def test_log_phi_tail_continuity():
    for z in (-5.0, -19.999, -20.0, -20.001, -35.0, -300.0):
        assert O.log_phi(z) == pytest.approx(float(scipy.special.log_ndtr(z)), rel=1e-10)
