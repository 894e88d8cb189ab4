"""Pins of the oracle's collision model (Sec. IV-E): arm spheres against
obstacle capsules (closed-form point-segment distances, a zero-length
capsule equals a sphere, a dense chain of spheres converges to the capsule)
and the arm's self-collision pairs (against an independent forward
kinematics of the sphere centres)."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2609_22608_amd import workload as W

from . import kin


def test_point_segment_closed_forms():
    p0, p1 = [0.0, 0.0, 0.0], [1.0, 0.0, 0.0]
    assert O.point_segment([0.5, 0.3, 0.0], p0, p1) == pytest.approx(0.3, rel=1e-15)
    assert O.point_segment([-0.4, 0.3, 0.0], p0, p1) == pytest.approx(0.5, rel=1e-15)
    assert O.point_segment([1.3, 0.0, 0.4], p0, p1) == pytest.approx(0.5, rel=1e-15)
    assert O.point_segment([0.2, -0.3, 0.4], p0, p1) == pytest.approx(0.5, rel=1e-15)
    # degenerate segment: the distance to its point
    assert O.point_segment([1.0, 2.0, 2.0], [0, 0, 0], [0, 0, 0]) == pytest.approx(3.0)
    # oblique segment: distance to the line through (1,1,0) along (1,1,0)/sqrt 2
    d = O.point_segment([1.0, 0.0, 0.0], [0, 0, 0], [2, 2, 0])
    assert d == pytest.approx(math.sqrt(0.5), rel=1e-15)


def _edges(arm, n, seed):
    rng = np.random.default_rng(seed)
    return W.uniform_states(arm, n, rng), W.uniform_states(arm, n, rng)


def test_zero_length_capsule_equals_sphere_obstacle():
    arm = W.make_arm(0)
    A = O.make_oarm(arm)
    obs = W.make_obstacles(arm, 4, seed=3)
    caps = np.concatenate([obs[:, :3], obs[:, :3], obs[:, 3:]], axis=1)
    x0, x1 = _edges(arm, 6, 1)
    for e in range(6):
        a = O.rho_c(A, x0[e], x1[e], 0.6, 16, obs)
        b = O.rho_c(A, x0[e], x1[e], 0.6, 16, None, caps=caps)
        assert a == b
        # spheres and capsules together: the larger ratio
        both = O.rho_c(A, x0[e], x1[e], 0.6, 16, obs[:2], caps=caps[2:])
        assert both == max(O.rho_c(A, x0[e], x1[e], 0.6, 16, obs[:2]),
                           O.rho_c(A, x0[e], x1[e], 0.6, 16, None, caps=caps[2:]))


def test_capsule_equals_dense_chain_of_spheres():
    """A capsule of radius r over a 0.75 m segment against 20,001 spheres of
    radius r spread along the segment: the chain's distances exceed the
    segment's by at most h^2 / (8 d) (h the spacing), so the two ratios agree
    to 1e-6 relative."""
    arm = W.make_arm(0)
    A = O.make_oarm(arm)
    rng = np.random.default_rng(5)
    x0, x1 = _edges(arm, 4, 2)
    for e in range(4):
        c = rng.uniform(-0.4, 0.4, 3) + np.array([0.0, 0.0, 0.5])
        d = rng.normal(size=3)
        d *= 0.375 / np.linalg.norm(d)
        cap = np.concatenate([c - d, c + d, [0.06]])
        chain = np.concatenate([np.linspace(c - d, c + d, 20001), np.full((20001, 1), 0.06)], 1)
        a = O.rho_c(A, x0[e], x1[e], 0.5, 8, None, caps=cap[None])
        b = O.rho_c(A, x0[e], x1[e], 0.5, 8, chain)
        # the deciding distance is at least (smallest arm radius + 0.06) / a
        h = 0.75 / 20000
        dmin = (np.min(arm["sph"][:, 3]) + 0.06) / a
        assert a >= b
        assert a / b - 1 <= h * h / (8 * dmin * dmin) * (1 + 1e-6) + 1e-14


def test_self_pairs_against_independent_kinematics():
    """rho_self = max over samples and pairs of (r_a + r_b + margin) /
    |c_a - c_b| with sphere centres from homogeneous DH transforms
    written in the tests (not the oracle's recursion)."""
    arm = W.make_arm(0)
    A = O.make_oarm(arm)
    link = np.asarray(arm["sph_link"])
    pairs = np.array([(a, b) for a in range(len(link)) for b in range(a + 1, len(link))
                      if link[b] - link[a] >= 2], np.int32)
    assert len(pairs) > 300
    x0, x1 = _edges(arm, 5, 3)
    S, T, m = 8, 0.7, 0.01
    for e in range(5):
        best = 0.0
        for s in range(S):
            t = T * s / (S - 1)
            q = O.cubic(x0[e], x1[e], T, t)[0]
            Fr = kin.frames(arm, q)
            cen = np.array([Fr[link[k] - 1][:3, :3] @ arm["sph"][k][:3] + Fr[link[k] - 1][:3, 3]
                            for k in range(len(link))])
            r = arm["sph"][:, 3]
            dist = np.linalg.norm(cen[pairs[:, 0]] - cen[pairs[:, 1]], axis=1)
            best = max(best, np.max((r[pairs[:, 0]] + r[pairs[:, 1]] + m) / dist))
        assert O.rho_self(A, x0[e], x1[e], T, S, pairs, m) == pytest.approx(best, rel=1e-12)


def test_edge_check_adds_self_pairs():
    """The fixed-duration check takes the larger of the obstacle and self
    ratios; S_SELF marks a self-collision (two overlapping spheres of one
    link, a pair the offline pruning would drop, force it here)."""
    arm = W.make_arm(0)
    A = O.make_oarm(arm)
    link = np.asarray(arm["sph_link"])
    same = [(a, a + 1) for a in range(len(link) - 1) if link[a] == link[a + 1]][:1]
    far = [(0, len(link) - 1)]
    # slow rest-to-rest moves around the middle of the joint range
    rng = np.random.default_rng(4)
    q0 = rng.uniform(-1.2, 1.2, (20, 7))
    x0 = np.concatenate([q0, np.zeros((20, 7))], 1)
    x1 = np.concatenate([q0 + rng.uniform(-0.2, 0.2, (20, 7)), np.zeros((20, 7))], 1)
    T = np.full(20, 1.2)
    base = O.edge_check(A, x0, x1, T, 16)
    ok = (base["status"] & (O.S_NONE | O.S_VEL | O.S_POS)) == 0
    assert ok.sum() >= 3
    r_far = O.edge_check(A, x0, x1, T, 16, pairs=far)
    r_same = O.edge_check(A, x0, x1, T, 16, pairs=same)
    for e in np.nonzero(ok)[0]:
        rs = O.rho_self(A, x0[e], x1[e], 1.2, 16, same)
        assert rs > 1 and r_same["status"][e] & O.S_SELF and r_same["status"][e] & O.S_COLL
        assert r_same["rho"][e, 4] == max(base["rho"][e, 4], rs)
        assert r_far["rho"][e, 4] == max(base["rho"][e, 4], O.rho_self(A, x0[e], x1[e], 1.2, 16, far))
    # the self part is not evaluated where a limit check fails
    assert np.isnan(r_same["rho"][~ok, 4]).all()
    assert ((r_same["status"][~ok] & O.S_SELF) == 0).all()
