"""Pins of the oracle's multi-round N-ary refinement of the minimum feasible
time below the grid (Sec. IV-D, the N-ary search after Def. 7): closed forms
on a one-joint arm, the search's invariants and a brute-force scan on the
7-DOF arm."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2609_22608_amd import workload as W

from .test_oracle_search import one_dof_arm


@pytest.mark.parametrize("N", [2, 3, 5, 8])
def test_one_dof_rest_to_rest_continuous_minimum(N):
    """Rest-to-rest on one joint without gravity or friction: the peak torque
    6 I |dq| / T^2 sits at the sampled endpoints, so the minimum feasible
    time is T*_tau = sqrt(6 I |dq| / taumax) when power does not bind
    (W_max large), and T*_P = (36 I dq^2 kappa_S / W_max)^(1/3) when it
    does, kappa_S = max over the samples of |(1 - 2u)(u - u^2)|.  The refined
    T lies in [T*, T* + eps] and the round count is ceil(log_N(w0 / eps))."""
    S, eps = 16, 1e-6
    I = 0.05 + 2.0 * 0.3**2
    u = np.arange(S) / (S - 1)
    kappa = np.max(np.abs((1 - 2 * u) * (u - u * u)))
    grid = W.t_grid(32, 0.02, 1.0)
    checked = 0
    for wmax, binding in ((1e9, "torque"), (2.0, "power")):
        A = O.make_oarm(one_dof_arm(wmax=wmax), O.T_RIGID)
        for dq in np.linspace(0.05, 2.5, 25):
            t_tau = math.sqrt(6 * I * dq / 20.0)
            t_p = (36 * I * dq * dq * kappa / wmax) ** (1.0 / 3.0)
            t_star = max(t_tau, t_p)
            if not (grid[0] < t_star <= grid[-1]):
                continue
            assert (t_p > t_tau) == (binding == "power")
            j = int(np.nonzero(grid >= t_star)[0][0])
            x0 = np.array([[0.1, 0.0]])
            x1 = np.array([[0.1 + dq, 0.0]])
            r = O.edge_refine(A, x0, x1, [j], grid, S, N, eps)
            T = r["T"][0]
            assert t_star * (1 - 1e-12) <= T <= t_star + eps * (1 + 1e-9), (dq, T, t_star)
            w0 = grid[j] - grid[j - 1]
            assert r["rounds"][0] == math.ceil(math.log(w0 / eps) / math.log(N) - 1e-12)
            assert r["T"][0] - r["lo"][0] <= eps
            checked += 1
    assert checked > 30


def test_refinement_invariants_on_the_7dof_arm():
    """Tiny workload, every feasible edge: the refined T lies in
    (grid[j-1], grid[j]], is feasible, the final lower end is infeasible (or
    the grid point below, infeasible by the grid search) and within eps."""
    sh = W.CONFIGS["tiny"]
    wl = W.make_workload(sh, seed=1)
    A = O.make_oarm(wl["arm"])
    idx, _ = O.plan_knn(wl["tree_x"], wl["cand"]["x"], sh.k)
    x0, x1, ok = O.edges_of(wl["tree_x"], wl["cand"]["x"], idx)
    g = O.edge_time(A, x0, x1, wl["grid"], sh.samples, parent_ok=ok)
    f = np.nonzero(g["j"] >= 0)[0]
    assert len(f) > 50
    eps = 1e-4
    r = O.edge_refine(A, x0[f], x1[f], g["j"][f], wl["grid"], sh.samples, 4, eps)
    grid = wl["grid"]
    for i, e in enumerate(f):
        j = g["j"][e]
        T, lo = r["T"][i], r["lo"][i]
        assert (grid[j - 1] if j > 0 else 0.0) <= lo < T <= grid[j]
        assert T - lo <= eps
        assert max(O.slot_rho(A, x0[e], x1[e], T, sh.samples)) <= 1.0
        assert r["rho"][i, 0] == max(O.slot_rho(A, x0[e], x1[e], T, sh.samples))
        if lo > 0:
            assert max(O.slot_rho(A, x0[e], x1[e], lo, sh.samples)) > 1.0
        # post-checks at the refined duration
        assert r["rho"][i, 1] == O.rho_v(A, x0[e], x1[e], T)
        assert r["rho"][i, 2] == O.rho_q(A, x0[e], x1[e], T)
        st = (O.S_VEL if r["rho"][i, 1] > 1 else 0) | (O.S_POS if r["rho"][i, 2] > 1 else 0)
        assert r["status"][i] == st
    # edges without a feasible slot are not refined
    nf = np.nonzero(g["j"] < 0)[0][:5]
    rn = O.edge_refine(A, x0[nf], x1[nf], g["j"][nf], wl["grid"], sh.samples, 4, eps)
    assert np.isnan(rn["T"]).all() and (rn["status"] == O.S_NONE).all()


def test_refinement_equals_brute_force_where_monotone():
    """A dense scan of 4,001 durations over the grid slot below the result
    locates the first feasible one; on edges where feasibility changes once
    along that scan, the refinement agrees to eps + the scan's spacing, for
    several N."""
    sh = W.CONFIGS["tiny"]
    wl = W.make_workload(sh, seed=2)
    A = O.make_oarm(wl["arm"])
    idx, _ = O.plan_knn(wl["tree_x"], wl["cand"]["x"], sh.k)
    x0, x1, ok = O.edges_of(wl["tree_x"], wl["cand"]["x"], idx)
    g = O.edge_time(A, x0, x1, wl["grid"], sh.samples, parent_ok=ok)
    f = np.nonzero((g["j"] > 0))[0][:24]
    grid = wl["grid"]
    eps = 1e-5
    res = {N: O.edge_refine(A, x0[f], x1[f], g["j"][f], grid, sh.samples, N, eps)
           for N in (2, 3, 7)}
    checked = 0
    for i, e in enumerate(f):
        j = g["j"][e]
        ts = np.linspace(grid[j - 1], grid[j], 4001)
        feas = np.array([max(O.slot_rho(A, x0[e], x1[e], t, sh.samples)) <= 1.0 for t in ts])
        if np.count_nonzero(np.diff(feas.astype(int))) != 1:
            continue
        t_bf = ts[np.argmax(feas)]
        for N, r in res.items():
            assert abs(r["T"][i] - t_bf) <= eps + (ts[1] - ts[0]), (e, N)
        checked += 1
    assert checked >= 15
