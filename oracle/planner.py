"""FP64 oracle of the planner's anytime outer loop (Algorithm 1, Sec. IV-D:
the incumbent, the t_best bound on free candidates and the arrival-time
pruning of Eq. (8)).

TEST INFRASTRUCTURE ONLY: the tests and the benchmark's CPU leg use it to
check the GPU library; the product package never imports it.

It composes the pinned primitives of this package -- kNN, the grid search of
Def. 7 with its post-checks, the fixed-duration check, the risk of Eq. (2) --
in the order of Algorithm 1 and adds the steps around them:

- the incumbent: after every round, the rendezvous node of largest J
  (ties: the earlier node), and t_best = its time-to-come; Algorithm 1 starts
  with t_best = t_fall;
- the bound on free candidates: only durations with t(p) + T <= t_best (the
  candidate's arrival is bounded; a node that arrives after t_best has
  T_n >= t_n > t_best and would be pruned by Eq. (8) anyway);
- Prune: Eq. (8)'s earliest reach time T_n; a node is kept when T_n exists
  and T_n <= t_best, and so are node 0 (the measured state), the incumbent
  and every ancestor of a kept node, so that what remains is a tree; kept
  nodes are compacted in their order and parents renumbered.

Values the library keeps in FP32 (node times, durations, t_best) are formed
here in float32 with the same sums, so that the bound and the attachment
see identical numbers; ratios, distances, roots and J are FP64.
"""
from __future__ import annotations

import numpy as np

from . import (S_BAD, S_COLL, S_NONE, S_NOPARENT, S_POS, S_VEL, edge_check, edge_time, edges_of,
               fk_point, plan_knn, risk_score)

FAIL = S_NONE | S_VEL | S_POS | S_COLL | S_BAD | S_NOPARENT
F32 = np.float32


def flight_at(flight, T):
    """Eq. (1): x(T) = x0 + v0 T + g T^2 / 2."""
    T = np.asarray(T, np.float64)[..., None]
    return flight["x0"] + flight["v0"] * T + 0.5 * flight["g"] * T * T


def reach_poly(p, t_n, flight, v_tip):
    """Coefficients (highest power first) of
    G(T) = |p - x(T)|^2 - V_tip^2 (T - t_n)^2; for T >= t_n, the condition of
    Eq. (8), t_n + |p - x(T)| / V_tip <= T, is G(T) <= 0."""
    c0 = np.asarray(p, np.float64) - flight["x0"]  # p - x(T) = c0 + c1 T + c2 T^2
    c1 = -np.asarray(flight["v0"], np.float64)
    c2 = -0.5 * np.asarray(flight["g"], np.float64)
    v2 = float(v_tip) ** 2
    t_n = float(t_n)
    return np.array([c2 @ c2, 2 * (c1 @ c2), c1 @ c1 + 2 * (c0 @ c2) - v2,
                     2 * (c0 @ c1) + 2 * v2 * t_n, c0 @ c0 - v2 * t_n * t_n])


def _real_roots(c, lo, hi):
    """Real roots of the polynomial c in (lo, hi], ascending."""
    c = np.trim_zeros(np.asarray(c, np.float64), "f")
    if len(c) < 2:
        return np.zeros(0)
    r = np.roots(c)
    re = r.real[np.abs(r.imag) <= 1e-7 * (1 + np.abs(r.real))]
    return np.sort(re[(re > lo) & (re <= hi)])


def reach_time(A, X, t_node, flight, v_tip, blade):
    """Eq. (8) for every node: T_n = min{T in [t_enter, t_fall] :
    t_n + |p_n - x(T)| / V_tip <= T}, NaN when no such T exists; p_n is the
    blade point `blade` of the last link at the node's configuration.

    Written out: on [a, b] = [max(t_enter, t_n), t_fall] (empty: NaN) the
    condition is G(T) <= 0; T_n = a when G(a) <= 0, else the first real root
    of the quartic G in (a, b]."""
    P = fk_point(A, np.asarray(X, np.float64), np.asarray(blade, np.float64))
    out = np.full(len(P), np.nan)
    for i, (p, tn) in enumerate(zip(P, np.asarray(t_node, np.float64))):
        a, b = max(float(flight["t_enter"]), tn), float(flight["t_fall"])
        if a > b:
            continue
        c = reach_poly(p, tn, flight, v_tip)
        if np.polyval(c, a) <= 0:
            out[i] = a
            continue
        scale = 1.0 + abs(c[-1]) + float(v_tip) ** 2 * b * b
        for r in _real_roots(c, a, b):
            if np.polyval(c, r) <= 1e-9 * scale:
                out[i] = r
                break
    return out


def reach_slack(A, X, t_node, flight, v_tip, blade, t_best):
    """Smallest G over [a, min(t_fall, t_best)] (NaN when that interval is
    empty), from the endpoints and the critical points of G: a node is kept by
    Eq. (8) exactly when this is <= 0.  Tests use its size as the distance of
    the decision from its boundary.  Also returns the interval length."""
    P = fk_point(A, np.asarray(X, np.float64), np.asarray(blade, np.float64))
    g = np.full(len(P), np.nan)
    w = np.full(len(P), np.nan)
    for i, (p, tn) in enumerate(zip(P, np.asarray(t_node, np.float64))):
        a = max(float(flight["t_enter"]), tn)
        b = min(float(flight["t_fall"]), float(t_best))
        w[i] = b - a
        if a > b:
            continue
        c = reach_poly(p, tn, flight, v_tip)
        pts = np.concatenate([[a, b], _real_roots(np.polyder(c), a, b)])
        g[i] = np.polyval(c, pts).min()
    return g, w


def prune(parent, n, T_reach, t_best, incumbent=-1):
    """Keep set of Prune (Algorithm 1) and the order-preserving renumbering.

    keep0: node 0, the incumbent, and every node with T_n <= t_best; keep:
    keep0 and every ancestor of a node in it.  node_map[i] is the new index
    of kept node i, -1 for a pruned one."""
    parent = np.asarray(parent)[:n]
    T = np.asarray(T_reach, np.float64)[:n]
    keep0 = np.isfinite(T) & (T <= float(t_best))
    keep0[0] = True
    if 0 <= incumbent < n:
        keep0[incumbent] = True
    keep = keep0.copy()
    for i in np.nonzero(keep0)[0]:
        v = int(parent[i])
        while 0 <= v < n and not keep[v]:
            keep[v] = True
            v = int(parent[v])
    node_map = np.where(keep, np.cumsum(keep) - 1, -1).astype(np.int64)
    return keep, node_map


def _slot_bound(t_par, grid32, t_best):
    """Largest slot j with t(p) + grid[j] <= t_best in FP32, -1 when none."""
    s = (t_par[:, None] + grid32[None, :]).astype(F32)
    ok = s <= F32(t_best)
    return np.where(ok.any(1), len(grid32) - 1 - np.argmax(ok[:, ::-1], axis=1), -1)


def new_state(tree_x, tree_t, ld, flight, parent=None):
    """Planner state of one problem: a tree of capacity ld with the given
    nodes, and the initial incumbent (none; t_best = t_fall)."""
    n = len(tree_x)
    X = np.zeros((ld, 14), F32)
    X[:n] = tree_x
    t = np.zeros(ld, F32)
    t[:n] = tree_t
    par = np.full(ld, -1, np.int64)
    if parent is not None:
        par[:n] = parent
    return dict(X=X, t=t, parent=par, nu=np.zeros(ld, F32), n=n, ld=ld,
                J=-np.inf, node=-1, t_best=F32(flight["t_fall"]))


def round_step(A, st, cand, k, grid, S, R, obs=None, caps=None, margin=0.0):
    """One round of Algorithm 1 for one problem, in place on the state st.

    cand: dict x [B][14], kind [B] (1 goal), t_req [B] and the goals' flights
    (flight: v_rel [B], v0 [B][3], t_fall [B]).
    Free candidates search the grid below the t_best bound; goal candidates
    are checked once at T = t_req - t(p); each candidate joins the valid
    parent of least t(p) + T (first in kNN order on ties), appended in
    candidate order up to the capacity; attached goal nodes are scored and
    the incumbent is updated.  Returns the round's per-edge and per-candidate
    results."""
    n = st["n"]
    cx = np.asarray(cand["x"], F32)
    B = len(cx)
    idx, _ = plan_knn(st["X"][:n], cx, k)
    x0, x1, ok = edges_of(st["X"][:n], cx, idx)
    flat = idx.reshape(-1)
    t_par = st["t"][np.maximum(flat, 0)]
    kind = np.repeat(np.asarray(cand["kind"]), k)
    grid32 = np.asarray(grid, F32)
    jb = _slot_bound(t_par, grid32, st["t_best"])
    free = edge_time(A, x0, x1, grid, S, obs, jmax=jb, parent_ok=ok, margin=margin, caps=caps)
    Tg = (np.repeat(np.asarray(cand["t_req"], F32), k) - t_par).astype(F32)
    goal = edge_check(A, x0, x1, np.maximum(Tg, 1e-3).astype(np.float64), S, obs, margin=margin,
                      caps=caps)
    g_st = goal["status"].astype(np.int64)
    g_ok = (ok > 0) & (Tg > 0) & ((g_st & FAIL) == 0)
    f_ok = (free["j"] >= 0) & ((free["status"].astype(np.int64) & FAIL) == 0)
    valid = np.where(kind == 1, g_ok, f_ok)
    T = np.where(kind == 1, Tg, grid32[np.maximum(free["j"], 0)]).astype(F32)
    rv = np.where(kind == 1, goal["rho"][:, 2], free["rho"][:, 1])
    cost = np.where(valid, (t_par + T).astype(F32), F32(np.inf)).reshape(B, k)
    pick = np.argmin(cost, axis=1)
    has = np.isfinite(cost.min(axis=1))
    node = np.full(B, -1, np.int64)
    J = np.full(B, -np.inf)
    best, best_node = -np.inf, -1
    pos = n
    for b in np.nonzero(has)[0]:
        if pos >= st["ld"]:
            break
        e = b * k + pick[b]
        par = int(flat[e])
        st["X"][pos] = cx[b]
        st["t"][pos] = cost[b, pick[b]]
        st["parent"][pos] = par
        st["nu"][pos] = F32(max(float(st["nu"][par]), float(rv[e])))
        node[b] = pos
        if cand["kind"][b] == 1:
            fl = cand["flight"]
            J[b] = risk_score(R, [float(st["t"][pos])], [fl["v_rel"][b]], [float(st["nu"][pos])],
                              [fl["v0"][b][2]], [fl["t_fall"][b]])[0]
            if J[b] > best:
                best, best_node = J[b], pos
        pos += 1
    st["n"] = pos
    if best > st["J"]:
        st["J"], st["node"], st["t_best"] = best, best_node, F32(st["t"][best_node])
    return dict(idx=idx, jb=jb, free=free, goal=goal, kind=kind, valid=valid, T=T, node=node, J=J,
                best=best, best_node=best_node, strict=_strict(kind, free, goal, ok, Tg))


def _strict(kind, free, goal, ok, Tg):
    """Edges whose decision lies outside the 1e-3 band of every deciding
    ratio (inside it the GPU may take either side)."""
    g_far = np.all((np.abs(goal["rho"][:, :4] - 1) > 1e-3) | np.isnan(goal["rho"][:, :4]), axis=1)
    return np.where(kind == 1, (ok == 0) | (Tg <= 0) | g_far, free["margin"] > 1e-3)


def prune_step(A, st, flight, v_tip, blade):
    """Prune (Algorithm 1) in place; returns (T_reach, keep, node_map)."""
    n = st["n"]
    T = reach_time(A, st["X"][:n], st["t"][:n], flight, v_tip, blade)
    keep, nm = prune(st["parent"], n, T, st["t_best"], st["node"])
    kept = np.nonzero(keep)[0]
    m = len(kept)
    par = st["parent"][kept]
    st["X"][:m] = st["X"][kept]
    st["t"][:m] = st["t"][kept]
    st["nu"][:m] = st["nu"][kept]
    st["parent"][:m] = np.where(par >= 0, nm[np.maximum(par, 0)], -1)
    st["parent"][m:n] = -1
    st["n"] = m
    if st["node"] >= 0:
        st["node"] = int(nm[st["node"]])
    return T, keep, nm


def cycle(A, st, rounds, n_iter, n_round, k, grid, S, R, flight, v_tip, blade, obs=None,
          caps=None, margin=0.0):
    """One planning cycle: n_iter anytime iterations of n_round rounds, round
    a * n_round + r drawing its candidates from rounds[a * n_round + r], with
    Prune after every iteration.  Returns the per-round and per-prune
    records."""
    log = []
    for a in range(n_iter):
        for r in range(n_round):
            log.append(("round", round_step(A, st, rounds[a * n_round + r], k, grid, S, R, obs,
                                            caps, margin)))
        log.append(("prune", prune_step(A, st, flight, v_tip, blade)))
    return log
