"""GPU parity of the planner's anytime outer loop (Algorithm 1) against the
FP64 oracle: the reach time of Eq. (8), Prune (keep rule, ancestor closure,
order-preserving compaction), and whole planning cycles (rounds with the
t_best bound and the incumbent, Prune after every iteration), eager and
replayed from a HIP graph.

Edge decisions are exact (near-limit ratios are decided in FP64 by the
search), and so are Prune's decisions (outcomes close to their boundary are
recomputed in FP64); the seeds are checked, on the oracle's side only, to
hold no decision within 1e-9 of a ratio limit or 1e-6 of a reach boundary.
Trees therefore match bit for bit (states and times are copies and FP32
sums); nu (max of FP32 rho_v) within 1e-5; J within 1e-4 relative; reach
times within 2 us plus their FP32 root error 1e-5 / |G'(T_n)|."""
import numpy as np
import pytest

import oracle as O
from oracle import planner as P
from paper_2609_22608_amd import workload as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2609_22608_amd import fn  # noqa: E402

V_TIP = 4.0


def _oflight(f):
    return dict(x0=np.asarray(f["x0"], float), v0=np.asarray(f["v0"], float),
                g=np.asarray(f["g"], float), t_enter=f["t_enter"], t_fall=f["t_fall"])


def _reach_bar(A, X, t, fl, blade, ref):
    """Per-node tolerance on T_n: 2 us + 1e-5 / |G'(T_n)| (the FP32 root's
    error), 0 where T_n = a (both sides return a exactly)."""
    p = O.fk_point(A, X.astype(np.float64), blade.astype(np.float64))
    bar = np.zeros(len(ref))
    for i in np.nonzero(np.isfinite(ref))[0]:
        a = max(fl["t_enter"], float(t[i]))
        if ref[i] == a:
            continue
        c = P.reach_poly(p[i], float(t[i]), fl, V_TIP)
        bar[i] = 2e-6 + 1e-5 / max(abs(np.polyval(np.polyder(c), ref[i])), 1e-12)
    return bar


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_reach_time_matches_oracle(seed):
    arm = W.make_arm(0)
    A = O.make_oarm(arm)
    rng = np.random.default_rng(seed)
    n = 3000
    X = W.uniform_states(arm, n, rng).astype(np.float32)
    t = rng.uniform(0, 0.9, n).astype(np.float32)  # some nodes start too late to reach
    f = W.make_flight(seed, launch_dist=(1.0, 1.6))
    fl = _oflight(f)
    blade = W.blade_midpoint(arm)
    ctx = fn.Context(arm, 16, 16, 4)
    tree, ld, _ = fn.tree_soa(X)
    T = ctx.reach_time(tree, ld, n, fn.dev(t), f, V_TIP, blade).cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    ref = P.reach_time(A, X, t, fl, V_TIP, blade)
    assert np.array_equal(np.isnan(T), np.isnan(ref))
    ok = np.isfinite(ref)
    err = np.abs(T - ref)[ok]
    bar = _reach_bar(A, X, t, fl, blade, ref)[ok]
    print(f"seed {seed}: {ok.sum()} of {n} nodes reach the object, max |dT| {err.max():.2e} s, "
          f"at T_n = a {int((bar == 0).sum())}")
    assert np.all(err <= bar)
    assert 0.05 * n < ok.sum() < 0.95 * n
    ctx.close()


def _forest(rng, n):
    return np.array([-1] + [int(rng.integers(-1, i)) for i in range(1, n)], np.int64)


def _prune_set(arm, seed, n_problems=3):
    """Problems with random forests, times, nu and an incumbent node and
    t_best; dummy candidates (Prune does not read them)."""
    rng = np.random.default_rng([seed, 9])
    out = []
    for p in range(n_problems):
        n = int(rng.integers(300, 3000))
        X = W.uniform_states(arm, n, rng).astype(np.float32)
        t = rng.uniform(0, 0.4, n).astype(np.float32)
        t[0] = 0.0
        f = W.make_flight(seed * 10 + p, launch_dist=(1.0, 1.6))
        inc = int(rng.integers(1, n))
        tb = np.float32(rng.uniform(f["t_enter"] + 0.05, f["t_fall"]))
        out.append(dict(X=X, t=t, parent=_forest(rng, n), nu=rng.uniform(0, 1, n).astype(np.float32),
                        flight=f, inc=inc, t_best=tb,
                        cand=W.make_candidates(arm, 16, 0.5, seed * 10 + p)))
    return out


def prune_band(A, pr, blade):
    """Nodes whose keep decision lies within 1e-6 of its boundary (the
    oracle's slack of Eq. (8) or the reach window's width), the incumbent
    excepted."""
    fl = _oflight(pr["flight"])
    g, w = P.reach_slack(A, pr["X"], pr["t"], fl, V_TIP, W.blade_midpoint(pr["arm"]), pr["t_best"])
    band = (np.abs(g) <= 1e-6) | (np.abs(w) <= 1e-6)
    band[pr["inc"]] = False
    return band


@pytest.mark.parametrize("seed", [5, 7])
def test_prune_matches_oracle(seed):
    arm = W.make_arm(0)
    A = O.make_oarm(arm)
    blade = W.blade_midpoint(arm)
    probs = _prune_set(arm, seed)
    ctx = fn.Context(arm, 4096, 64, 8, max_edges=512, max_problems=len(probs))
    bt = fn.Batch(ctx, fn.dev(W.t_grid(32, 0.02, 1.0)), 16, 8)
    for pr in probs:
        pr["arm"] = arm
        assert not prune_band(A, pr, blade).any()
        P_ = bt.add_problem(pr["X"], pr["t"], pr["cand"], np.zeros((0, 4), np.float32),
                            capacity=len(pr["X"]) + 8, flight=pr["flight"], parent=pr["parent"])
        P_["nu"][:len(pr["X"])] = torch.as_tensor(pr["nu"], device="cuda")
        P_["incumbent"].copy_(torch.tensor([1.0, float(pr["inc"]), float(pr["t_best"]), 0.0]))
    bt.prepare()
    bt.prune(V_TIP, blade)
    torch.cuda.synchronize()
    for i, (pr, G) in enumerate(zip(probs, bt.problems)):
        n = len(pr["X"])
        st = P.new_state(pr["X"], pr["t"], G["ld"], _oflight(pr["flight"]), parent=pr["parent"])
        st["nu"][:n] = pr["nu"]
        st["node"], st["t_best"], st["J"] = pr["inc"], pr["t_best"], 1.0
        T, keep, nm = P.prune_step(A, st, _oflight(pr["flight"]), V_TIP, blade)
        m = st["n"]
        assert int(G["n_nodes"].item()) == m, i
        tree = G["tree"].cpu().numpy()
        assert np.array_equal(tree[:, :m].T, st["X"][:m]), i
        assert np.array_equal(G["t_node"].cpu().numpy()[:m], st["t"][:m]), i
        assert np.array_equal(G["nu"].cpu().numpy()[:m], st["nu"][:m]), i
        par = G["parent"].cpu().numpy()
        assert np.array_equal(par[:m], st["parent"][:m]), i
        assert np.all(par[m:n] == -1), i
        inc = G["incumbent"].cpu().numpy()
        assert int(inc[1]) == st["node"], i
        R = G["out_reach"].cpu().numpy()[:n].astype(np.float64)
        assert np.array_equal(np.isnan(R), np.isnan(T)), i
        ok = np.isfinite(T)
        assert np.all(np.abs(R - T)[ok] <= _reach_bar(A, pr["X"], pr["t"], _oflight(pr["flight"]),
                                                       blade, T)[ok]), i
        print(f"problem {i}: {n} nodes, {m} kept ({int(ok.sum())} reach the object)")
        assert 0 < m < n
    ctx.close()


CYCLE_SEEDS = (0, 3, 4)


def cycle_set(arm):
    return [W.make_cycle_problem(arm, s, 400 + 150 * (s % 3), 160) for s in CYCLE_SEEDS]


def build_cycle(arm, probs, capacity_extra=700, edge_form=0):
    k = probs[0]["k"]
    B = len(probs[0]["rounds"][0]["x"])
    ctx = fn.Context(arm, 4096, B * len(probs), k, max_edges=B * k * len(probs),
                     max_problems=len(probs))
    ctx.set_tuning(edge_form=edge_form)
    bt = fn.Batch(ctx, fn.dev(probs[0]["grid"]), probs[0]["samples"], k)
    for c in probs:
        bt.add_problem(c["tree_x"], c["tree_t"], c["rounds"], c["obs"],
                       capacity=len(c["tree_x"]) + capacity_extra, flight=c["flight"])
    bt.prepare()
    return ctx, bt


def oracle_cycle(arm, c, ld, n_iter=2, n_round=2):
    A = O.make_oarm(arm)
    R = O.make_orisk(sigma_mode=1)
    fl = _oflight(c["flight"])
    st = P.new_state(c["tree_x"], c["tree_t"], ld, fl)
    log = P.cycle(A, st, c["rounds"], n_iter, n_round, c["k"], c["grid"], c["samples"], R, fl,
                  V_TIP, W.blade_midpoint(arm), obs=c["obs"])
    return st, log


def snapshot(bt):
    return [{key: P_[key].clone() for key in ("tree", "t_node", "parent", "nu", "n_nodes",
                                              "incumbent", "out_reach")} for P_ in bt.problems]


@pytest.mark.parametrize("edge_form", [0, 3])
def test_cycle_matches_oracle(edge_form):
    """Two anytime iterations of two rounds on three problems: final trees,
    incumbents and the last Prune's reach times against the oracle's cycle;
    with the one-kernel and the ordered two-phase search (its triage bounds
    the free edges by t_best like the search)."""
    arm = W.make_arm(0)
    probs = cycle_set(arm)
    ctx, bt = build_cycle(arm, probs, edge_form=edge_form)
    bt.cycle(2, 2, V_TIP, W.blade_midpoint(arm))
    torch.cuda.synchronize()
    A = O.make_oarm(arm)
    for i, (c, G) in enumerate(zip(probs, bt.problems)):
        st, log = oracle_cycle(arm, c, G["ld"])
        m = st["n"]
        assert int(G["n_nodes"].item()) == m, i
        assert np.array_equal(G["tree"].cpu().numpy()[:, :m].T, st["X"][:m]), i
        assert np.array_equal(G["t_node"].cpu().numpy()[:m], st["t"][:m]), i
        assert np.array_equal(G["parent"].cpu().numpy()[:m], st["parent"][:m]), i
        assert np.allclose(G["nu"].cpu().numpy()[:m], st["nu"][:m], rtol=0, atol=1e-5), i
        inc = G["incumbent"].cpu().numpy()
        assert int(inc[1]) == st["node"] and inc[2] == st["t_best"] and inc[3] == 4, i
        assert abs(inc[0] - st["J"]) <= 1e-4 * max(1.0, abs(st["J"])), i
        T_last = log[-1][1][0]
        R = G["out_reach"].cpu().numpy()[:len(T_last)].astype(np.float64)
        assert np.array_equal(np.isnan(R), np.isnan(T_last)), i
        n_att = sum(int((r[1]["node"] >= 0).sum()) for r in log if r[0] == "round")
        n_free = sum(int(((r[1]["node"] >= 0) & (np.asarray(c["rounds"][j]["kind"]) == 0)).sum())
                     for j, r in enumerate([r for r in log if r[0] == "round"]))
        kept = [int(r[1][1].sum()) for r in log if r[0] == "prune"]
        print(f"problem {i}: {len(c['tree_x'])} initial nodes, {n_att} attached ({n_free} free), "
              f"kept after prunes {kept}, J* {st['J']:.4f} at t_best {st['t_best']:.4f}")
        assert n_att >= 10 and n_free >= 3
    ctx.close()


@pytest.mark.parametrize("edge_form", [0, 3])
def test_cycle_graph_replay_equals_eager(edge_form):
    """The whole cycle captured as one HIP graph: three replays (trees reset
    by eager copies in between) equal the eager cycle bit for bit."""
    arm = W.make_arm(0)
    probs = cycle_set(arm)[:2]
    ctx, bt = build_cycle(arm, probs, edge_form=edge_form)
    blade = W.blade_midpoint(arm)
    bt.cycle(2, 2, V_TIP, blade)
    torch.cuda.synchronize()
    ref = snapshot(bt)
    s = torch.cuda.Stream()
    bt.reset_trees()
    torch.cuda.synchronize()
    bt.capture_cycle(s, 2, 2, V_TIP, blade)
    for rep in range(3):
        bt.reset_trees()
        torch.cuda.synchronize()
        bt.replay()
        torch.cuda.synchronize()
        got = snapshot(bt)
        for a, b in zip(ref, got):
            for key in a:
                x, y = a[key], b[key]
                if x.dtype == torch.float32:
                    x, y = x.view(torch.int32), y.view(torch.int32)
                assert torch.equal(x, y), (rep, key)
    ctx.close()


def test_cycle_arguments_are_validated():
    arm = W.make_arm(0)
    probs = cycle_set(arm)[:1]
    ctx, bt = build_cycle(arm, probs)
    blade = W.blade_midpoint(arm)
    with pytest.raises(fn.FnError, match="rounds"):
        bt.cycle(3, 2, V_TIP, blade)  # 6 > 4 prepared rounds
    with pytest.raises(fn.FnError, match="V_tip"):
        bt.cycle(1, 1, 0.0, blade)
    with pytest.raises(fn.FnError, match="round"):
        bt.round(4)
    ctx.close()
    # no incumbent: no cycle
    c = probs[0]
    ctx = fn.Context(arm, 4096, 160, 8, max_edges=1280, max_problems=1)
    bt = fn.Batch(ctx, fn.dev(c["grid"]), c["samples"], 8)
    bt.add_problem(c["tree_x"], c["tree_t"], c["rounds"], c["obs"], capacity=len(c["tree_x"]) + 8)
    bt.prepare()
    with pytest.raises(fn.FnError, match="incumbent"):
        bt.cycle(1, 1, V_TIP, blade)
    ctx.close()
