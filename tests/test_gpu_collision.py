"""GPU parity of the collision model (Sec. IV-E) against the FP64 oracle:
obstacle capsules in the edge search (plain and screened) and in the
refinement, and the full-resolution fixed-duration check (S above the
search's 64 samples) with spheres, capsules and the arm's self-collision
pairs.  Bars as for the search: decisions bit-exact on every edge whose
oracle margin exceeds 1e-3 (or whose ratios all lie outside 1e-3 of 1), ratios
within 1e-4 relative."""
import numpy as np
import pytest

import oracle as O
from paper_2609_22608_amd import workload as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2609_22608_amd import fn  # noqa: E402

from .test_gpu_parity import compare_edges  # noqa: E402


@pytest.mark.parametrize("mode", [fn.SEARCH_PLAIN, fn.SEARCH_SCREEN])
def test_search_with_capsules_sampled(mode):
    """One-iteration shape with its 5 obstacle spheres plus 5 capsules of
    0.75 m; 384 sampled edges against the oracle."""
    wl = W.make_workload(W.CONFIGS["iteration"], seed=103)
    sh = wl["shape"]
    caps = W.make_capsules(wl["arm"], 5, seed=103)
    ctx = fn.Context(wl["arm"], sh.n_nodes, sh.batch, sh.k)
    tree, ld, n = fn.tree_soa(wl["tree_x"])
    cand = fn.dev(wl["cand"]["x"])
    idx, _ = ctx.plan_knn(tree, ld, n, cand, sh.k)
    out = ctx.edge_time_batch(tree, ld, n, cand, idx, fn.dev(wl["grid"]), sh.samples,
                              fn.dev(wl["obs"]), mode=mode, caps=fn.dev(caps))
    base = ctx.edge_time_batch(tree, ld, n, cand, idx, fn.dev(wl["grid"]), sh.samples,
                               fn.dev(wl["obs"]), mode=mode)
    torch.cuda.synchronize()
    nbr = idx.cpu().numpy()
    sel = np.random.default_rng(11 + mode).choice(nbr.size, 384, replace=False)
    x0, x1, ok = O.edges_of(wl["tree_x"], wl["cand"]["x"], nbr)
    A = O.make_oarm(wl["arm"])
    ref = O.edge_time(A, x0[sel], x1[sel], wl["grid"], sh.samples, wl["obs"], parent_ok=ok[sel],
                      caps=caps)
    compare_edges(out, ref, sel, label=f"capsules mode {mode}")
    more = ((out["status"] & fn.S_COLL) > 0).sum().item()
    less = ((base["status"] & fn.S_COLL) > 0).sum().item()
    print(f"colliding edges: {less} with spheres, {more} with spheres and capsules")
    assert more > less
    ctx.close()


def test_refine_with_capsules():
    """Refinement at the one-iteration shape with its obstacle spheres and 8
    capsules: 48 sampled candidates (384 edges) against the oracle, started
    from the oracle's grid slots; collisions occur at the refined duration."""
    wl = W.make_workload(W.CONFIGS["iteration"], seed=101)
    sh = wl["shape"]
    caps = W.make_capsules(wl["arm"], 8, seed=101, r=(0.05, 0.12))
    rows = np.sort(np.random.default_rng(4).choice(sh.batch, 48, replace=False))
    A = O.make_oarm(wl["arm"])
    idx, _ = O.plan_knn(wl["tree_x"], wl["cand"]["x"][rows], sh.k)
    x0, x1, ok = O.edges_of(wl["tree_x"], wl["cand"]["x"][rows], idx)
    g = O.edge_time(A, x0, x1, wl["grid"], sh.samples, wl["obs"], parent_ok=ok, caps=caps)
    eps = 2e-5
    ref = O.edge_refine(A, x0, x1, g["j"], wl["grid"], sh.samples, 3, eps, wl["obs"], caps=caps)
    ctx = fn.Context(wl["arm"], sh.n_nodes, len(rows), sh.k)
    tree, ld, n = fn.tree_soa(wl["tree_x"])
    r = ctx.edge_refine(tree, ld, n, fn.dev(wl["cand"]["x"][rows]), fn.dev(idx, torch.int32),
                        fn.dev(g["j"], torch.int16), fn.dev(wl["grid"]), sh.samples, n_ary=3,
                        eps=eps, obs=fn.dev(wl["obs"]), caps=fn.dev(caps))
    torch.cuda.synchronize()
    f = g["j"] >= 0
    T = r["T"].cpu().numpy()
    close = np.abs(T[f] - ref["T"][f]) <= 2 * eps + 1e-5 * ref["T"][f]
    assert close.mean() >= 0.99
    rr = ref["rho"][f]
    far = close & np.all(np.abs(rr[:, 1:3] - 1) > 1e-3, axis=1)
    far &= np.isnan(rr[:, 3]) | (np.abs(rr[:, 3] - 1) > 1e-3)
    gs = r["status"].cpu().numpy()[f].astype(np.int64) & (fn.S_VEL | fn.S_POS | fn.S_COLL)
    assert np.array_equal(gs[far], ref["status"][f][far].astype(np.int64))
    assert ((ref["status"][f][far] & O.S_COLL) > 0).sum() >= 10
    ctx.close()


@pytest.mark.parametrize("S", [64, 200, 1000])
def test_full_resolution_check_with_capsules_and_self_pairs(S):
    """edge_check at S = 64, 200 and 1,000 samples with 4 obstacle spheres, 4
    capsules and every sphere pair on links two or more apart (margin 5 mm),
    on slow edges around the middle of the joint range (so that most pass
    their limit checks and reach the clearance)."""
    arm = W.make_arm(0)
    rng = np.random.default_rng(S)
    E = 256
    q0 = rng.uniform(-1.6, 1.6, (E, 7))
    x0 = W._f32(np.concatenate([q0, rng.uniform(-0.2, 0.2, (E, 7))], 1))
    x1 = W._f32(np.concatenate([q0 + rng.uniform(-0.6, 0.6, (E, 7)),
                                rng.uniform(-0.2, 0.2, (E, 7))], 1))
    T = W._f32(rng.uniform(0.8, 1.6, E))
    obs = W.make_obstacles(arm, 4, seed=S)
    caps = W.make_capsules(arm, 4, seed=S)
    pairs = W.self_pairs_apart(arm, 2)
    ctx = fn.Context(arm, 16, E, 4, max_edges=E)
    ctx.set_self_pairs(pairs, margin=0.005)
    out = ctx.edge_check(fn.dev(x0), fn.dev(x1), fn.dev(T), S, fn.dev(obs), caps=fn.dev(caps))
    torch.cuda.synchronize()
    A = O.make_oarm(arm)
    ref = O.edge_check(A, x0, x1, T, S, obs, caps=caps, pairs=pairs, margin_self=0.005)
    st = out["status"].cpu().numpy().astype(np.uint16).astype(np.int64)
    rho = out["rho"].cpu().numpy().astype(np.float64)
    rr = ref["rho"]
    strict = np.all((np.abs(rr - 1) > 1e-3) | np.isnan(rr), axis=1)
    dec = fn.S_DECISION | fn.S_SELF
    assert np.array_equal(st[strict] & dec, ref["status"][strict].astype(np.int64) & dec)
    both = ~np.isnan(rho) & ~np.isnan(rr)
    assert np.allclose(rho[both], rr[both], rtol=1e-4, atol=1e-6)
    assert np.array_equal(np.isnan(rho[strict]), np.isnan(rr[strict]))
    lim = (ref["status"] & (O.S_NONE | O.S_VEL | O.S_POS)) == 0
    n_self = int(((ref["status"] & O.S_SELF) > 0).sum())
    print(f"S = {S}: {lim.sum()} edges reach the clearance, {int(((ref['status'] & O.S_COLL) > 0).sum())} "
          f"collide ({n_self} with themselves), {(~strict).sum()} in the band")
    assert lim.sum() >= 40
    # removing the pairs removes the self part
    ctx.set_self_pairs([], 0.0)
    out2 = ctx.edge_check(fn.dev(x0), fn.dev(x1), fn.dev(T), S, fn.dev(obs), caps=fn.dev(caps))
    torch.cuda.synchronize()
    assert ((out2["status"].cpu().numpy().astype(np.int64) & fn.S_SELF) == 0).all()
    ctx.close()


def test_self_pairs_and_capsules_are_validated():
    arm = W.make_arm(0)
    ctx = fn.Context(arm, 16, 16, 4)
    with pytest.raises(fn.FnError, match="pair 0"):
        ctx.set_self_pairs([(0, 0)])
    with pytest.raises(fn.FnError, match="pair 1"):
        ctx.set_self_pairs([(0, 5), (3, 40)])
    with pytest.raises(fn.FnError, match="pairs"):
        ctx.set_self_pairs(np.zeros((1025, 2), np.int32) + [0, 1])
    x = torch.zeros((4, 14), device="cuda")
    T = torch.ones(4, device="cuda")
    caps = torch.zeros((17, 7), device="cuda")
    with pytest.raises(fn.FnError, match="capsules"):
        ctx.edge_check(x, x, T, 16, caps=caps)
    ctx.close()
