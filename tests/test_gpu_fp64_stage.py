"""The FP64 stage on edges whose decisions lie inside the 1e-3 band: slot
decisions on a fine grid, and clearance ratios placed inside the band.

A 256-slot grid over 0.55-0.57 s spaces the slots about 8e-5 apart in
ratio, so an edge whose minimum time falls inside it meets a run of slots
within 1e-3 of 1: the search hands over the first of them, goes on to the
next candidate (often again in the band), and the FP64 stage decides both
and walks on in FP64 when both fail.  Every such decision is FP64 on both
sides, so T index and status must equal the FP64 oracle on every edge whose
oracle margin is above 1e-9 (the two FP64 evaluations differ in rounding
only, ~1e-14).  Margins: the smallest |rho - 1| the decision rests on.
"""
import numpy as np
import pytest

import oracle as O
from paper_2609_22608_amd import workload as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2609_22608_amd import fn  # noqa: E402


@pytest.fixture(scope="module")
def fine():
    sh = W.CONFIGS["iteration"]
    wl = W.make_workload(sh, seed=606)
    nb = 256
    cx = wl["cand"]["x"][:nb]
    idx, _ = O.plan_knn(wl["tree_x"], cx, sh.k)
    x0, x1, ok = O.edges_of(wl["tree_x"], cx, idx)
    grid = W.t_grid(256, 0.55, 0.57)
    ref = O.edge_time(O.make_oarm(wl["arm"]), x0, x1, grid, sh.samples, wl["obs"], parent_ok=ok)
    return sh, wl, cx, idx, grid, ref


@pytest.mark.parametrize("mode", [fn.SEARCH_PLAIN, fn.SEARCH_SCREEN])
def test_band_decisions_equal_the_fp64_oracle(fine, mode):
    sh, wl, cx, idx, grid, ref = fine
    in_band = ref["margin"] < 1e-3
    inside = ref["j"] > 0
    # the grid does what it is meant to: edges decided inside the band,
    # several of them with the minimum time strictly inside the grid
    assert in_band.sum() >= 20 and (inside & in_band).sum() >= 15
    ctx = fn.Context(wl["arm"], sh.n_nodes, len(cx), sh.k)
    tree, ld, n = fn.tree_soa(wl["tree_x"])
    out = ctx.edge_time_batch(tree, ld, n, fn.dev(cx), fn.dev(idx, torch.int32), fn.dev(grid),
                              sh.samples, fn.dev(wl["obs"]), mode=mode)
    torch.cuda.synchronize()
    gj = out["j"].cpu().numpy().astype(np.int64)
    st = out["status"].cpu().numpy().astype(np.uint16)
    gs = st.astype(np.int64) & fn.S_DECISION
    sel = ref["margin"] > 1e-9
    bad = sel & ((gj != ref["j"]) | (gs != ref["status"].astype(np.int64)))
    n64 = int(((st & fn.S_RECHECK64) > 0).sum())
    print(f"mode {mode}: {len(gj)} edges, {int(in_band.sum())} in the band, "
          f"{int((inside & in_band).sum())} with j* inside the grid, FP64 stage {n64}, "
          f"mismatches {int(bad.sum())}")
    assert bad.sum() == 0, np.nonzero(bad)[0][:10]
    # every in-band decision went through the FP64 stage (0.9e-3: clear of the
    # band's edge by far more than the FP32 error)
    deep = ref["margin"] < 0.9e-3
    assert np.all((st[deep & sel] & fn.S_RECHECK64) > 0)
    gm = out["margin"].cpu().numpy()
    fin = np.isfinite(ref["margin"]) & in_band
    assert np.allclose(gm[fin], ref["margin"][fin], rtol=1e-3, atol=2e-6)
    ctx.close()


def _obstacle_radius_for(A, x0, x1, T, S, centre, target):
    """Radius r of one obstacle at `centre` with oracle rho_c = target (bisection
    on r: rho_c grows with r), or None when no radius in [0, 2] gives it."""
    def rc(r):
        return O.rho_c(A, x0, x1, T, S, np.array([[*centre, r]], np.float64))
    lo, hi = 0.0, 2.0
    if not (rc(lo) < target < rc(hi)):
        return None
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        if rc(mid) < target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


@pytest.mark.parametrize("mode", [fn.SEARCH_PLAIN, fn.SEARCH_SCREEN])
def test_clearance_in_the_band_is_decided_in_fp64(mode):
    """One obstacle sized so that an edge's clearance ratio at its result slot
    is 1 -/+ 3e-4 (inside the 1e-3 band, on either side of the limit): the
    FP32 post-check queues the edge, the FP64 stage evaluates the clearance
    (its per-pair table of 1 / need^2) and the collision bit equals the FP64
    oracle's on both sides."""
    sh = W.CONFIGS["iteration"]
    wl = W.make_workload(sh, seed=707)
    A = O.make_oarm(wl["arm"])
    cx = wl["cand"]["x"][:48]
    idx, _ = O.plan_knn(wl["tree_x"], cx, sh.k)
    x0, x1, ok = O.edges_of(wl["tree_x"], cx, idx)
    grid = wl["grid"]
    ref = O.edge_time(A, x0, x1, grid, sh.samples, parent_ok=ok)
    # edges clear at their result without obstacles
    cand_edges = np.nonzero((ref["j"] >= 0) & (ref["status"] == 0) & (ref["margin"] > 1e-2))[0]
    assert len(cand_edges) >= 4
    ctx = fn.Context(wl["arm"], sh.n_nodes, 1, sh.k)
    tree, ld, n = fn.tree_soa(wl["tree_x"])
    centres = [np.asarray(o[:3], np.float64) for o in wl["obs"]]
    checked = 0
    for e in cand_edges:
        T = float(grid[ref["j"][e]])
        for target, coll in ((1.0 + 3e-4, True), (1.0 - 3e-4, False)):
            r = None
            for c in centres:
                r = _obstacle_radius_for(A, x0[e], x1[e], T, sh.samples, c, target)
                if r is not None:
                    break
            if r is None:
                continue
            obs = np.array([[*c, r]], np.float32)
            # the float32 obstacle moves the oracle's ratio by ~1e-8: decide on it
            rc = O.rho_c(A, x0[e], x1[e], T, sh.samples, obs.astype(np.float64))
            assert abs(rc - target) < 1e-5
            b, i = divmod(int(e), sh.k)
            nbr = np.full((1, sh.k), -1, np.int32)
            nbr[0, i] = idx[b, i]
            out = ctx.edge_time_batch(tree, ld, n, fn.dev(cx[b:b + 1]), fn.dev(nbr, torch.int32),
                                      fn.dev(grid), sh.samples, fn.dev(obs), mode=mode)
            torch.cuda.synchronize()
            st = int(out["status"].cpu().numpy()[i]) & 0xffff
            assert int(out["j"].cpu().numpy()[i]) == ref["j"][e]
            assert st & fn.S_RECHECK64, (e, target)
            assert bool(st & fn.S_COLL) == (rc > 1.0) == coll, (e, target, rc, st)
            rho = out["rho"].cpu().numpy()[i]
            assert abs(rho[3] - rc) < 1e-6, (rho, rc)
            checked += 1
        if checked >= 8:
            break
    assert checked >= 4
    ctx.close()
