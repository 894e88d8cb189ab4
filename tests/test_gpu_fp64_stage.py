"""The FP64 stage on edges whose decisions all lie inside the 1e-3 band.

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
