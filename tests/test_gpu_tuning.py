"""Launch mappings do not change results; the autotuner, the kernel timing
events and the batched round's host-side validation."""
import numpy as np
import pytest

from paper_2609_22608_amd import workload as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2609_22608_amd import autotune, fn  # noqa: E402


@pytest.fixture(scope="module")
def iteration():
    sh = W.CONFIGS["iteration"]
    wl = W.make_workload(sh, seed=303)
    ctx = fn.Context(wl["arm"], sh.n_nodes, sh.batch, sh.k)
    tree, ld, n = fn.tree_soa(wl["tree_x"])
    yield sh, wl, ctx, tree, ld, n, fn.dev(wl["cand"]["x"])
    ctx.close()


def test_knn_result_is_independent_of_the_launch_mapping(iteration):
    sh, wl, ctx, tree, ld, n, cand = iteration
    ref = None
    # chunk lists per query: 48 (default), 12, 192 (general merge), 24, 96
    # (sort-based merge over two entries per lane); all three scan forms (the
    # matrix-core form: 16 queries per wavefront, at most 4096 wavefronts:
    # 12, 192 and 48 entries)
    for tw, mc, form in ((0, 0, 0), (1024, 256, 1), (16384, 64, 1), (2048, 4096, 1),
                         (8192, 512, 1), (4096, 512, 2), (1024, 256, 2), (16384, 64, 2),
                         (8192, 512, 2), (1024, 256, 3), (16384, 64, 3), (2048, 4096, 3),
                         (1024, 512, 3)):
        ctx.set_tuning(tw, mc, form)
        idx, d2 = ctx.plan_knn(tree, ld, n, cand, sh.k)
        torch.cuda.synchronize()
        got = (idx.cpu().numpy(), d2.cpu().numpy())
        if ref is None:
            ref = got
        else:
            assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), (tw, mc, form)
    ctx.set_tuning(0, 0, 0)


def test_autotuner_picks_a_candidate_and_caches_it(iteration, tmp_path):
    sh, wl, ctx, tree, ld, n, cand = iteration
    cache = autotune.Cache(str(tmp_path / "t.json"))
    ch, times = autotune.tune_knn(ctx, tree, ld, n, cand, sh.k, reps=1, cache=cache)
    grid = list(autotune.knn_grid())
    assert (ch.knn_target_waves, ch.knn_min_chunk, ch.knn_form) in grid
    assert len(times) == len(grid) and {f for _, _, f in grid} == set(autotune.KNN_FORMS)
    assert ch.ms == min(times.values())
    ch2, times2 = autotune.tune_knn(ctx, tree, ld, n, cand, sh.k, cache=cache)
    assert ch2 == ch and times2 == {}  # from the cache
    ctx.set_tuning(0, 0, 0)


def test_edge_form_tuner_picks_a_form_and_caches_it(iteration, tmp_path):
    sh, wl, ctx, tree, ld, n, cand = iteration
    idx, _ = ctx.plan_knn(tree, ld, n, cand, sh.k, want_d2=False)
    grid, obs = fn.dev(wl["grid"]), fn.dev(wl["obs"])
    cache = autotune.Cache(str(tmp_path / "e.json"))
    ctx.set_tuning(2048, 512, 1)  # a kNN mapping the edge tuner must keep
    ch, times = autotune.tune_edge(ctx, tree, ld, n, cand, idx, grid, sh.samples, obs,
                                   reps=1, cache=cache)
    assert ctx._tuning[:3] == (2048, 512, 1)
    assert ch.edge_form in autotune.EDGE_FORMS
    assert set(times) == {f"edge_form {f}" for f in autotune.EDGE_FORMS}
    assert ctx.edge_form == ch.edge_form
    ch2, times2 = autotune.tune_edge(ctx, tree, ld, n, cand, idx, grid, sh.samples, obs,
                                     cache=autotune.Cache(str(tmp_path / "e.json")))
    assert ch2 == ch and times2 == {}  # from the cache file
    assert ctx._tuning[:3] == (2048, 512, 1)
    ctx.set_tuning(0, 0, 0, edge_form=0)


def test_kernel_timing_events(iteration):
    sh, wl, ctx, tree, ld, n, cand = iteration
    idx, _ = ctx.plan_knn(tree, ld, n, cand, sh.k, want_d2=False)
    grid, obs = fn.dev(wl["grid"]), fn.dev(wl["obs"])
    ctx.kernel_timing(True)
    assert ctx.kernel_times() == []
    for mode in (fn.SEARCH_PLAIN, fn.SEARCH_SCREEN, fn.SEARCH_SCREEN):
        ctx.edge_time_batch(tree, ld, n, cand, idx, grid, sh.samples, obs, mode=mode)
    ms = ctx.kernel_times()
    assert len(ms) == 3 and all(t > 0 for t in ms)
    assert ms[0] > ms[1]  # the plain search evaluates far more points
    assert ctx.kernel_times() == []  # cleared
    ctx.kernel_timing(False)
    ctx.edge_time_batch(tree, ld, n, cand, idx, grid, sh.samples, obs, mode=fn.SEARCH_SCREEN)
    assert ctx.kernel_times() == []


def test_tuning_and_problem_set_are_validated(iteration):
    sh, wl, ctx, tree, ld, n, cand = iteration
    with pytest.raises(fn.FnError, match="multiple of 64"):
        ctx.set_tuning(4096, 100)
    with pytest.raises(fn.FnError, match="target waves"):
        ctx.set_tuning(1 << 20, 512)
    with pytest.raises(fn.FnError, match="form"):
        ctx.set_tuning(4096, 512, 4)
    with pytest.raises(fn.FnError, match="form"):
        ctx.set_tuning(edge_form=4)
    ctx.set_tuning(edge_form=0)
    with pytest.raises(fn.FnError, match="max_problems = 0"):
        fn.Batch(ctx, fn.dev(wl["grid"]), sh.samples, sh.k).prepare()
    arm, probs = W.make_problem_set(2, 5, nodes=(300, 600), batch=(40, 60))
    sumB = sum(p["shape"].batch for p in probs)
    c2 = fn.Context(arm, 4096, sumB, 8, max_edges=sumB * 8, max_problems=2)
    bt = fn.Batch(c2, fn.dev(probs[0]["grid"]), 32, 8)
    with pytest.raises(fn.FnError, match="no prepared problem set"):
        bt.launch()
    with pytest.raises(fn.FnError, match="nothing captured"):
        bt.replay()
    for wl2 in probs:
        bt.add_problem(wl2["tree_x"], wl2["tree_t"], wl2["cand"], wl2["obs"],
                       capacity=wl2["shape"].n_nodes + 64)
    bt.prepare()
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    bt.capture(s)
    bt.replay()
    torch.cuda.synchronize()
    # a prepare discards the captured graph (it holds the old launch geometry)
    bt.prepare()
    with pytest.raises(fn.FnError, match="nothing captured"):
        bt.replay()
    for wl2 in probs:  # four problems, cap two
        bt.add_problem(wl2["tree_x"], wl2["tree_t"], wl2["cand"], wl2["obs"],
                       capacity=wl2["shape"].n_nodes + 64)
    with pytest.raises(fn.FnError, match="problems"):
        bt.prepare()
    c2.close()


def test_batch_tuner_times_both_edge_forms_and_caches(tmp_path):
    """tune_batch times every kNN mapping in each mode with the one-kernel
    search, then the ordered two-phase search at the screened mode's best
    mapping; the winner is left prepared and cached, and a cache hit restores
    it without timing."""
    arm, probs = W.make_problem_set(3, 5, nodes=(300, 800), batch=(40, 80))
    sh = probs[0]["shape"]
    sumB = sum(p["shape"].batch for p in probs)
    ctx = fn.Context(arm, 4096, sumB, sh.k, max_edges=sumB * sh.k, max_problems=len(probs))
    bt = fn.Batch(ctx, fn.dev(probs[0]["grid"]), sh.samples, sh.k)
    for wl in probs:
        bt.add_problem(wl["tree_x"], wl["tree_t"], wl["cand"], wl["obs"],
                       capacity=wl["shape"].n_nodes + 256)
    bt.prepare()
    cands = ((1024, 256), (2048, 512))
    cache = autotune.Cache(str(tmp_path / "b.json"))
    ch, times = autotune.tune_batch(bt, reps=1, cache=cache, candidates=cands)
    n_grid = len(list(autotune.knn_grid(cands)))
    assert len(times) == 2 * n_grid + 1  # both modes, then the ordered form once
    assert sum(k.endswith("/e3") for k in times) == 1
    assert ch.edge_form in (1, 3) and ch.ms == min(times.values())
    assert ctx.edge_form == ch.edge_form and bt.mode == ch.mode
    ch2, times2 = autotune.tune_batch(bt, cache=autotune.Cache(str(tmp_path / "b.json")),
                                      candidates=cands)
    assert ch2 == ch and times2 == {}
    ctx.close()
