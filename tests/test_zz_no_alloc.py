"""edge_time_batch_noalloc (scratch in a static device array) against
edge_time_batch (scratch in the context), through the C ABI: identical
outputs on two calls in a row, the second one smaller, in every search
mode; sizes beyond the array are refused on the host."""
import numpy as np
import pytest

from paper_2609_22608_amd import workload as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2609_22608_amd import fn  # noqa: E402

KEYS = ("j", "status", "margin", "rho", "work", "screened")


def _inputs(shape, seed):
    wl = W.make_workload(W.CONFIGS[shape], seed=seed)
    tree, ld, n = fn.tree_soa(wl["tree_x"])
    cand = fn.dev(wl["cand"]["x"])
    obs = fn.dev(wl["obs"]) if len(wl["obs"]) else None
    return wl, tree, ld, n, cand, fn.dev(wl["grid"]), obs


def _same(a, b, label):
    """Bit-identical outputs (float outputs compared as bit patterns: the
    clearance ratio is NaN where it is not evaluated)."""
    for key in KEYS:
        x, y = a[key], b[key]
        if x.dtype == torch.float32:
            x, y = x.view(torch.int32), y.view(torch.int32)
        assert torch.equal(x, y), (label, key)


@pytest.mark.parametrize("mode", [fn.SEARCH_SCREEN, fn.SEARCH_PLAIN, fn.SEARCH_WINDOW])
def test_noalloc_equals_context_scratch_on_two_calls(mode):
    big = _inputs("iteration", 101)    # 32,768 edges: the array's maximum
    small = _inputs("tiny", 1)         # 256 edges
    sh = big[0]["shape"]
    ctx = fn.Context(big[0]["arm"], sh.n_nodes, sh.batch, sh.k)
    assert fn.lib().fn_noalloc_scratch_bytes() > 0
    for label, (wl, tree, ld, n, cand, grid, obs) in (("full", big), ("smaller", small)):
        s = wl["shape"]
        idx, _ = ctx.plan_knn(tree, ld, n, cand, s.k, want_d2=False)
        kw = {}
        if mode == fn.SEARCH_WINDOW:
            lo = np.random.default_rng(3).integers(0, s.n_t + 1, idx.numel()).astype(np.int16)
            kw = dict(win_lo=fn.dev(lo, torch.int16), win_half=4)
        print(f"noalloc mode {mode}, {label} call: {idx.numel()} edges", flush=True)
        a = ctx.edge_time_batch(tree, ld, n, cand, idx, grid, s.samples, obs, mode=mode, **kw)
        b = ctx.edge_time_batch(tree, ld, n, cand, idx, grid, s.samples, obs, mode=mode,
                                noalloc=True, **kw)
        torch.cuda.synchronize()
        _same(a, b, f"mode {mode}, {label} call")
        assert int((a["status"] & fn.S_RECHECK64).count_nonzero()) > 0 or label == "smaller"
    ctx.close()


def test_noalloc_refuses_more_edges_than_its_array():
    wl, tree, ld, n, cand, grid, obs = _inputs("tiny", 1)
    ctx = fn.Context(wl["arm"], 1024, 16384, 4)
    B = 8193  # 8193 x 4 = 32,772 edges > 32,768
    nbr = torch.zeros((B, 4), dtype=torch.int32, device="cuda")
    cand_big = torch.zeros((B, 14), dtype=torch.float32, device="cuda")
    with pytest.raises(fn.FnError, match="edge_time_batch_noalloc: 32772 edges"):
        ctx.edge_time_batch(tree, ld, n, cand_big, nbr, grid, 16, noalloc=True)
    ctx.close()
