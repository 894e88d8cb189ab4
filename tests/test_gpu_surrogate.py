"""GPU parity of the learned T-window surrogate (MFMA forward / backward,
Adam) against the FP64 MLP oracle with the same BF16 rounding points, and
the windowed search it drives."""
import os
import tempfile

import numpy as np
import pytest

import oracle as O
from oracle import mlp as M
from paper_2609_22608_amd import workload as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2609_22608_amd import fn  # noqa: E402


@pytest.fixture(scope="module")
def setup():
    arm = W.make_arm(0)
    ctx = fn.Context(arm, 16384, 4096, 8)
    return arm, ctx


def _batch(arm, n, seed):
    rng = np.random.default_rng(seed)
    x0 = W.uniform_states(arm, n, rng)
    x1 = W.uniform_states(arm, n, rng)
    X = W._f32(np.concatenate([x0, x1], axis=1))
    j = rng.integers(-1, 64, n).astype(np.int16)
    return X, j


def test_forward_matches_oracle(setup):
    arm, ctx = setup
    params = M.init_params(11)
    net = fn.Surrogate(ctx)
    net.set_params(M.pack(params))
    X, _ = _batch(arm, 1000, 1)
    grid = W.t_grid(64, 0.02, 1.0)
    out, win = net.infer(fn.dev(X), fn.dev(grid))
    torch.cuda.synchronize()
    Y = out.cpu().numpy().astype(np.float64)
    ref, _ = M.forward(params, M.features(X[:, :14], X[:, 14:], arm), bf=True)
    err = np.abs(Y - ref)
    print(f"forward abs err: max {err.max():.2e}, median {np.median(err):.2e}, "
          f"|Y| max {np.abs(ref).max():.2f}")
    assert err.max() <= 2e-2 * max(1.0, np.abs(ref).max())
    assert np.median(err) <= 1e-3


@pytest.mark.parametrize("N", [1, 63, 64, 65, 4097])
def test_fused_inference_ragged_rows_and_windows(setup, N):
    """The one-launch inference kernel over a ragged number of rows: outputs
    against the BF16-emulating oracle, and the window of every row from its
    own output (nearest grid slot of the predicted log T, minus half, or n_t
    below the logit threshold)."""
    arm, ctx = setup
    params = M.init_params(21)
    net = fn.Surrogate(ctx)
    net.set_params(M.pack(params))
    X, _ = _batch(arm, N, 40 + N)
    grid = W.t_grid(64, 0.02, 1.0)
    out, win = net.infer(fn.dev(X), fn.dev(grid), half=3, logit_min=0.1)
    torch.cuda.synchronize()
    Y = out.cpu().numpy().astype(np.float64)
    ref, _ = M.forward(params, M.features(X[:, :14], X[:, 14:], arm), bf=True)
    err = np.abs(Y - ref)
    assert err.max() <= 2e-2 * max(1.0, np.abs(ref).max())
    assert np.median(err) <= 1e-3
    y = out.cpu().numpy()
    lg = np.log(grid.astype(np.float32)).astype(np.float32)
    lt = np.float32(0.5) * (lg[0] + lg[-1]) + np.float32(0.5) * (lg[-1] - lg[0]) * y[:, 0]
    d = np.abs(lt[:, None] - lg[None, :])
    j = np.argmin(d, axis=1)
    exp = np.where(y[:, 1] >= np.float32(0.1), np.maximum(0, j - 3), 64)
    got = win.cpu().numpy().astype(np.int64)
    srt = np.sort(d, axis=1)
    tie = (srt[:, 1] - srt[:, 0]) < 1e-5  # nearest slot decided by rounding
    assert np.array_equal(got[~tie], exp[~tie])


@pytest.mark.parametrize("B,k", [(1, 1), (37, 8), (512, 8)])
def test_window_gathers_edge_rows_like_features_then_infer(setup, B, k):
    """surrogate_window (edge rows gathered inside the inference kernel)
    returns bit for bit what edge_features followed by surrogate_infer
    returns, padded and out-of-range parents included, with 32 to 256 rows
    per workgroup."""
    arm, ctx = setup
    params = M.init_params(31)
    net = fn.Surrogate(ctx)
    net.set_params(M.pack(params))
    rng = np.random.default_rng(B)
    tree_x = W._f32(W.uniform_states(arm, 300, rng))
    tree, ld, n = fn.tree_soa(tree_x)
    cand = fn.dev(W._f32(W.uniform_states(arm, B, rng)))
    nbr = rng.integers(0, n, (B, k)).astype(np.int32)
    nbr.reshape(-1)[::7] = -1        # padded parents
    nbr.reshape(-1)[3::11] = n + 5   # beyond the node count
    idx = fn.dev(nbr, torch.int32)
    grid = fn.dev(W.t_grid(64, 0.02, 1.0))
    X = fn.edge_features(ctx, tree, ld, n, cand, idx)
    ys = []
    for rows in (32, 64, 128, 256):  # rows per workgroup of the fused kernel
        ctx.set_tuning(mlp_rows=rows)
        ys.append(net.infer(X, grid, half=4, logit_min=0.05))
        ys.append(net.window(tree, ld, n, cand, idx, grid, half=4, logit_min=0.05, want_out=True))
    ctx.set_tuning(mlp_rows=0)
    torch.cuda.synchronize()
    for y, w in ys[1:]:
        assert torch.equal(ys[0][0].view(torch.int32), y.view(torch.int32))
        assert torch.equal(ys[0][1], w)


def test_gradient_matches_oracle(setup):
    arm, ctx = setup
    params = M.init_params(12)
    net = fn.Surrogate(ctx)
    net.set_params(M.pack(params))
    X, j = _batch(arm, 512, 2)
    grid = W.t_grid(64, 0.02, 1.0)
    g, l3 = net.grad(fn.dev(X), fn.dev(j, torch.int16), fn.dev(grid))
    torch.cuda.synchronize()
    gg = M.unpack(g.cpu().numpy().astype(np.float64))
    Y, cache = M.forward(params, M.features(X[:, :14], X[:, 14:], arm), bf=True)
    t, f = M.targets(j, grid)
    L, lm, lb, dY = M.loss(Y, t, f)
    ref = M.backward(params, cache, dY, bf=True)
    assert l3.cpu().numpy()[0] == pytest.approx(L, rel=1e-3)
    for i, (a, b) in enumerate(zip(gg, ref)):
        rel = np.linalg.norm(a - b) / max(1e-30, np.linalg.norm(b))
        print(f"param tensor {i}: relative gradient error {rel:.2e}")
        assert rel <= 2e-2, i


def test_one_adam_step_matches_oracle(setup):
    arm, ctx = setup
    params = M.init_params(13)
    net = fn.Surrogate(ctx)
    net.set_params(M.pack(params))
    X, j = _batch(arm, 256, 3)
    grid = W.t_grid(64, 0.02, 1.0)
    net.train(fn.dev(X), fn.dev(j, torch.int16), fn.dev(grid), epochs=1, batch=256, lr=1e-3,
              cosine=False)
    new = M.unpack(net.get_params().astype(np.float64))
    # oracle: the same (only) minibatch, permuted rows do not change a full-batch gradient
    Y, cache = M.forward(params, M.features(X[:, :14], X[:, 14:], arm), bf=True)
    t, f = M.targets(j, grid)
    _, _, _, dY = M.loss(Y, t, f)
    grads = M.backward(params, cache, dY, bf=True)
    zeros = [np.zeros_like(p) for p in params]
    ref, _, _ = M.adam_step(params, grads, zeros, zeros, 1, 1e-3)
    for p0, a, b, gr in zip(params, new, ref, grads):
        big = np.abs(gr) > 1e-2 * np.abs(gr).max()
        assert np.allclose((a - p0)[big], (b - p0)[big], rtol=1e-3, atol=1e-7)


def test_save_load_roundtrip(setup):
    arm, ctx = setup
    net = fn.Surrogate(ctx, seed=5)
    p = net.get_params()
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "s.bin")
        net.save(path)
        net2 = fn.Surrogate.load(ctx, path)
        assert np.array_equal(net2.get_params(), p)


def test_training_learns_and_window_is_exact(setup):
    """Labels from the exact search on one-iteration-shaped batches; a short
    training run must cut the loss, and windowed search driven by the
    trained network must equal the plain search on held-out edges."""
    arm, ctx = setup
    sh = W.CONFIGS["iteration"]
    grid = fn.dev(W.t_grid(sh.n_t, sh.t_min, sh.t_max))
    Xs, ys = [], []
    for seed in range(1000, 1004):
        wl = W.make_workload(sh, seed=seed, arm=arm)
        tree, ld, n = fn.tree_soa(wl["tree_x"])
        cand = fn.dev(wl["cand"]["x"])
        idx, _ = ctx.plan_knn(tree, ld, n, cand, sh.k, want_d2=False)
        out = ctx.edge_time_batch(tree, ld, n, cand, idx, grid, sh.samples, fn.dev(wl["obs"]),
                                  mode=fn.SEARCH_SCREEN)
        Xs.append(fn.edge_features(ctx, tree, ld, n, cand, idx))
        ys.append(out["j"].clone())
    X = torch.cat(Xs)
    y = torch.cat(ys)
    net = fn.Surrogate(ctx, seed=1)
    losses = net.train(X, y, grid, epochs=8, batch=2048, lr=2e-3)
    torch.cuda.synchronize()
    L = losses.cpu().numpy()
    print("epoch losses (total, squared error, cross-entropy)\n", L)
    assert L[-1, 0] < 0.85 * L[0, 0]
    assert L[-1, 1] < 0.7 * L[0, 1]
    # held-out batch: windowed == plain on every edge
    wl = W.make_workload(sh, seed=2_000_001, arm=arm)
    tree, ld, n = fn.tree_soa(wl["tree_x"])
    cand = fn.dev(wl["cand"]["x"])
    obs = fn.dev(wl["obs"])
    idx, _ = ctx.plan_knn(tree, ld, n, cand, sh.k, want_d2=False)
    feats = fn.edge_features(ctx, tree, ld, n, cand, idx)
    _, win = net.infer(feats, grid, half=4)
    a = ctx.edge_time_batch(tree, ld, n, cand, idx, grid, sh.samples, obs, mode=fn.SEARCH_PLAIN)
    b = ctx.edge_time_batch(tree, ld, n, cand, idx, grid, sh.samples, obs, mode=fn.SEARCH_WINDOW,
                            win_lo=win, win_half=4)
    torch.cuda.synchronize()
    assert torch.equal(a["j"], b["j"])
    da = a["status"].cpu().numpy().astype(np.uint16) & fn.S_DECISION
    db = b["status"].cpu().numpy().astype(np.uint16) & fn.S_DECISION
    assert np.array_equal(da, db)
    sb = b["status"].cpu().numpy().astype(np.uint16)
    feasible = a["j"].cpu().numpy() >= 0
    miss = ((sb & fn.S_WIN_MISS) > 0)
    below = ((sb & fn.S_WIN_BELOW) > 0)
    assert ((sb & (fn.S_WIN_HIT | fn.S_WIN_MISS)) > 0).all()
    print(f"window miss rate over F-feasible edges {miss[feasible].mean():.4f}, "
          f"all edges {miss.mean():.4f}; below-window full passes {below.mean():.4f}; "
          f"work plain {a['work'].sum().item()} window {b['work'].sum().item()}")
    assert b["work"].sum().item() < a["work"].sum().item()
    # the windowed search never evaluates more than the screened one
    c = ctx.edge_time_batch(tree, ld, n, cand, idx, grid, sh.samples, obs, mode=fn.SEARCH_SCREEN)
    torch.cuda.synchronize()
    assert b["work"].sum().item() <= c["work"].sum().item()
    # 384 sampled held-out edges of the windowed search against the FP64 oracle
    nbr = idx.cpu().numpy()
    sel = np.random.default_rng(17).choice(nbr.size, 384, replace=False)
    x0, x1, ok = O.edges_of(wl["tree_x"], wl["cand"]["x"], nbr)
    ref = O.edge_time(O.make_oarm(arm), x0[sel], x1[sel], wl["grid"], sh.samples, wl["obs"],
                      parent_ok=ok[sel])
    gj = b["j"].cpu().numpy().astype(np.int64)[sel]
    gs = db[sel].astype(np.int64)
    strict = ref["margin"] > 1e-3
    assert strict.sum() >= 350
    bad = strict & ((gj != ref["j"]) | (gs != ref["status"]))
    assert bad.sum() == 0, np.nonzero(bad)[0][:10]
