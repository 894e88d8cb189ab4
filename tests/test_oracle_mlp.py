"""Pins of the MLP oracle: finite differences, torch float64 autograd (an
independent library routine), the first Adam step, the bf16 rounding, the
local rounding bounds of the bf16 mode (with planted rounding mistakes that
must break them) and the loss definition."""
import numpy as np
import pytest

from oracle import mlp as M

torch = pytest.importorskip("torch")


def small_batch(seed=0, n=16):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1, 1, (n, M.N_IN))
    t = rng.uniform(-1, 1, n)
    f = (rng.uniform(0, 1, n) > 0.4).astype(float)
    return X, t, f


def total_loss(params, X, t, f):
    Y, _ = M.forward(params, X)
    return M.loss(Y, t, f)[0]


def test_gradients_against_central_differences():
    params = M.init_params(1)
    X, t, f = small_batch()
    Y, cache = M.forward(params, X)
    _, _, _, dY = M.loss(Y, t, f)
    grads = M.backward(params, cache, dY)
    rng = np.random.default_rng(2)
    h = 1e-6
    for li, p in enumerate(params):
        for _ in range(4):
            idx = tuple(rng.integers(0, s) for s in p.shape)
            old = p[idx]
            p[idx] = old + h
            lp = total_loss(params, X, t, f)
            p[idx] = old - h
            lm = total_loss(params, X, t, f)
            p[idx] = old
            fd = (lp - lm) / (2 * h)
            assert grads[li][idx] == pytest.approx(fd, rel=1e-5, abs=1e-9), (li, idx)


def test_gradients_against_torch_autograd_float64():
    params = M.init_params(3)
    X, t, f = small_batch(4, 32)
    Y, cache = M.forward(params, X)
    L, lm, lb, dY = M.loss(Y, t, f)
    grads = M.backward(params, cache, dY)
    tp = [torch.tensor(p, dtype=torch.float64, requires_grad=True) for p in params]
    Xt = torch.tensor(X)
    h = Xt
    for W, b in ((tp[0], tp[1]), (tp[2], tp[3]), (tp[4], tp[5])):
        h = torch.nn.functional.silu(h @ W.T + b)
    Yt = h @ tp[6].T + tp[7]
    ft = torch.tensor(f)
    nf = max(1.0, float(f.sum()))
    Lt = (((Yt[:, 0] - torch.tensor(t)) * ft) ** 2).sum() / nf + \
        torch.nn.functional.binary_cross_entropy_with_logits(Yt[:, 1], ft)
    Lt.backward()
    assert float(Lt) == pytest.approx(L, rel=1e-12)
    for g, p in zip(grads, tp):
        assert np.allclose(g, p.grad.numpy(), rtol=1e-10, atol=1e-14)


def test_silu_derivative():
    z = np.linspace(-30, 30, 1001)
    h = 1e-6
    fd = (M.silu(z + h) - M.silu(z - h)) / (2 * h)
    assert np.allclose(M.dsilu(z), fd, rtol=1e-6, atol=1e-8)


def test_first_adam_step_is_sign_step():
    """t = 1: m_hat = g and v_hat = g^2, so the update is lr g / (|g| + eps)."""
    params = M.init_params(5)
    rng = np.random.default_rng(6)
    grads = [rng.normal(size=p.shape) for p in params]
    zeros = [np.zeros_like(p) for p in params]
    new, m, v = M.adam_step(params, grads, zeros, zeros, 1, 1e-3)
    for p0, p1, g in zip(params, new, grads):
        assert np.allclose(p0 - p1, 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-18)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(7)
    x = np.concatenate([rng.normal(size=10000) * 10.0 ** rng.integers(-8, 8, 10000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 65504.0, 3.0e38]])
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.bf16(x), ref)


def test_bf16_forward_close_to_fp64():
    params = M.init_params(8)
    X, _, _ = small_batch(9, 64)
    Y, _ = M.forward(params, X)
    Yb, _ = M.forward(params, X, bf=True)
    assert np.max(np.abs(Y - Yb)) < 0.05 * max(1.0, np.max(np.abs(Y)))


def test_loss_definition_special_cases():
    Y = np.array([[0.5, 0.0], [2.0, 100.0]])
    L, lm, lb, _ = M.loss(Y, np.array([0.5, 0.0]), np.array([1.0, 0.0]))
    assert lm == pytest.approx(0.0)
    # BCE(0 logit, 1) = log 2; BCE(100, 0) = 100 + log(1 + e^-100)
    assert lb == pytest.approx((np.log(2) + 100.0) / 2, rel=1e-12)
    t, f = M.targets(np.array([0, 63, -1]), np.geomspace(0.02, 1.0, 64))
    assert t[0] == pytest.approx(-1.0) and t[1] == pytest.approx(1.0) and f[2] == 0.0



# Local rounding bounds of the bf16-emulating mode.  Rounding to bfloat16
# (8 significant bits, nearest even, reached through float32) has relative
# error at most U, and a rounded value is a bfloat16 number.  Layer by layer,
# given the mode's own rounded inputs: the activations must be bfloat16
# numbers within U of SiLU of the pre-activations, the pre-activations (kept
# in high precision) must be within U |A| |W|^T (the weight rounding) plus
# the FP64 accumulation error of the exact affine map, and the bound must not
# be vacuous.  A coarser rounding, a missing rounding of an activation, a
# truncating rounding or an extra rounding of a pre-activation each break one
# of these.
U = 2.0 ** -8 + 2.0 ** -24


def _is_bf16(x):
    f = np.asarray(x, np.float64).astype(np.float32)
    return (f.astype(np.float64) == np.asarray(x)) & ((f.view(np.uint32) & 0xFFFF) == 0)


def _affine_bound(A, W, b, Z):
    """(|Z - A W^T - b|, bound) for a layer whose weights are rounded."""
    ex = A @ W.T + b
    g = W.shape[1] * 2.0 ** -52
    bnd = U * np.abs(A) @ np.abs(W).T + g * (np.abs(A) @ np.abs(W).T + np.abs(b)) * (1 + U)
    return np.abs(Z - ex), bnd


def _check_bf_forward(params, X):
    Yb, cb = M.forward(params, X, bf=True)
    A, Z = cb["A"], cb["Z"]
    Ws, bs = params[0::2], params[1::2]
    assert np.all(_is_bf16(A[0])) and np.all(np.abs(A[0] - X) <= U * np.abs(X))
    ratios = []
    for l in range(3):
        err, bnd = _affine_bound(A[l], Ws[l], bs[l], Z[l])
        assert np.all(err <= bnd), l
        ratios.append(np.max(err / bnd))
        s = M.silu(Z[l])
        assert np.all(_is_bf16(A[l + 1])), l
        assert np.all(np.abs(A[l + 1] - s) <= U * np.abs(s)), l
        # pre-activations stay unrounded
        assert np.mean(_is_bf16(Z[l])) < 0.05, l
    err, bnd = _affine_bound(A[3], Ws[3], bs[3], Yb)
    assert np.all(err <= bnd)
    ratios.append(np.max(err / bnd))
    return Yb, cb, ratios


def test_bf16_forward_within_local_rounding_bounds():
    for seed in (3, 4):
        params = M.init_params(seed)
        X, _, _ = small_batch(seed + 10, 64)
        Y, _ = M.forward(params, X)
        Yb, _, ratios = _check_bf_forward(params, X)
        # the weight rounding shows: each bound is reached to a fair fraction
        assert min(ratios) > 0.02, ratios
        # and the result differs from the FP64 network by far more than FP32 rounding
        assert np.max(np.abs(Yb - Y)) > 1e-4 * np.max(np.abs(Y))


@pytest.mark.parametrize("mistake", ["coarse", "no_act_round", "truncate"])
def test_rounding_mistakes_break_local_bounds(monkeypatch, mistake):
    params = M.init_params(3)
    X, _, _ = small_batch(13, 64)
    if mistake == "coarse":
        def rnd(x):
            # 6 significant bits instead of 8
            m, e = np.frexp(np.asarray(x, np.float64))
            return np.ldexp(np.round(m * 64.0) / 64.0, e)
        monkeypatch.setattr(M, "bf16", rnd)
    elif mistake == "no_act_round":
        monkeypatch.setattr(M, "bf16", lambda x: np.asarray(x, np.float64))
    else:
        def rnd(x):
            # truncation toward zero instead of nearest even
            f = np.asarray(x, np.float64).astype(np.float32)
            return (f.view(np.uint32) & np.uint32(0xFFFF0000)).view(np.float32).astype(np.float64)
        monkeypatch.setattr(M, "bf16", rnd)
    with pytest.raises(AssertionError):
        _check_bf_forward(params, X)


def test_bf16_top_layer_gradient_within_local_bound():
    params = M.init_params(5)
    X, t, f = small_batch(15, 64)
    Yb, cb = M.forward(params, X, bf=True)
    _, _, _, dY = M.loss(Yb, t, f)
    gb = M.backward(params, cb, dY, bf=True)
    A3 = cb["A"][3]
    ex = dY.T @ A3
    err = np.abs(gb[6] - ex)
    bnd = U * np.abs(dY).T @ np.abs(A3) + A3.shape[0] * 2.0 ** -52 * np.abs(dY).T @ np.abs(A3) * (1 + U)
    assert np.all(err <= bnd)
    assert np.max(err / bnd) > 0.02
    # the bias gradient is the unrounded column sum
    assert np.allclose(gb[7], dY.sum(axis=0), rtol=1e-15, atol=0)
