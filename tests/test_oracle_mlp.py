"""Pins of the MLP oracle: finite differences, torch float64 autograd (an
independent library routine), the first Adam step, the bf16 rounding and the
loss definition."""
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
