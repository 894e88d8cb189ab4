"""FP64 oracle of the learned T-window surrogate (test infrastructure only).

A 4-layer MLP 28 -> 256 -> 256 -> 256 -> 2 with SiLU after the first three
layers maps the two boundary states of an edge to (standardised log T*,
feasibility logit).  Loss: mean squared error on the first output over the
edges that have a feasible slot, plus binary cross-entropy with logits on the
second.  Adam with bias correction (Kingma and Ba, 2015).

Plain numpy in float64.  With ``bf=True`` the values the GPU kernels round
to bfloat16 are rounded here at the same points (round to nearest even, via
float32), everything else stays FP64; this is how the kernels' arithmetic is
defined, and it lets gradients be compared tightly.
"""
from __future__ import annotations

import numpy as np

WIDTH = 256
N_IN = 28
N_OUT = 2
SHAPES = [(WIDTH, N_IN), (WIDTH,), (WIDTH, WIDTH), (WIDTH,), (WIDTH, WIDTH), (WIDTH,),
          (N_OUT, WIDTH), (N_OUT,)]
N_PARAMS = int(sum(np.prod(s) for s in SHAPES))


def unpack(flat):
    out, o = [], 0
    for s in SHAPES:
        n = int(np.prod(s))
        out.append(np.asarray(flat[o:o + n], np.float64).reshape(s))
        o += n
    return out


def pack(params):
    return np.concatenate([np.asarray(p, np.float64).reshape(-1) for p in params])


def init_params(seed: int):
    """U(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases, seeded."""
    rng = np.random.default_rng(seed)
    ps = []
    for s in SHAPES:
        fan_in = s[1] if len(s) == 2 else (N_IN if len(ps) == 0 else WIDTH)
        if len(s) == 1:
            fan_in = ps[-1].shape[1]
        a = 1.0 / np.sqrt(fan_in)
        ps.append(rng.uniform(-a, a, s).astype(np.float32).astype(np.float64))
    return ps


def bf16(x):
    """Round to bfloat16 (nearest even) through float32; returns float64."""
    f = np.asarray(x, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(f)
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def sigmoid(z):
    z = np.asarray(z, np.float64)
    out = np.empty_like(z)
    p = z >= 0
    out[p] = 1.0 / (1.0 + np.exp(-z[p]))
    e = np.exp(z[~p])
    out[~p] = e / (1.0 + e)
    return out


def silu(z):
    return z * sigmoid(z)


def dsilu(z):
    s = sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


def features(x0, x1, arm):
    """28 normalised inputs: joint positions as (q - centre)/half-range and
    velocities as qd/qdmax, for the edge's start then end state."""
    cen = 0.5 * (arm["qmax"] + arm["qmin"])
    half = 0.5 * (arm["qmax"] - arm["qmin"])
    x0 = np.asarray(x0, np.float64)
    x1 = np.asarray(x1, np.float64)
    return np.concatenate([(x0[:, :7] - cen) / half, x0[:, 7:] / arm["qdmax"],
                           (x1[:, :7] - cen) / half, x1[:, 7:] / arm["qdmax"]], axis=1)


def targets(j, grid):
    """(t, f): t = standardised log T* of the result slot (0 where none),
    f = 1 when a slot was found.  Standardisation maps [log T_min, log T_max]
    to [-1, 1]."""
    lg = np.log(np.asarray(grid, np.float64))
    mu = 0.5 * (lg[0] + lg[-1])
    sg = 0.5 * (lg[-1] - lg[0])
    j = np.asarray(j)
    f = (j >= 0).astype(np.float64)
    t = np.where(j >= 0, (lg[np.maximum(j, 0)] - mu) / sg, 0.0)
    return t, f


def forward(params, X, bf=False):
    W1, b1, W2, b2, W3, b3, W4, b4 = params
    g = bf16 if bf else (lambda a: np.asarray(a, np.float64))
    A = [g(X)]
    Z = []
    for W, b in ((W1, b1), (W2, b2), (W3, b3)):
        z = A[-1] @ g(W).T + b
        Z.append(z)
        A.append(g(silu(z)))
    Y = A[-1] @ g(W4).T + b4
    return Y, dict(A=A, Z=Z)


def loss(Y, t, f):
    """(L, L_mse, L_bce, dL/dY)."""
    n = Y.shape[0]
    nf = max(1.0, float(f.sum()))
    r = (Y[:, 0] - t) * f
    lm = float((r * r).sum() / nf)
    z = Y[:, 1]
    # BCE with logits, stable form: max(z, 0) - z f + log(1 + exp(-|z|))
    lb = float((np.maximum(z, 0) - z * f + np.log1p(np.exp(-np.abs(z)))).sum() / n)
    dY = np.zeros_like(Y)
    dY[:, 0] = 2.0 * r / nf
    dY[:, 1] = (sigmoid(z) - f) / n
    return lm + lb, lm, lb, dY


def backward(params, cache, dY, bf=False):
    """Gradients of the loss w.r.t. every parameter, same order as params."""
    W1, b1, W2, b2, W3, b3, W4, b4 = params
    g = bf16 if bf else (lambda a: np.asarray(a, np.float64))
    A, Z = cache["A"], cache["Z"]
    Ws = [W1, W2, W3, W4]
    grads = [None] * 8
    dZ = dY
    for l in (3, 2, 1, 0):
        dzb = g(dZ)
        grads[2 * l] = dzb.T @ A[l]
        grads[2 * l + 1] = dZ.sum(axis=0)
        if l > 0:
            dA = dzb @ g(Ws[l])
            dZ = dA * dsilu(Z[l - 1])
    return grads


def adam_step(params, grads, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (step count t >= 1) with bias correction; returns new
    (params, m, v)."""
    out_p, out_m, out_v = [], [], []
    for p, gr, mm, vv in zip(params, grads, m, v):
        mm = b1 * mm + (1 - b1) * gr
        vv = b2 * vv + (1 - b2) * gr * gr
        mh = mm / (1 - b1 ** t)
        vh = vv / (1 - b2 ** t)
        out_p.append(p - lr * mh / (np.sqrt(vh) + eps))
        out_m.append(mm)
        out_v.append(vv)
    return out_p, out_m, out_v
