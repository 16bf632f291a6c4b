"""FP64 reference of the likelihood prescreen network.

Not part of the paper (its sampler uses exact likelihoods only).  The
prescreen is a fully connected network 11 -> 256 -> 256 -> 256 -> 1 with the
exact GELU activation g(z) = z Phi(z) = z (1 + erf(z / sqrt 2)) / 2, trained by
mean squared error on standardised (unit-cube point, log L) pairs with Adam
(Kingma & Ba 2015): m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2,
p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

Parameters are a list [(W1, b1), ..., (W4, b4)] with W_l of shape
[fan_in, fan_out]; a layer computes z = a W + b.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SIZES = (11, 256, 256, 256, 1)
BETA1, BETA2, EPS = 0.9, 0.999, 1e-8


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    # d/dz [z Phi(z)] = Phi(z) + z phi(z)
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(params, x):
    """Returns (y [n], cache) with cache = [(a_in, z)] per layer."""
    a = np.asarray(x, dtype=np.float64)
    cache = []
    for li, (w, b) in enumerate(params):
        z = a @ w + b
        cache.append((a, z))
        a = z if li == len(params) - 1 else gelu(z)
    return a[:, 0], cache


def loss(params, x, t):
    y, _ = forward(params, x)
    return float(np.mean((y - t) ** 2))


def backward(params, cache, y, t):
    """Gradients of the mean squared error with respect to every (W, b)."""
    n = y.shape[0]
    dz = (2.0 / n) * (y - t)[:, None]
    grads = [None] * len(params)
    for li in range(len(params) - 1, -1, -1):
        a_in, z = cache[li]
        grads[li] = (a_in.T @ dz, dz.sum(axis=0))
        if li > 0:
            da = dz @ params[li][0].T
            dz = da * gelu_grad(cache[li - 1][1])
    return grads


def adam_step(params, grads, state, lr):
    """One Adam update in place; ``state`` = dict(t, m, v)."""
    state["t"] += 1
    t = state["t"]
    for li in range(len(params)):
        for j in range(2):
            g = grads[li][j]
            state["m"][li][j] = BETA1 * state["m"][li][j] + (1 - BETA1) * g
            state["v"][li][j] = BETA2 * state["v"][li][j] + (1 - BETA2) * g * g
            mh = state["m"][li][j] / (1 - BETA1 ** t)
            vh = state["v"][li][j] / (1 - BETA2 ** t)
            p = params[li][j] - lr * mh / (np.sqrt(vh) + EPS)
            params[li] = (p, params[li][1]) if j == 0 else (params[li][0], p)


def adam_state(params):
    return dict(t=0, m=[[np.zeros_like(w), np.zeros_like(b)] for w, b in params],
                v=[[np.zeros_like(w), np.zeros_like(b)] for w, b in params])


def init(seed: int, sizes=SIZES):
    """He-normal weights, zero biases (any initialisation serves the tests)."""
    rng = np.random.default_rng(seed)
    return [(rng.normal(0.0, math.sqrt(2.0 / a), size=(a, b)), np.zeros(b)) for a, b in zip(sizes[:-1], sizes[1:])]


def bf16(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64.

    bfloat16 keeps the sign, the 8 exponent bits and the top 7 fraction bits
    of an IEEE binary32 value; the value is first rounded to binary32.
    """
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward_bf16(params, x):
    """Forward pass with the quantisation points of the BF16 inference path.

    Reading (not in the paper): the standardised input, the weights of the
    three hidden layers and the activations entering hidden layers 2 and 3 are
    rounded to bfloat16; every product and sum is exact (FP64 here); biases,
    GELU and the 256 -> 1 output layer stay at full precision.
    """
    a = bf16(x)
    n_layers = len(params)
    for li, (w, b) in enumerate(params):
        if li == n_layers - 1:
            return (a @ w + b)[:, 0]
        z = a @ bf16(w) + b
        a = gelu(z)
        if li < n_layers - 2:
            a = bf16(a)
    return a[:, 0]


def flatten(params):
    """Parameter list -> one vector: W1, b1, W2, b2, ... (W row-major [in, out])."""
    return np.concatenate([np.concatenate([w.reshape(-1), b.reshape(-1)]) for w, b in params])


def unflatten(vec, sizes=SIZES):
    vec = np.asarray(vec, dtype=np.float64)
    out, o = [], 0
    for a, b in zip(sizes[:-1], sizes[1:]):
        w = vec[o:o + a * b].reshape(a, b)
        o += a * b
        out.append((w, vec[o:o + b].copy()))
        o += b
    return out
