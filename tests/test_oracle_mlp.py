"""Pins of the MLP oracle: GELU against its definition, gradients against
central finite differences (P18), Adam against its closed form on a scalar
quadratic, and learning on a smooth target."""
import math

import numpy as np
from scipy import integrate, stats

from oracle import mlp as M


def test_gelu_is_z_times_normal_cdf():
    z = np.linspace(-6, 6, 101)
    assert np.allclose(M.gelu(z), z * stats.norm.cdf(z), rtol=1e-13, atol=1e-15)
    # derivative by integration of the derivative formula
    for a, b in [(-3.0, -1.0), (-0.5, 2.0), (1.0, 4.0)]:
        val, _ = integrate.quad(lambda s: float(M.gelu_grad(np.array(s))), a, b, epsabs=1e-13)
        assert abs(val - (M.gelu(np.array(b)) - M.gelu(np.array(a)))) < 1e-11


def test_gradients_match_finite_differences():
    sizes = (11, 7, 5, 3, 1)
    params = M.init(3, sizes)
    params = [(w, np.random.default_rng(9 + i).normal(0, 0.1, b.shape)) for i, (w, b) in enumerate(params)]
    rng = np.random.default_rng(4)
    x = rng.uniform(size=(13, 11))
    t = rng.normal(size=13)
    y, cache = M.forward(params, x)
    grads = M.backward(params, cache, y, t)
    h = 1e-6
    for li in range(4):
        for j in range(2):
            p = params[li][j]
            g = grads[li][j]
            flat = p.reshape(-1)
            for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
                old = flat[idx]
                flat[idx] = old + h
                lp = M.loss(params, x, t)
                flat[idx] = old - h
                lm = M.loss(params, x, t)
                flat[idx] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - g.reshape(-1)[idx]) <= 1e-6 * max(1.0, abs(fd)), (li, j, idx, fd, g.reshape(-1)[idx])


def test_adam_closed_form_first_step():
    # First Adam step moves every parameter by -lr sign(g) (bias-corrected
    # moments m/(1-b1) = g and sqrt(v/(1-b2)) = |g|), up to eps.
    params = [(np.array([[1.0, -2.0]]), np.array([0.5, 0.0]))]
    grads = [(np.array([[0.3, -4.0]]), np.array([-1e-3, 2.0]))]
    st = M.adam_state(params)
    M.adam_step(params, grads, st, lr=0.01)
    assert np.allclose(params[0][0], [[0.99, -1.99]], atol=1e-9)
    assert np.allclose(params[0][1], [0.51, -0.01], atol=1e-6)


def test_learns_a_smooth_function():
    sizes = (11, 32, 32, 32, 1)
    params = M.init(1, sizes)
    st = M.adam_state(params)
    rng = np.random.default_rng(2)
    x = rng.uniform(size=(512, 11))
    t = np.sin(3 * x[:, 0]) + x[:, 1] ** 2 - 0.5 * x[:, 2]
    l0 = M.loss(params, x, t)
    for _ in range(300):
        y, cache = M.forward(params, x)
        M.adam_step(params, M.backward(params, cache, y, t), st, lr=3e-3)
    assert M.loss(params, x, t) < 0.05 * l0


def test_bf16_rounding_ties_to_even_and_fixed_points():
    one = 1.0
    # halfway between 1 and 1 + 2^-7 -> even (1.0); halfway between 1 + 2^-7
    # and 1 + 2^-6 -> even (1 + 2^-6); just above halfway -> up
    assert M.bf16(np.array([one + 2.0 ** -8]))[0] == 1.0
    assert M.bf16(np.array([one + 3 * 2.0 ** -8]))[0] == one + 2.0 ** -6
    assert M.bf16(np.array([one + 2.0 ** -8 + 2.0 ** -20]))[0] == one + 2.0 ** -7
    assert M.bf16(np.array([-(one + 2.0 ** -8 + 2.0 ** -20)]))[0] == -(one + 2.0 ** -7)
    rng = np.random.default_rng(0)
    v = rng.normal(size=10000) * 10.0 ** rng.uniform(-5, 5, size=10000)
    q = M.bf16(v)
    assert np.all(np.abs(q - v) <= 2.0 ** -8 * np.abs(v) * 1.0000001)
    assert np.array_equal(M.bf16(q), q)  # idempotent
    # 8 significant bits: q * 2^-e has at most 8 bits
    m, _ = np.frexp(q)
    assert np.all((m * 256.0) == np.round(m * 256.0))


def test_forward_bf16_equals_forward_on_representable_values():
    sizes = (11, 16, 16, 16, 1)
    rng = np.random.default_rng(3)
    params = [(M.bf16(rng.normal(0, 0.3, (a, b))), rng.normal(0, 0.1, b)) for a, b in zip(sizes[:-1], sizes[1:])]
    x = M.bf16(rng.normal(size=(7, 11)))
    y_q = M.forward_bf16(params, x)
    # with activations also representable the two agree; here only the inputs
    # and weights are, so compare against a forward that rounds activations
    a = x
    for li, (w, b) in enumerate(params[:-1]):
        a = M.gelu(a @ w + b)
        if li < 2:
            a = M.bf16(a)
    y_ref = (a @ params[-1][0] + params[-1][1])[:, 0]
    assert np.allclose(y_q, y_ref, rtol=0, atol=1e-13)
    y = M.forward(params, x)[0]
    assert np.max(np.abs(y - y_q)) < 0.05 * np.max(np.abs(y)) + 1e-3


def test_flatten_roundtrip_layout():
    p = M.init(0)
    v = M.flatten(p)
    assert v.size == 11 * 256 + 256 + 2 * (256 * 256 + 256) + 256 + 1 == 134913
    q = M.unflatten(v)
    assert all(np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) for a, b in zip(p, q))
    assert v[0] == p[0][0][0, 0] and v[1] == p[0][0][0, 1] and v[11 * 256] == p[0][1][0]
