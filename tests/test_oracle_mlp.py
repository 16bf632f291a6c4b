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
