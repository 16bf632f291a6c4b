"""Pins of the oracle's fiducial search (differential evolution) and of the
conditional peak of (d_L, phi_c)."""
import itertools
import math

import numpy as np
import pytest

import gwsynth
from oracle import fiducial as F
from oracle import likelihood as L


@pytest.mark.parametrize("pop", [4, 5, 7])
def test_partner_selection_is_a_bijection(pop):
    # every (k1, k2, k3) gives three distinct partners other than i, and the
    # map onto ordered triples is one to one
    for i in range(pop):
        seen = set()
        for k1, k2, k3 in itertools.product(range(pop - 1), range(pop - 2), range(pop - 3)):
            u = [(k1 + 0.5) / (pop - 1), (k2 + 0.5) / (pop - 2), (k3 + 0.5) / (pop - 3)]
            r = F.de_partners(i, pop, u)
            assert len({i, *r}) == 4 and all(0 <= v < pop for v in r)
            seen.add(r)
        assert len(seen) == (pop - 1) * (pop - 2) * (pop - 3)


def test_trial_crossover_and_reflection():
    rng = np.random.default_rng(0)
    x = rng.uniform(0.2, 0.8, size=(6, 11))
    lo, hi = np.zeros(11), np.ones(11)
    u = F.de_uniforms(3, 0, 2)
    r1, r2, r3 = F.de_partners(2, 6, u)
    jr = int(math.floor(u[3] * 11))
    t0 = F.de_trial(x, 2, np.concatenate([u[:4], np.ones(11)]), 0.6, 0.0, lo, hi)  # CR = 0: jrand only
    diff = np.nonzero(t0 != x[2])[0]
    assert set(diff) <= {jr}
    assert t0[jr] == x[r1, jr] + 0.6 * (x[r2, jr] - x[r3, jr])
    t1 = F.de_trial(x, 2, u, 0.6, 1.0, lo, hi)  # CR = 1: the whole mutant
    assert np.array_equal(t1, x[r1] + 0.6 * (x[r2] - x[r3]))
    # reflection: a huge step stays in a narrow box and mirrors at its walls
    lo2, hi2 = np.full(11, 0.4), np.full(11, 0.6)
    t2 = F.de_trial(x, 2, u, 50.0, 1.0, lo2, hi2)
    assert np.all((t2 >= 0.4) & (t2 <= 0.6))
    xx = np.full((4, 11), 0.5)
    xx[1, 0], xx[2, 0], xx[3, 0] = 0.5, 0.58, 0.5  # v = 0.5 + 1.0 * 0.08 = 0.58 inside
    uu = np.concatenate([[0.1, 0.1, 0.1, 0.0], np.zeros(11)])  # partners 1, 2, 3; cross everything
    assert F.de_partners(0, 4, uu) == (1, 2, 3)
    assert F.de_trial(xx, 0, uu, 1.0, 1.0, lo2, hi2)[0] == 0.58
    xx[2, 0] = 0.65  # v = 0.65 > 0.6: reflected to 0.55
    assert abs(F.de_trial(xx, 0, uu, 1.0, 1.0, lo2, hi2)[0] - 0.55) < 1e-15


def test_search_finds_a_known_maximum_and_never_loses_it():
    c = np.linspace(0.3, 0.7, 11)

    def obj(x):
        return -np.sum(((x - c) / 0.05) ** 2, axis=1)

    x0 = np.random.default_rng(1).uniform(size=(60, 11))
    best = []
    x, fx = x0, obj(x0)
    for g in range(0, 160, 20):
        x, fx, _, b = F.de_search(obj, x, 20, seed=9 + g)
        best.append(fx[b])
    assert all(a <= b for a, b in zip(best, best[1:]))
    assert np.max(np.abs(x[b] - c)) < 2e-3


def test_conditional_peak_is_the_plain_likelihood_maximum():
    prob = gwsynth.make_problem(4.0, 20.0, 40.0, psd_scale=1e-49)
    th = gwsynth.prior_draws(gwsynth.SEEDS["injection"], 1)[0]
    th[6] = 80.0
    prob.data = prob.data + L.strain(th, prob)
    t1 = th.copy()
    t1[6], t1[11] = 1.0, 0.0
    z1, hh1 = L.overlap(t1, prob)
    d, phi = F.conditional_peak(z1, hh1)
    # brute force over a fine grid around the prediction, unexpanded residual form
    ds = d * (1 + np.linspace(-0.02, 0.02, 41))
    ps = phi + np.linspace(-0.05, 0.05, 41)
    vals = np.array([[L.loglike_direct(np.concatenate([th[:6], [dd], th[7:11], [pp], th[12:]]), prob)
                      for pp in ps] for dd in ds])
    j, m = np.unravel_index(np.argmax(vals), vals.shape)
    assert j == 20 and m == 20
