"""Pins of the oracle's P-P statistics: closed forms and a conjugate model."""
import math

import numpy as np

from oracle import pp


def test_credible_level_weighted_and_unweighted():
    x = np.array([0.1, 0.5, 0.2, 0.9, 0.7])
    assert pp.credible_level(x, np.ones(5), 0.6) == 3 / 5
    assert pp.credible_level(x, np.ones(5), 0.5) == 2 / 5  # strictly below
    w = np.array([1.0, 0.0, 0.0, 3.0, 0.0])
    assert pp.credible_level(x, w, 0.95) == 1.0
    assert pp.credible_level(x, w, 0.5) == 0.25


def test_ks_pvalue_single_sample_closed_form():
    # one sample x: D = max(x, 1 - x) and P(D >= d) = 2 (1 - d) for d >= 1/2
    for x in (0.3, 0.05, 0.5, 0.81):
        d = max(x, 1 - x)
        assert math.isclose(pp.ks_pvalue([x]), 2 * (1 - d), rel_tol=1e-12)


def test_fisher_closed_forms():
    # k = 1: the combined p-value is p; k = 2 with equal p:
    # X = -4 ln p ~ chi^2_4, survival exp(-X/2)(1 + X/2) = p^2 (1 - 2 ln p)
    for p in (0.3, 0.01, 0.9):
        assert math.isclose(pp.fisher_combined([p]), p, rel_tol=1e-12)
        assert math.isclose(pp.fisher_combined([p, p]), p * p * (1 - 2 * math.log(p)), rel_tol=1e-12)


def test_pp_curve():
    q = np.array([0.1, 0.4, 0.4, 0.9])
    assert np.array_equal(pp.pp_curve(q, [0.0, 0.1, 0.4, 0.5, 1.0]), [0.0, 0.25, 0.75, 0.75, 1.0])


def test_calibrated_and_overconfident_posteriors():
    # Conjugate Gaussian model: theta ~ N(0, 1), y ~ N(theta, s^2), so the
    # posterior is N(y / (1 + s^2), s^2 / (1 + s^2)).  Exact posterior draws
    # give uniform credible levels; a posterior three times too narrow is
    # under-covered and the KS test rejects it.
    rng = np.random.default_rng(4)
    s = 0.5
    good, narrow = [], []
    for _ in range(400):
        th = rng.normal()
        y = th + s * rng.normal()
        mu, sd = y / (1 + s * s), s / math.sqrt(1 + s * s)
        z = rng.normal(size=2000)
        w = np.ones(z.size)
        good.append(pp.credible_level(mu + sd * z, w, th))
        narrow.append(pp.credible_level(mu + sd / 3 * z, w, th))
    assert pp.ks_pvalue(good) > 1e-3
    assert pp.ks_pvalue(narrow) < 1e-10
    assert pp.fisher_combined([pp.ks_pvalue(good), pp.ks_pvalue(narrow)]) < 1e-6
