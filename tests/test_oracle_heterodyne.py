"""Pins of the heterodyne oracle: exact special cases, convergence, bin rule."""
import math

import numpy as np
import pytest

import gwsynth
from oracle import heterodyne as H
from oracle import likelihood as L


@pytest.fixture(scope="module")
def het_problem(loud_problem):
    het = H.setup(loud_problem, loud_problem.theta_inj, 200)
    return loud_problem, het


def test_reference_point_is_exact(het_problem):
    # P14: theta = theta0 gives r = 1 in every bin, so the binned sums are the
    # full-band sums regrouped.
    prob, het = het_problem
    dd = L.data_inner(prob)
    for marg in (L.PLAIN, L.PHASE, L.PHASE_DIST):
        full = L.loglike(het.theta0, prob, marg, dd)
        got = H.loglike(het.theta0, prob, het, marg, dd)
        assert abs(got - full) < 1e-9 * dd, (marg, got, full)


@pytest.mark.parametrize("col,val", [(6, 137.0), (11, 2.1), (10, 0.3), (7, 2.0)])
def test_extrinsic_scalar_changes_are_exact(het_problem, col, val):
    # Changing only d_L, phi_c, psi or iota multiplies each h_i by a constant,
    # so r_i is flat and the linear expansion is exact.
    prob, het = het_problem
    th = het.theta0.copy()
    th[col] = val
    dd = L.data_inner(prob)
    for marg in (L.PLAIN, L.PHASE):
        assert abs(H.loglike(th, prob, het, marg, dd) - L.loglike(th, prob, marg, dd)) < 1e-9 * dd


def test_error_shrinks_with_bins(loud_problem):
    prob = loud_problem
    th0 = prob.theta_inj
    pts = gwsynth.near_posterior(77, th0, 6, scale=0.5)
    dd = L.data_inner(prob)
    full = np.array([L.loglike(t, prob, L.PHASE, dd) for t in pts])
    errs = []
    for nb in (20, 80, 320):
        het = H.setup(prob, th0, nb)
        got = np.array([H.loglike(t, prob, het, L.PHASE, dd) for t in pts])
        errs.append(np.max(np.abs(got - full)))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.05


def test_bin_rule_equal_phase_bound_steps():
    g = gwsynth.freq_grid(128.0, 20.0, 2048.0)
    f = g.freqs
    e = H.bin_edges(f, 500, 0)
    assert e[0] == 0 and e[-1] == len(f) - 1 and np.all(np.diff(e) > 0)
    phi = H.phase_bound(f, f[0], f[-1])
    step = (phi[-1] - phi[0]) / 500
    d = np.diff(phi[e])
    # equal increments up to snapping to the fine grid (one bin of slope)
    slope = np.abs(np.gradient(phi, f))[e[:-1]] * g.df
    assert np.all(np.abs(d - step) <= slope + np.abs(np.gradient(phi, f))[e[1:]] * g.df + 1e-12)
    # low frequencies get narrow bins, high frequencies wide ones
    w = np.diff(f[e])
    assert w[0] < w[-1]


def test_paper_operation_count():
    # Sec. III.D: N_b N_d = 1.5e4 operations at N_b = 5000 for 3 detectors,
    # against ~7.8e5 for the full-resolution sum of the 128 s segment.
    g = gwsynth.freq_grid(128.0, 20.0, 2048.0)
    e = H.bin_edges(g.freqs, 5000, 0)
    assert (len(e) - 1) * 3 == 15000
    assert abs(3 * g.n_freq - 7.8e5) / 7.8e5 < 0.01


def test_geometric_rule():
    f = gwsynth.freq_grid(128.0, 20.0, 2048.0).freqs
    e = H.bin_edges(f, 500, 1)
    r = f[e[1:]] / f[e[:-1]]
    assert np.allclose(r, (2048.0 / 20.0) ** (1 / 500), rtol=0.02)
