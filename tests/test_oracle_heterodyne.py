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


@pytest.mark.parametrize("rule,n_bins", [(0, 60), (1, 37)])
def test_linear_ratio_is_exact(loud_problem, monkeypatch, rule, n_bins):
    # Sec. III.D expands r_i = h_i / h0_i to first order in each bin.  With the
    # fiducial h0 = h(theta) / (alpha + beta f) the ratio is exactly linear in
    # f, so the expansion is exact: every binned Z_i equals the full-band sum,
    # and the binned <h_i|h_i> equals the full-band one once the dropped term
    # |r1|^2 4 df sum_k |h0_ik|^2 (f_k - f_c)^2 / S_ik is added back.  r1 = beta
    # is far from zero here, so the A1 and B1 terms (their signs, the bin
    # centre, the slope) carry a large share of both sums.
    prob = loud_problem
    th = prob.theta_inj.copy()
    alpha, beta = 1.0 + 0.2j, 1.5e-3 - 1.0e-3j  # beta per Hz: |beta f| reaches 0.9 at 512 Hz
    f = L.freqs(prob)
    true_strain = L.strain
    h = true_strain(th, prob)
    h0 = h / (alpha + beta * f)[None, :]
    monkeypatch.setattr(L, "strain", lambda theta, p, *a, **k: h0)
    het = H.setup(prob, th, n_bins, rule)
    monkeypatch.undo()
    z_bin, hh_bin = H.overlaps(th, prob, het)
    e = het.edges
    nb = len(e) - 1
    for i in range(h.shape[0]):
        w = 4.0 * prob.df / prob.psd[i]
        z_full = np.sum(np.conj(prob.data[i]) * h[i] * w)
        hh_full = np.sum(np.abs(h[i]) ** 2 * w)
        scale = np.sum(np.abs(prob.data[i]) * np.abs(h[i]) * w)
        assert abs(z_bin[i] - z_full) < 1e-11 * scale, (i, z_bin[i], z_full)
        b2 = 0.0
        for b in range(nb):
            stop = e[b + 1] + 1 if b == nb - 1 else e[b + 1]
            sl = slice(e[b], stop)
            fc = 0.5 * (f[e[b]] + f[e[b + 1]])
            b2 += np.sum(np.abs(h0[i, sl]) ** 2 * w[sl] * (f[sl] - fc) ** 2)
        assert abs(hh_bin[i] + abs(beta) ** 2 * b2 - hh_full) < 1e-11 * hh_full, (i, hh_bin[i], hh_full)
        # the pin has teeth: the first-order terms alone move Z_i and <h_i|h_i>
        # by ~1e-4 of their scale, seven orders above the tolerance
        r0 = alpha + beta * 0.5 * (het.f_edges[1:] + het.f_edges[:-1])
        assert abs(np.sum(het.a1[i] * beta)) > 1e-6 * scale
        assert abs(np.sum(2.0 * het.b1[i] * (r0 * np.conj(beta)).real)) > 1e-6 * hh_full
