"""Pins of the oracle's post-hoc reconstruction of d_L and phi_c.

The two-stage draw (distance from its marginal, then the phase given the
distance) must reproduce the joint posterior of (d_L, phi_c) that the plain,
unmarginalised likelihood gives on the same grids.  That joint is computed here
by brute force, as -1/2 <d - h | d - h> with h evaluated at every (d_j, phi_m).
This pins the phase sign, the d^2 weights and the Bessel factor without using
the reconstruction's own formula.
"""
import copy
import math

import numpy as np
import pytest

import gwsynth
from oracle import heterodyne as H
from oracle import likelihood as L
from oracle import reconstruct as R


@pytest.fixture(scope="module")
def tiny_problem():
    """4 s, 20-40 Hz (81 bins x 3 detectors), PSD scale 1e-49, an injection
    at 120 Mpc, and a 40-point distance grid on [10, 200] Mpc."""
    prob = gwsynth.make_problem(4.0, 20.0, 40.0, psd_scale=1e-49)
    th = gwsynth.prior_draws(gwsynth.SEEDS["injection"], 1)[0]
    th[6] = 120.0
    prob.data = prob.data + L.strain(th, prob)
    prob.theta_inj = th
    dg, dw = gwsynth.distance_grid(40)
    prob.dist_grid, prob.dist_logw = dg, dw
    return prob


def test_draw_index_rule():
    logw = np.log([1.0, 2.0, 3.0, 4.0])  # cumulative 1, 3, 6, 10
    assert R.draw_index(logw, 0.0999) == 0
    assert R.draw_index(logw, 0.1) == 1  # first index whose cumulative weight exceeds u * total
    assert R.draw_index(logw, 0.2999) == 1
    assert R.draw_index(logw, 0.3) == 2
    assert R.draw_index(logw, 0.9999) == 3
    assert R.draw_index(logw + 1e3, 0.3) == 2  # shift invariance
    u = np.random.default_rng(0).uniform(size=200)
    assert all(R.draw_index(np.zeros(1000), v) == math.floor(v * 1000) for v in u)
    # zero-weight entries are never drawn
    lw = np.array([-np.inf, 0.0, -np.inf, 0.0, -np.inf])
    assert {R.draw_index(lw, v) for v in np.linspace(0.001, 0.999, 50)} == {1, 3}


def test_two_stage_draw_equals_brute_force_joint(tiny_problem):
    prob = tiny_problem
    n_phase = 512
    th = gwsynth.near_posterior(3, prob.theta_inj, 1, scale=0.3)[0]
    z1, hh1 = R.sample_overlap(th, prob, L.PHASE_DIST)
    d = np.asarray(prob.dist_grid)
    kappa_max = abs(z1) / d.min()
    # informative, and resolved by the phase grid: the N-point sum of
    # exp(kappa cos phi) differs from 2 pi I0(kappa) N / (2 pi) by about
    # exp(-N^2 / (2 kappa)) relative
    assert 5.0 < kappa_max and math.exp(-n_phase ** 2 / (2 * kappa_max)) < 1e-20
    # brute force: w_j + log L_plain(theta | d_j, phi_m), unexpanded residual form
    logp = np.empty((d.size, n_phase))
    phis = R.phase_grid(n_phase)
    for j, dj in enumerate(d):
        for m, ph in enumerate(phis):
            t = th.copy()
            t[6], t[11] = dj, ph
            logp[j, m] = prob.dist_logw[j] + L.loglike_direct(t, prob)
    joint = np.exp(logp - logp.max())
    joint /= joint.sum()
    pd = np.exp(R.distance_logweights(z1, hh1, prob) - R.distance_logweights(z1, hh1, prob).max())
    pd /= pd.sum()
    two = np.empty_like(joint)
    for j, dj in enumerate(d):
        pm = np.exp(R.phase_logweights(z1 / dj, n_phase) - np.max(R.phase_logweights(z1 / dj, n_phase)))
        two[j] = pd[j] * pm / pm.sum()
    assert np.max(np.abs(two - joint)) < 1e-10
    assert np.max(np.abs(pd - joint.sum(axis=1))) < 1e-10


def test_stratified_draws_reproduce_the_distance_conditional(tiny_problem):
    prob = tiny_problem
    th = prob.theta_inj.copy()
    z1, hh1 = R.sample_overlap(th, prob, L.PHASE_DIST)
    lw = R.distance_logweights(z1, hh1, prob)
    p = np.exp(lw - lw.max())
    p /= p.sum()
    n = 20000
    j = np.array([R.draw_index(lw, (i + 0.5) / n) for i in range(n)])
    hist = np.bincount(j, minlength=p.size) / n
    assert np.max(np.abs(hist - p)) <= 1.0 / n + 1e-12


def test_reconstruct_values_and_modes(tiny_problem):
    prob = tiny_problem
    th = prob.theta_inj.copy()
    d, phi, j, m = R.reconstruct(th, prob, (0.37, 0.81), L.PHASE_DIST, n_phase=512)
    assert d == prob.dist_grid[j] and phi == 2 * math.pi * m / 512
    # phase alone: d_L is the sample's, the draw at u = 1/2 sits near the mode -arg Z
    t = th.copy()
    t[6] = 60.0
    d2, phi2, j2, m2 = R.reconstruct(t, prob, (0.5, 0.5), L.PHASE, n_phase=2048)
    assert d2 == 60.0 and j2 == -1
    z, _ = R.sample_overlap(t, prob, L.PHASE)
    mode = (-np.angle(z)) % (2 * math.pi)
    gap = abs((phi2 - mode + math.pi) % (2 * math.pi) - math.pi)
    assert gap < 3.0 / math.sqrt(abs(z))  # within three widths of the von Mises conditional
    bad = th.copy()
    bad[1] = 1.5
    out = R.reconstruct(bad, prob, (0.5, 0.5), L.PHASE_DIST)
    assert math.isnan(out[0]) and math.isnan(out[1]) and out[2] == -1 and out[3] == -1
    with pytest.raises(ValueError):
        R.reconstruct(th, prob, (0.5, 0.5), L.PLAIN)


def test_heterodyned_reconstruction_at_the_fiducial(tiny_problem):
    # P14: at theta = theta0 the binned overlaps equal the full-band ones, so
    # the draws agree (the uniforms are kept away from CDF boundaries).
    prob = copy.copy(tiny_problem)
    het = H.setup(prob, prob.theta_inj, 20)
    th = prob.theta_inj.copy()
    for u in [(0.2113, 0.4567), (0.7321, 0.1234)]:
        a = R.reconstruct(th, prob, u, L.PHASE_DIST)
        b = R.reconstruct(th, prob, u, L.PHASE_DIST, het=het)
        assert a[2] == b[2] and a[3] == b[3]


def test_time_phase_draw_equals_brute_force_joint(tiny_problem, monkeypatch):
    # The phase+time marginal's pair (t_c, phi_c): the two-stage draw equals the
    # joint posterior of the unmarginalised likelihood on the time grid times a
    # 256-point phase grid, evaluated by brute force with t_c and phi_c set in
    # the parameter vector (this pins the sign of the time shift).
    prob = tiny_problem
    n_phase = 256
    monkeypatch.setattr(L, "TIME_WINDOW", 0.02)  # 2 sampling intervals a side, 4 points each
    th = gwsynth.near_posterior(4, prob.theta_inj, 1, scale=0.3)[0]
    th[6] = 150.0
    t, z, hh = R.time_conditional(th, prob)
    assert t.size == 17
    phis = R.phase_grid(n_phase)
    logp = np.empty((t.size, n_phase))
    for j, tj in enumerate(t):
        for m, ph in enumerate(phis):
            tt = th.copy()
            tt[12], tt[11] = tj, ph
            logp[j, m] = L.loglike_direct(tt, prob)
    joint = np.exp(logp - logp.max())
    joint /= joint.sum()
    pt = np.exp(R.time_logweights(z, hh) - R.time_logweights(z, hh).max())
    pt /= pt.sum()
    two = np.empty_like(joint)
    for j in range(t.size):
        pm = np.exp(R.phase_logweights(z[j], n_phase) - np.max(R.phase_logweights(z[j], n_phase)))
        two[j] = pt[j] * pm / pm.sum()
    assert np.max(np.abs(two - joint)) < 1e-10
    tc, phi, j, m = R.reconstruct_time(th, prob, (0.41, 0.77), n_phase)
    assert tc == t[j] and phi == 2 * math.pi * m / n_phase


def test_heterodyned_time_draw_at_the_fiducial(tiny_problem):
    # with the fiducial at t_c = 0 the binned overlaps at t_j = 0 equal the
    # full band's; the time weights agree closely near the peak
    prob = tiny_problem
    th = prob.theta_inj.copy()
    th[12] = 0.0
    het = H.setup(prob, th, 40)
    t, z, hh = R.time_conditional(th, prob)
    th_, zh, hhh = R.time_conditional(th, prob, het)
    j0 = int(np.argmin(np.abs(t)))
    assert abs(z[j0] - zh[j0]) < 1e-9 * abs(z[j0]) and abs(hh[j0] - hhh[j0]) < 1e-9 * hh[j0]
