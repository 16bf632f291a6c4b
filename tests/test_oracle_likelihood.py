"""Pins of the oracle likelihood: closed forms, invariants, brute force, quadrature."""
import copy
import math

import numpy as np
import pytest
from scipy import integrate

import gwsynth
from oracle import detector as D
from oracle import likelihood as L
from oracle import waveform as W


def _theta(**kw):
    th = gwsynth.prior_draws(21, 1)[0]
    names = gwsynth.PARAM_NAMES
    for k, v in kw.items():
        th[names.index(k)] = v
    return th


def test_hh_closed_form(small_problem):
    # P2: <h_i|h_i> = A^2 |P_i|^2 4 df sum_k f_k^(-7/3) / S_ik, with
    # P_i = F+ (1 + cos^2 iota)/2 - i Fx cos(iota); the network sum is rho^2.
    prob = small_problem
    f = prob.freqs
    for seed in range(4):
        th = gwsynth.prior_draws(100 + seed, 1)[0]
        h = L.strain(th, prob)
        a = W.amplitude(th[0], th[6])
        ci = math.cos(th[7])
        for i in range(3):
            fp, fx = D.antenna_pattern(prob.det_tensor[i], th[8], th[9], th[10])
            p2 = (fp * 0.5 * (1 + ci * ci)) ** 2 + (fx * ci) ** 2
            want = a * a * p2 * 4 * prob.df * np.sum(f ** (-7.0 / 3.0) / prob.psd[i])
            got = L.inner(h[i], h[i], prob.psd[i], prob.df)
            assert math.isclose(got, want, rel_tol=1e-12)


def test_distance_scaling(small_problem):
    # P3: <h|h> ~ 1/d^2 and Z ~ 1/d.
    th = _theta(dl=40.0)
    z1, hh1 = L.overlap(th, small_problem)
    th2 = th.copy()
    th2[6] = 160.0
    z2, hh2 = L.overlap(th2, small_problem)
    assert math.isclose(hh1 / hh2, 16.0, rel_tol=1e-13)
    assert abs(z1 / z2 - 4.0) < 1e-12


def test_phase_marginal_brute_force(loud_problem):
    # P4 (Sec. III.A: brute-force phase summation equals the Bessel form):
    # the PHASE log-likelihood is the log-mean-exp of PLAIN over a dense phi_c
    # grid (trapezoid on a periodic integrand), and PLAIN is a pure sinusoid.
    prob = loud_problem
    th = prob.theta_inj.copy()
    th[0] += 2e-5
    dd = L.data_inner(prob)
    n = 2048
    vals = []
    for j in range(n):
        t = th.copy()
        t[11] = 2 * math.pi * j / n
        vals.append(L.loglike(t, prob, L.PLAIN, dd))
    vals = np.array(vals)
    lme = np.max(vals) + math.log(np.mean(np.exp(vals - np.max(vals))))
    got = L.loglike(th, prob, L.PHASE, dd)
    assert abs(got - lme) < 1e-9 * max(1.0, abs(got))
    # |Z| is invariant under phi_c and PLAIN(phi) = c + |Z0| cos(phi + arg Z0)
    t0 = th.copy()
    t0[11] = 0.0
    z0, hh = L.overlap(t0, prob)
    c = -0.5 * dd - 0.5 * hh
    phis = 2 * math.pi * np.arange(n) / n
    assert np.allclose(vals, c + abs(z0) * np.cos(phis + np.angle(z0)), rtol=0, atol=1e-8 * abs(z0))
    t1 = th.copy()
    t1[11] = 1.234
    z1, _ = L.overlap(t1, prob)
    assert math.isclose(abs(z1), abs(z0), rel_tol=1e-12)


def test_noiseless_injection(small_problem):
    # P6: d = h(theta_inj) gives PLAIN logL(theta_inj) = 0 and logL(theta) <= 0.
    prob = copy.copy(small_problem)
    th = _theta(dl=15.0)
    prob.data = L.strain(th, prob)
    hh = L.data_inner(prob)
    assert abs(L.loglike(th, prob, L.PLAIN)) < 1e-12 * hh
    assert abs(L.loglike_direct(th, prob)) < 1e-12 * hh
    for s in range(5):
        other = gwsynth.prior_draws(300 + s, 1)[0]
        assert L.loglike(other, prob, L.PLAIN) <= 1e-12 * hh


def test_expanded_equals_direct(loud_problem):
    prob = loud_problem
    for s in range(3):
        th = gwsynth.near_posterior(40 + s, prob.theta_inj, 1)[0]
        a = L.loglike(th, prob, L.PLAIN)
        b = L.loglike_direct(th, prob)
        assert abs(a - b) < 1e-9 * max(1.0, L.data_inner(prob))


def test_noise_statistics(small_problem):
    # P7: E<n|n> = 2 N_f per detector; <n|h> ~ N(0, <h|h>) over noise seeds.
    prob = copy.copy(small_problem)
    th = _theta(dl=30.0)
    h = L.strain(th, prob)
    hh = sum(L.inner(h[i], h[i], prob.psd[i], prob.df) for i in range(3))
    nn, nh = [], []
    for seed in range(300):
        n = gwsynth.gaussian_noise(1000 + seed, prob.psd, prob.df)
        nn.append(L.inner(n[0], n[0], prob.psd[0], prob.df))
        nh.append(sum(L.inner(n[i], h[i], prob.psd[i], prob.df) for i in range(3)))
    nn, nh = np.array(nn), np.array(nh)
    n_f = prob.n_freq
    assert abs(nn.mean() - 2 * n_f) < 4 * math.sqrt(4 * n_f / 300)
    assert abs(nh.mean()) < 4 * math.sqrt(hh / 300)
    assert 0.75 < nh.var() / hh < 1.3


def test_time_shift_is_a_dft(small_problem):
    # P12: Z(t_c = j / (N df)) equals the length-N DFT of the per-bin products
    # at t_c = 0, times exp(-2 pi i k0 j / N).  Pins the Fourier sign of t_c.
    prob = small_problem
    th = _theta(tc=0.0, dl=20.0)
    h0 = L.strain(th, prob)
    c = sum(4 * prob.df * np.conj(prob.data[i]) * h0[i] / prob.psd[i] for i in range(3))
    n = prob.n_freq
    dft = np.fft.fft(c)
    for j in (1, 7, 100, n - 3):
        t = th.copy()
        t[12] = j / (n * prob.df)
        z, _ = L.overlap(t, prob)
        want = dft[j] * np.exp(-2j * math.pi * prob.k0 * j / n)
        assert abs(z - want) < 1e-9 * np.sum(np.abs(c))


def test_delay_equals_tc_shift(small_problem):
    # The detector delay acts exactly like a shift of t_c for that detector.
    prob = copy.copy(small_problem)
    th = _theta()
    h = L.strain(th, prob)
    for i in range(3):
        dt = D.time_delay(prob.det_pos[i], th[8], th[9])
        geo = copy.copy(prob)
        geo.det_pos = np.zeros_like(prob.det_pos)
        t2 = th.copy()
        t2[12] += dt
        hg = L.strain(t2, geo)
        assert np.allclose(h[i], hg[i], rtol=1e-9, atol=1e-9 * np.abs(h[i]).max())


def test_distance_marginal_vs_quadrature(loud_problem):
    # P15: grid log-sum-exp against adaptive quadrature of the same integral with
    # the continuous prior p(d) = 3 d^2 / (d_max^3 - d_min^3).
    prob = loud_problem
    dd = L.data_inner(prob)
    for s in range(3):
        th = gwsynth.near_posterior(60 + s, prob.theta_inj, 1)[0]
        got = L.loglike(th, prob, L.PHASE_DIST, dd)
        t1 = th.copy()
        t1[11] = 0.0
        t1[6] = 1.0
        z1, hh1 = L.overlap(t1, prob)
        zabs = abs(z1)
        lo, hi = 10.0, 200.0
        logs = [(-0.5 * hh1 / d ** 2 + float(L.log_i0(zabs / d))) for d in np.linspace(lo, hi, 4001)]
        m = max(logs)
        f = lambda d: 3 * d * d / (hi ** 3 - lo ** 3) * math.exp(-0.5 * hh1 / d ** 2 + float(L.log_i0(zabs / d)) - m)
        val, err = integrate.quad(f, lo, hi, limit=400, epsabs=0, epsrel=1e-12, points=[math.sqrt(hh1) / max(zabs, 1e-300)])
        want = -0.5 * dd + m + math.log(val)
        assert abs(got - want) < 2e-5, (got, want)


def test_log_i0_against_series():
    # ln I0 against its defining power series (small x) and the exponential
    # bound I0(x) <= e^x (large x).
    for x in (0.0, 0.1, 1.0, 5.0, 20.0):
        terms, t = [], 1.0
        for k in range(200):
            terms.append(t)
            t *= (x * x / 4) / ((k + 1) * (k + 1))
        s = math.fsum(terms)
        assert math.isclose(float(L.log_i0(x)), math.log(s), rel_tol=1e-13, abs_tol=1e-15)
    for x in (50.0, 700.0, 1e5):
        v = float(L.log_i0(x))
        assert x - 0.5 * math.log(2 * math.pi * x) < v < x


def test_unphysical_is_minus_inf(small_problem):
    th = _theta()
    for col, val in [(0, -1.0), (1, 1.5), (1, 0.0), (6, -3.0), (3, np.nan)]:
        t = th.copy()
        t[col] = val
        assert L.loglike(t, small_problem, L.PLAIN) == -math.inf
    t = th.copy()
    t[6] = -3.0  # distance column is ignored when marginalised
    assert np.isfinite(L.loglike(t, small_problem, L.PHASE_DIST))
