"""Pins of the oracle waveform against closed forms and textbook relations."""
import math

import numpy as np
import pytest

from oracle import waveform as W

TSUN = 4.925490947641267e-6


def _theta(mc=1.2, q=0.8, chi1=0.0, chi2=0.0, l1=0.0, l2=0.0, dl=100.0, iota=0.3,
           ra=1.0, dec=0.2, psi=0.4, phic=0.7, tc=0.01):
    return np.array([mc, q, chi1, chi2, l1, l2, dl, iota, ra, dec, psi, phic, tc])


def test_mass_relations_invert():
    # Independent route: component masses back to chirp mass and mass ratio.
    for mc, q in [(1.1, 0.5), (1.25, 0.8), (1.4, 1.0)]:
        eta, mtot, x1, x2, delta = W.masses(mc, q)
        m1, m2 = mtot * x1, mtot * x2
        assert math.isclose((m1 * m2) ** 0.6 / (m1 + m2) ** 0.2, mc, rel_tol=1e-14)
        assert math.isclose(m2 / m1, q, rel_tol=1e-14)
        assert math.isclose(delta, math.sqrt(1 - 4 * eta), rel_tol=1e-12, abs_tol=1e-15)


def test_newtonian_phase_closed_form():
    # P8: with all corrections removed, Psi depends on Mc alone:
    # Psi = 2 pi f tc - phic - pi/4 + 3/128 (pi Mc f)^(-5/3).
    f = np.linspace(20.0, 2048.0, 777)
    for q in (0.5, 0.9, 1.0):
        th = _theta(mc=1.3, q=q)
        got = W.phase(th, f, newtonian_only=True)
        want = (2 * math.pi * f * th[12] - th[11] - math.pi / 4
                + 3.0 / 128.0 * (math.pi * th[0] * TSUN * f) ** (-5.0 / 3.0))
        assert np.allclose(got, want, rtol=1e-13, atol=1e-9)


def test_stationary_phase_time_to_merger():
    # P10: dPsi/df = 2 pi tc - 2 pi t(f) with the leading-order chirp time
    # t(f) = 5/256 (pi f)^(-8/3) (Mc)^(-5/3) (Peters-Mathews), by central differences.
    th = _theta(mc=1.25, tc=0.05)
    f = np.array([20.0, 35.0, 80.0, 300.0, 1000.0])
    h = 1e-4 * f
    d = (W.phase(th, f + h, True) - W.phase(th, f - h, True)) / (2 * h)
    mcs = th[0] * TSUN
    t_f = 5.0 / 256.0 * (math.pi * f) ** (-8.0 / 3.0) * mcs ** (-5.0 / 3.0)
    assert np.allclose(d, 2 * math.pi * th[12] - 2 * math.pi * t_f, rtol=1e-6)
    # the signal lasts ~160 s from 20 Hz for a BNS (sanity of units)
    assert 100.0 < t_f[0] < 250.0


def test_tidal_equal_mass():
    # P9: q = 1, Lambda1 = Lambda2 = L gives Lambda-tilde = L, delta-Lambda-tilde = 0.
    eta, mtot, x1, x2, delta = W.masses(1.2, 1.0)
    for lam in (0.0, 400.0, 5000.0):
        lt, dlt = W.tidal_combinations(eta, delta, lam, lam)
        assert math.isclose(lt, lam, rel_tol=1e-14, abs_tol=1e-12)
        assert abs(dlt) < 1e-12 * max(lam, 1.0)


def test_tidal_mass_weighted_form():
    # Lambda-tilde in its mass-weighted form (Flanagan & Hinderer 2008):
    # 16/13 [(m1 + 12 m2) m1^4 L1 + (m2 + 12 m1) m2^4 L2] / M^5.
    for q, l1, l2 in [(0.5, 100.0, 3000.0), (0.8, 1234.0, 2345.0), (0.95, 0.0, 5000.0)]:
        eta, mtot, x1, x2, delta = W.masses(1.2, q)
        lt, _ = W.tidal_combinations(eta, delta, l1, l2)
        want = 16.0 / 13.0 * ((x1 + 12 * x2) * x1 ** 4 * l1 + (x2 + 12 * x1) * x2 ** 4 * l2)
        assert math.isclose(lt, want, rel_tol=1e-12)


def test_tidal_sign_reduces_phase_cycles():
    # Tidal terms enter with the sign that reduces the accumulated phase at high f.
    f = np.array([1000.0])
    th0 = _theta(l1=0.0, l2=0.0)
    th1 = _theta(l1=2000.0, l2=2000.0)
    d = W.phase(th1, f) - W.phase(th0, f)
    assert d[0] < 0


def test_amplitude_units_and_scaling():
    a1 = W.amplitude(1.2, 100.0)
    assert math.isclose(W.amplitude(1.2, 50.0), 2 * a1, rel_tol=1e-15)
    assert math.isclose(W.amplitude(2.4, 100.0) / a1, 2 ** (5.0 / 6.0), rel_tol=1e-14)


def test_polarization_relative_phase():
    # hx = -i cos(iota) / ((1 + cos^2 iota)/2) * h+, exactly.
    f = np.linspace(20.0, 500.0, 50)
    th = _theta(iota=1.0)
    hp, hc = W.polarizations(th, f)
    ci = math.cos(1.0)
    assert np.allclose(hc, -1j * ci / (0.5 * (1 + ci * ci)) * hp, rtol=1e-14)
    assert np.allclose(np.abs(hp), 0.5 * (1 + ci * ci) * W.amplitude(th[0], th[6]) * f ** (-7 / 6), rtol=1e-13)


@pytest.mark.parametrize("field", [2, 3])
def test_spin_terms_vanish_at_zero_spin(field):
    eta, mtot, x1, x2, delta = W.masses(1.2, 0.7)
    p0, l0 = W.pn_coefficients(eta, x1, x2, delta, 0.0, 0.0, spins=False)
    p1, l1 = W.pn_coefficients(eta, x1, x2, delta, 0.0, 0.0, spins=True)
    assert np.array_equal(p0, p1) and np.array_equal(l0, l1)
    args = [0.0, 0.0]
    args[field - 2] = 0.05
    p2, _ = W.pn_coefficients(eta, x1, x2, delta, *args)
    assert p2[3] > p0[3]  # aligned spin raises the 1.5PN coefficient
