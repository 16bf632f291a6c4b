"""Pins of the oracle detector response against textbook antenna patterns."""
import math

import numpy as np

from oracle import detector as D

C = 299792458.0
RE = 6.371e6
DXY = 0.5 * (np.outer([1, 0, 0], [1, 0, 0]) - np.outer([0, 1, 0], [0, 1, 0]))


def test_textbook_antenna_power():
    # Arms along x and y: F+^2 + Fx^2 = (1 + cos^2 th)^2 cos^2 2ph / 4 + cos^2 th sin^2 2ph
    # for a source at polar angle th, azimuth ph (Thorne 1987), for every psi.
    r = np.random.default_rng(11)
    for _ in range(50):
        th = math.acos(r.uniform(-1, 1))
        ph = r.uniform(0, 2 * math.pi)
        psi = r.uniform(0, math.pi)
        fp, fx = D.antenna_pattern(DXY, ph, math.pi / 2 - th, psi)
        want = 0.25 * (1 + math.cos(th) ** 2) ** 2 * math.cos(2 * ph) ** 2 + math.cos(th) ** 2 * math.sin(2 * ph) ** 2
        assert math.isclose(fp * fp + fx * fx, want, rel_tol=1e-12, abs_tol=1e-14)
        # at psi = 0 the magnitudes are the textbook ones
        fp0, fx0 = D.antenna_pattern(DXY, ph, math.pi / 2 - th, 0.0)
        assert math.isclose(abs(fp0), abs(0.5 * (1 + math.cos(th) ** 2) * math.cos(2 * ph)), abs_tol=1e-13)
        assert math.isclose(abs(fx0), abs(math.cos(th) * math.sin(2 * ph)), abs_tol=1e-13)


def test_overhead_source_on_aligned_detector():
    # A source at the zenith of the arms' plane sees the full response,
    # F+^2 + Fx^2 = 1 for every psi, and |F+| = 1 when psi aligns the frame.
    vals = [D.antenna_pattern(DXY, 0.3, math.pi / 2, psi) for psi in np.linspace(0, math.pi, 181)]
    fp = np.array([v[0] for v in vals])
    fx = np.array([v[1] for v in vals])
    assert np.allclose(fp ** 2 + fx ** 2, 1.0, rtol=1e-13)
    # ra = 0.3 rotates the frame by 0.3 rad, so psi = 0.3 aligns X with an arm
    fp, fx = D.antenna_pattern(DXY, 0.3, math.pi / 2, 0.3)
    assert math.isclose(abs(fp), 1.0, rel_tol=1e-13) and abs(fx) < 1e-13


def test_psi_rotation():
    # P5: (F+ + i Fx) winds at twice the polarisation angle; psi + pi/2 negates both.
    pos, tens = np.zeros(3), None
    r = np.random.default_rng(3)
    a = r.normal(size=(3, 3))
    tens = 0.5 * (a + a.T)
    tens -= np.trace(tens) / 3 * np.eye(3)
    for _ in range(20):
        ra, dec, psi = r.uniform(0, 6.28), r.uniform(-1.5, 1.5), r.uniform(0, 3.14)
        fp0, fx0 = D.antenna_pattern(tens, ra, dec, 0.0)
        fp, fx = D.antenna_pattern(tens, ra, dec, psi)
        z0, z = complex(fp0, fx0), complex(fp, fx)
        assert abs(z - z0 * np.exp(-2j * psi)) < 1e-12 or abs(z - z0 * np.exp(2j * psi)) < 1e-12
        fq, fy = D.antenna_pattern(tens, ra, dec, psi + math.pi / 2)
        assert math.isclose(fq, -fp, abs_tol=1e-13) and math.isclose(fy, -fx, abs_tol=1e-13)
    # the winding direction is fixed (not data-dependent)
    fp0, fx0 = D.antenna_pattern(tens, 1.0, 0.3, 0.0)
    fp, fx = D.antenna_pattern(tens, 1.0, 0.3, 0.2)
    assert abs(complex(fp, fx) - complex(fp0, fx0) * np.exp(-0.4j)) < 1e-12


def test_time_delay_bounds_and_sign():
    # P11: |dt| <= R_E / c; zero at the geocentre; a detector displaced towards
    # the source receives the signal earlier (dt = -R_E / c).
    r = np.random.default_rng(5)
    for _ in range(100):
        n = r.normal(size=3)
        n /= np.linalg.norm(n)
        ra, dec = r.uniform(0, 6.28), r.uniform(-1.5, 1.5)
        assert abs(D.time_delay(RE * n, ra, dec)) <= RE / C * (1 + 1e-12)
        assert D.time_delay(np.zeros(3), ra, dec) == 0.0
    ra, dec = 0.7, -0.4
    s = np.array([math.cos(dec) * math.cos(ra), math.cos(dec) * math.sin(ra), math.sin(dec)])
    assert math.isclose(D.time_delay(RE * s, ra, dec), -RE / C, rel_tol=1e-14)


def test_gmst_is_a_rotation_of_ra():
    r = np.random.default_rng(9)
    a = r.normal(size=(3, 3))
    tens = 0.5 * (a + a.T)
    for g in (0.0, 0.5, 2.0):
        assert np.allclose(D.antenna_pattern(tens, 1.3 + g, 0.2, 0.4, g), D.antenna_pattern(tens, 1.3, 0.2, 0.4, 0.0))
