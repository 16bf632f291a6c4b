"""TaylorF2 stand-in waveform, evaluated bin by bin in FP64.

The paper's templates come from a precessing tidal phenomenological model
(Sec. III.A).  Its stand-in here is the closed-form stationary-phase inspiral:
3.5PN point-particle phase with aligned-spin terms, 5PN and 6PN tidal terms,
and the leading-order (Newtonian) amplitude.  Conventions:

    h+(f) = A (1 + cos^2 iota) / 2 * f^(-7/6) * exp(-i Psi(f))
    hx(f) = -i A cos(iota)         * f^(-7/6) * exp(-i Psi(f))

    Psi(f) = 2 pi f t_c - phi_c - pi/4
             + 3 / (128 eta v^5) * [ sum_j (p_j + l_j ln v) v^j
                                     - 39/2 Lt v^10
                                     + (-3115/64 Lt + 6595/364 delta dLt) v^12 ]

with v = (pi M f)^(1/3), M the total mass in seconds.  Coefficients follow
the published TaylorF2 expressions (Buonanno et al. 2009 for the
point-particle terms, Arun et al. 2009 / Bohe et al. 2013 for aligned-spin
terms with unit spin-induced quadrupole, Wade et al. 2014 for the tidal
combinations).  No high-frequency cut-off is applied.
"""
from __future__ import annotations

import math

import numpy as np

MSUN_S = 4.925490947641267e-6          # G Msun / c^3 (s)
C_SI = 299792458.0                      # m / s
MPC_SI = 3.085677581491367e22           # m
EULER_GAMMA = 0.5772156649015329


def masses(mc: float, q: float):
    """Symmetric mass ratio, total mass (Msun), fractions X1 >= X2, delta = X1 - X2."""
    m1 = 1.0 / (1.0 + q)
    m2 = q / (1.0 + q)
    eta = m1 * m2
    mtot = mc / eta ** 0.6
    return eta, mtot, m1, m2, m1 - m2


def tidal_combinations(eta: float, delta: float, lam1: float, lam2: float):
    """Effective tidal parameters (Lambda-tilde, delta-Lambda-tilde), Wade et al. 2014."""
    lp = lam1 + lam2
    lm = lam1 - lam2
    lt = (8.0 / 13.0) * ((1.0 + 7.0 * eta - 31.0 * eta ** 2) * lp
                         + delta * (1.0 + 9.0 * eta - 11.0 * eta ** 2) * lm)
    dlt = 0.5 * (delta * (1.0 - 13272.0 / 1319.0 * eta + 8944.0 / 1319.0 * eta ** 2) * lp
                 + (1.0 - 15910.0 / 1319.0 * eta + 32850.0 / 1319.0 * eta ** 2
                    + 3380.0 / 1319.0 * eta ** 3) * lm)
    return lt, dlt


def pn_coefficients(eta, x1, x2, delta, chi1, chi2, spins=True):
    """(p[0..7], l[0..7]) such that the bracket is sum_j (p_j + l_j ln v) v^j."""
    pi = math.pi
    p = np.zeros(8)
    l = np.zeros(8)
    p[0] = 1.0
    p[2] = 3715.0 / 756.0 + 55.0 / 9.0 * eta
    p[3] = -16.0 * pi
    p[4] = 15293365.0 / 508032.0 + 27145.0 / 504.0 * eta + 3085.0 / 72.0 * eta ** 2
    p5 = pi * (38645.0 / 756.0 - 65.0 / 9.0 * eta)
    p[6] = (11583231236531.0 / 4694215680.0 - 640.0 / 3.0 * pi ** 2
            - 6848.0 / 21.0 * EULER_GAMMA - 6848.0 / 21.0 * math.log(4.0)
            + (-15737765635.0 / 3048192.0 + 2255.0 / 12.0 * pi ** 2) * eta
            + 76055.0 / 1728.0 * eta ** 2 - 127825.0 / 1296.0 * eta ** 3)
    l[6] = -6848.0 / 21.0
    p[7] = pi * (77096675.0 / 254016.0 + 378515.0 / 1512.0 * eta - 74045.0 / 756.0 * eta ** 2)
    if spins:
        # 1.5PN spin-orbit, written per body: chi_i (113 X_i^2 + 75 eta) / 3.
        p[3] += (chi1 * (113.0 * x1 * x1 + 75.0 * eta) + chi2 * (113.0 * x2 * x2 + 75.0 * eta)) / 3.0
        sl = x1 * x1 * chi1 + x2 * x2 * chi2
        dsl = delta * (x2 * chi2 - x1 * chi1)
        # 2PN spin-spin (aligned, unit spin-induced quadrupole).
        sigma = 79.0 / 8.0 * eta * chi1 * chi2 + 81.0 / 16.0 * (x1 * x1 * chi1 * chi1 + x2 * x2 * chi2 * chi2)
        p[4] -= 10.0 * sigma
        # 2.5PN spin-orbit enters both the constant and the log coefficient.
        gam = (554345.0 / 1134.0 + 110.0 / 9.0 * eta) * sl + (13915.0 / 84.0 - 10.0 / 3.0 * eta) * dsl
        p5 -= gam
        # 3PN and 3.5PN spin-orbit.
        p[6] += pi * (3760.0 * sl + 1490.0 * dsl) / 3.0
        p[7] += ((-8980424995.0 / 762048.0 + 6586595.0 / 756.0 * eta - 305.0 / 36.0 * eta ** 2) * sl
                 - (170978035.0 / 48384.0 - 2876425.0 / 672.0 * eta - 4735.0 / 144.0 * eta ** 2) * dsl)
    p[5] = p5
    l[5] = 3.0 * p5
    return p, l


def phase(theta: np.ndarray, f: np.ndarray, newtonian_only: bool = False) -> np.ndarray:
    """Psi(f) in radians for one parameter vector (13 columns), FP64, per bin."""
    mc, q, chi1, chi2, lam1, lam2 = (float(x) for x in theta[:6])
    phic, tc = float(theta[11]), float(theta[12])
    eta, mtot, x1, x2, delta = masses(mc, q)
    f = np.asarray(f, dtype=np.float64)
    v = np.cbrt(math.pi * mtot * MSUN_S * f)
    if newtonian_only:
        bracket = np.ones_like(v)
    else:
        p, l = pn_coefficients(eta, x1, x2, delta, chi1, chi2)
        lnv = np.log(v)
        bracket = np.zeros_like(v)
        for j in range(8):
            bracket += (p[j] + l[j] * lnv) * v ** j
        lt, dlt = tidal_combinations(eta, delta, lam1, lam2)
        bracket += -19.5 * lt * v ** 10 + (-3115.0 / 64.0 * lt + 6595.0 / 364.0 * delta * dlt) * v ** 12
    return 2.0 * math.pi * f * tc - phic - 0.25 * math.pi + 3.0 / (128.0 * eta * v ** 5) * bracket


def amplitude(mc: float, dl_mpc: float) -> float:
    """Leading-order stationary-phase amplitude A (units s^(-1/6)) of a face-on source."""
    return (math.sqrt(5.0 / 24.0) * math.pi ** (-2.0 / 3.0)
            * C_SI / (dl_mpc * MPC_SI) * (mc * MSUN_S) ** (5.0 / 6.0))


def polarizations(theta: np.ndarray, f: np.ndarray, newtonian_only: bool = False):
    """(h+, hx) complex arrays on the frequencies ``f``."""
    f = np.asarray(f, dtype=np.float64)
    a = amplitude(float(theta[0]), float(theta[6]))
    ci = math.cos(float(theta[7]))
    base = a * f ** (-7.0 / 6.0) * np.exp(-1j * phase(theta, f, newtonian_only))
    return 0.5 * (1.0 + ci * ci) * base, -1j * ci * base
