"""Post-hoc reconstruction of the marginalised distance and phase (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Grid-marginalisation appendix: a parameter that the likelihood marginalises is
recovered after the run.  For each posterior sample, the sample's inner
products give the conditional posterior of the marginalised parameters on
their grid, and one value is drawn from that conditional.  For the
phase+distance marginal of Sec. III.A, with the template carrying
exp(+i phi_c), Z_1 the overlap and <h|h>_1 the norm at d_L = 1 Mpc, phi_c = 0,
and w_j the normalised log-weights of the d^2 prior on the distance grid:

    p(d_j, phi | theta, data)  ∝  exp(w_j - <h|h>_1 / (2 d_j^2) + Re(Z_1 e^{i phi}) / d_j).

The pair is drawn in two stages:
  * d_j from its marginal on the distance grid,
        ∝ exp(w_j - <h|h>_1 / (2 d_j^2)) I0(|Z_1| / d_j)
    (the terms of the distance-marginal log-sum-exp);
  * phi given d_j from exp(kappa cos(phi + arg Z_1)), kappa = |Z_1| / d_j,
    on the uniform phase grid phi_m = 2 pi m / N_phi.  This is the dense-grid
    form of the phase marginal that Sec. III.A names as an equivalent of the
    Bessel function.

With the phase marginal alone (d_L sampled), only the phase is drawn, from the
overlap at the sample's own d_L.  Each draw inverts the CDF of the grid
weights: it takes the first grid index whose cumulative weight exceeds u times
the total.

Reading (the paper gives no draw rule): the drawn values are the grid nodes
themselves, so that the credible levels of reconstructed parameters are
quantised by the grid, as the appendix notes.

With the phase and coalescence time marginalised (d_L sampled), the pair
(t_c, phi_c) is drawn the same way.  t_c = t_j comes from the time grid of the
marginal with weights exp(-<h|h>(t_j)/2 + ln I0(|Z(t_j)|)), Z(t_j) the overlap
of the template shifted by t_j (its norm depends on t_j only for the
heterodyned bins).  Then phi_c comes from exp(|Z(t_j)| cos(phi + arg Z(t_j))).
"""
from __future__ import annotations

import math

import numpy as np

from . import heterodyne, likelihood

N_PHASE = 2048  # default size of the phase grid


def draw_index(logw, u: float) -> int:
    """First index j with sum_{i <= j} w_i > u sum_i w_i (w = exp(logw))."""
    logw = np.asarray(logw, dtype=np.float64)
    w = np.exp(logw - np.max(logw))
    c = np.cumsum(w)
    j = int(np.searchsorted(c, u * c[-1], side="right"))
    if j >= c.size:  # u * total rounded up to the total
        j = int(np.nonzero(w > 0.0)[0][-1])
    return j


def distance_logweights(z1: complex, hh1: float, prob) -> np.ndarray:
    """Log-weights of the distance conditional on the grid."""
    d = np.asarray(prob.dist_grid, dtype=np.float64)
    return np.asarray(prob.dist_logw, dtype=np.float64) - 0.5 * hh1 / (d * d) + likelihood.log_i0(abs(z1) / d)


def phase_grid(n_phase: int) -> np.ndarray:
    return 2.0 * math.pi * np.arange(n_phase, dtype=np.float64) / n_phase


def phase_logweights(z: complex, n_phase: int) -> np.ndarray:
    """Log-weights kappa cos(phi_m + arg z) of the phase conditional, kappa = |z|."""
    return abs(z) * np.cos(phase_grid(n_phase) + np.angle(z))


def sample_overlap(theta, prob, marg: int, het=None):
    """(Z, <h|h>) of one sample, summed over detectors: at d_L = 1 Mpc for the
    distance marginal, at the sample's d_L otherwise; phi_c = 0."""
    th = np.array(theta, dtype=np.float64)
    th[11] = 0.0
    if marg == likelihood.PHASE_DIST:
        th[6] = 1.0
    if het is None:
        return likelihood.overlap(th, prob)
    z, hh = heterodyne.overlaps(th, prob, het)
    return complex(np.sum(z)), float(np.sum(hh))


def reconstruct(theta, prob, u, marg: int = likelihood.PHASE_DIST, n_phase: int = N_PHASE, het=None):
    """(d_L, phi_c, j, m) drawn for one sample with uniforms u = (u_d, u_phi).

    j is the distance-grid index (-1 when d_L is the sample's own) and m the
    phase-grid index.  Unphysical samples give NaN values and indices -1.
    """
    if marg not in (likelihood.PHASE, likelihood.PHASE_DIST):
        raise ValueError("reconstruction needs the phase or phase+distance marginal")
    if not likelihood.is_physical(theta, marg):
        return math.nan, math.nan, -1, -1
    z, hh = sample_overlap(theta, prob, marg, het)
    if marg == likelihood.PHASE_DIST:
        j = draw_index(distance_logweights(z, hh, prob), float(u[0]))
        d = float(prob.dist_grid[j])
        zc = z / d
    else:
        j, d, zc = -1, float(theta[6]), z
    m = draw_index(phase_logweights(zc, n_phase), float(u[1]))
    return d, 2.0 * math.pi * m / n_phase, j, m


def time_conditional(theta, prob, het=None):
    """(t_j, Z(t_j), <h|h>(t_j)) on the time grid of the marginal, for the
    template with phi_c = 0 shifted by t_j."""
    th = np.array(theta, dtype=np.float64)
    th[11] = 0.0
    th[12] = 0.0
    t = likelihood.time_grid(prob)
    if het is None:
        a, hh = likelihood.overlap_weights(th, prob)
        z = likelihood.time_shifted_overlaps(a, prob, t)
        return t, z, np.full(t.size, hh)
    z = np.empty(t.size, dtype=np.complex128)
    hh = np.empty(t.size)
    for j, tj in enumerate(t):
        th[12] = tj
        zi, hhi = heterodyne.overlaps(th, prob, het)
        z[j], hh[j] = complex(np.sum(zi)), float(np.sum(hhi))
    return t, z, hh


def time_logweights(z: np.ndarray, hh: np.ndarray) -> np.ndarray:
    return -0.5 * np.asarray(hh) + likelihood.log_i0(np.abs(z))


def reconstruct_time(theta, prob, u, n_phase: int = N_PHASE, het=None):
    """(t_c, phi_c, j, m) drawn for one sample of the phase+time marginal with
    uniforms u = (u_t, u_phi); j indexes the time grid from its first point.
    Unphysical samples give NaN values and indices -1."""
    if not likelihood.is_physical(theta, likelihood.PHASE_TIME):
        return math.nan, math.nan, -1, -1
    t, z, hh = time_conditional(theta, prob, het)
    j = draw_index(time_logweights(z, hh), float(u[0]))
    m = draw_index(phase_logweights(z[j], n_phase), float(u[1]))
    return float(t[j]), 2.0 * math.pi * m / n_phase, j, m
