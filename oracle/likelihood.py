"""Matched-filter log-likelihood and its analytic marginalisations (FP64).

Sec. III.A, Eq. (loglike):  log L = -1/2 sum_i <d_i - h_i | d_i - h_i>_i  with
<a|b>_i = 4 Re int a* b / S_i df.  On the uniform grid the integral is the
Riemann sum 4 df Re sum_k a_k* b_k / S_ik over every bin of the band.

Marginalisations (Sec. III.A and the grid-marginalisation appendix):
* coalescence phase, uniform on [0, 2 pi): with Z = sum_i 4 df sum_k
  d_ik* h_ik / S_ik evaluated at phi_c = 0 (h carries exp(+i phi_c)),
  log L = -<d|d>/2 - <h|h>/2 + ln I0(|Z|);
* distance on a grid d_j with normalised log-weights w_j of a d^2 prior:
  log L = -<d|d>/2 + logsumexp_j [ w_j - <h|h>_1 / (2 d_j^2) + ln I0(|Z_1| / d_j) ]
  where the subscript 1 means the template at d_L = 1 Mpc;
* coalescence time together with the phase, uniform on [-W, W] (the
  appendix's grid sum over time shifts, which the paper evaluates by FFT on
  the uniform grid and calls dense): on the grid t_j = j delta / R,
  |j| <= J R, J = floor(W / delta), with delta = T / N, T = 1 / df and N the
  smallest power of two >= 2 (k0 + n_freq - 1) (the sampling interval of the
  segment) and R = 4 (the oversampling: on the plain sampling interval the
  grid sum of I0(|Z|) misses the integral by tens of nats for loud signals),
  log L = -<d|d>/2 - <h|h>/2 + ln[ (1 / N_t) sum_j I0(|Z(t_j)|) ],
  Z(t) the phase-free overlap of the template shifted by t (h -> h exp(-2 pi i f t)),
  the template evaluated at t_c = 0.

Problems are any object with attributes k0, n_freq, df, data [n_det, n_freq]
complex, psd [n_det, n_freq], det_tensor [n_det, 3, 3], det_pos [n_det, 3],
gmst, dist_grid, dist_logw.
"""
from __future__ import annotations

import math
import os

import numpy as np
from scipy.special import i0e, logsumexp

from . import detector, waveform

PLAIN, PHASE, PHASE_DIST, PHASE_TIME = 0, 1, 2, 3
TIME_WINDOW = 0.1  # half-width (s) of the uniform t_c prior that PHASE_TIME marginalises
TIME_OVERSAMPLE = 4  # grid points per sampling interval of the segment


def freqs(prob) -> np.ndarray:
    return (prob.k0 + np.arange(prob.n_freq, dtype=np.float64)) * prob.df


def inner(a: np.ndarray, b: np.ndarray, psd: np.ndarray, df: float) -> float:
    """<a|b> = 4 df Re sum_k conj(a_k) b_k / S_k."""
    return 4.0 * df * float(np.sum((np.conj(a) * b / psd).real))


def strain(theta: np.ndarray, prob, newtonian_only: bool = False) -> np.ndarray:
    """Projected templates h_i(f) [n_det, n_freq] for one parameter vector."""
    f = freqs(prob)
    hp, hc = waveform.polarizations(theta, f, newtonian_only)
    ra, dec, psi = float(theta[8]), float(theta[9]), float(theta[10])
    out = np.empty((prob.data.shape[0], f.size), dtype=np.complex128)
    for i in range(out.shape[0]):
        fp, fx = detector.antenna_pattern(prob.det_tensor[i], ra, dec, psi, prob.gmst)
        dt = detector.time_delay(prob.det_pos[i], ra, dec, prob.gmst)
        out[i] = (fp * hp + fx * hc) * np.exp(-2j * math.pi * f * dt)
    return out


def log_i0(x):
    """ln I0(x) for x >= 0, through the exponentially scaled Bessel function."""
    x = np.asarray(x, dtype=np.float64)
    return x + np.log(i0e(x))


def is_physical(theta: np.ndarray, marg: int) -> bool:
    th = np.asarray(theta, dtype=np.float64)
    if not np.all(np.isfinite(th)):
        return False
    if th[0] <= 0.0 or th[1] <= 0.0 or th[1] > 1.0:
        return False
    if abs(th[2]) >= 1.0 or abs(th[3]) >= 1.0:
        return False
    if marg != PHASE_DIST and th[6] <= 0.0:
        return False
    return True


def data_inner(prob) -> float:
    """sum_i <d_i|d_i>."""
    return sum(inner(prob.data[i], prob.data[i], prob.psd[i], prob.df) for i in range(prob.data.shape[0]))


def overlap(theta: np.ndarray, prob):
    """(Z, <h|h>) summed over detectors: Z = sum_i 4 df sum_k d_ik* h_ik / S_ik."""
    h = strain(np.asarray(theta, dtype=np.float64), prob)
    z = 0j
    hh = 0.0
    for i in range(h.shape[0]):
        z += 4.0 * prob.df * np.sum(np.conj(prob.data[i]) * h[i] / prob.psd[i])
        hh += inner(h[i], h[i], prob.psd[i], prob.df)
    return complex(z), hh


def time_grid(prob, window: float | None = None, oversample: int | None = None) -> np.ndarray:
    """Time shifts t_j = j delta / R, |j| <= J R (TIME_WINDOW and
    TIME_OVERSAMPLE by default; see the module docstring)."""
    if window is None:
        window = TIME_WINDOW
    if oversample is None:
        oversample = TIME_OVERSAMPLE
    top = 2 * (int(prob.k0) + int(prob.n_freq) - 1)
    n = 1
    while n < top:
        n *= 2
    delta = 1.0 / (n * prob.df)
    jmax = int(math.floor(window / delta + 1e-9)) * int(oversample)
    return np.arange(-jmax, jmax + 1, dtype=np.float64) * (delta / oversample)


def overlap_weights(theta: np.ndarray, prob):
    """a_k = sum_i 4 df d_ik* h_ik / S_ik (so that Z = sum_k a_k) and <h|h>."""
    h = strain(np.asarray(theta, dtype=np.float64), prob)
    a = np.zeros(prob.n_freq, dtype=np.complex128)
    hh = 0.0
    for i in range(h.shape[0]):
        a += 4.0 * prob.df * np.conj(prob.data[i]) * h[i] / prob.psd[i]
        hh += inner(h[i], h[i], prob.psd[i], prob.df)
    return a, hh


def time_shifted_overlaps(a: np.ndarray, prob, t: np.ndarray, rows: int = 16) -> np.ndarray:
    """Z(t_j) = sum_k a_k exp(-2 pi i f_k t_j), by direct summation."""
    f = freqs(prob)
    out = np.empty(t.size, dtype=np.complex128)
    for j0 in range(0, t.size, rows):
        tt = t[j0:j0 + rows]
        out[j0:j0 + rows] = np.exp(-2j * math.pi * np.outer(tt, f)) @ a
    return out


def loglike(theta: np.ndarray, prob, marg: int = PLAIN, dd: float | None = None) -> float:
    """Log-likelihood of one parameter vector in marginalisation mode ``marg``."""
    if not is_physical(theta, marg):
        return -math.inf
    if dd is None:
        dd = data_inner(prob)
    th = np.array(theta, dtype=np.float64)
    if marg == PLAIN:
        h = strain(th, prob)
        out = -0.5 * dd
        for i in range(h.shape[0]):
            out += inner(prob.data[i], h[i], prob.psd[i], prob.df)
            out -= 0.5 * inner(h[i], h[i], prob.psd[i], prob.df)
        return out
    th[11] = 0.0
    if marg == PHASE_TIME:
        th[12] = 0.0
        a, hh = overlap_weights(th, prob)
        t = time_grid(prob)
        z = time_shifted_overlaps(a, prob, t)
        return -0.5 * dd - 0.5 * hh + float(logsumexp(log_i0(np.abs(z)))) - math.log(t.size)
    if marg == PHASE_DIST:
        th[6] = 1.0
    z, hh = overlap(th, prob)
    if marg == PHASE:
        return -0.5 * dd - 0.5 * hh + float(log_i0(abs(z)))
    d = np.asarray(prob.dist_grid, dtype=np.float64)
    terms = np.asarray(prob.dist_logw) - 0.5 * hh / (d * d) + log_i0(abs(z) / d)
    return -0.5 * dd + float(logsumexp(terms))


def loglike_direct(theta: np.ndarray, prob) -> float:
    """-1/2 sum_i <d_i - h_i | d_i - h_i>, unexpanded (for small checks)."""
    if not is_physical(theta, PLAIN):
        return -math.inf
    h = strain(np.asarray(theta, dtype=np.float64), prob)
    r = prob.data - h
    return -0.5 * sum(inner(r[i], r[i], prob.psd[i], prob.df) for i in range(r.shape[0]))


_POOL_PROB = None


def _pool_init(prob):
    global _POOL_PROB
    _POOL_PROB = prob


def _pool_eval(args):
    theta, marg, dd = args
    return loglike(theta, _POOL_PROB, marg, dd)


def loglike_many(thetas: np.ndarray, prob, marg: int = PLAIN, processes: int | None = 1) -> np.ndarray:
    """Evaluate many parameter vectors; ``processes`` > 1 uses a process pool."""
    thetas = np.asarray(thetas, dtype=np.float64)
    dd = data_inner(prob)
    if processes is None:
        processes = len(os.sched_getaffinity(0))
    if processes <= 1 or len(thetas) < 2:
        return np.array([loglike(t, prob, marg, dd) for t in thetas])
    import multiprocessing as mp
    ctx = mp.get_context("fork")
    with ctx.Pool(processes, initializer=_pool_init, initargs=(prob,)) as pool:
        res = pool.map(_pool_eval, [(t, marg, dd) for t in thetas], chunksize=max(1, len(thetas) // (4 * processes)))
    return np.array(res)
