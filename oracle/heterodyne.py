"""Heterodyned (relative-binning) likelihood, FP64, step by step.

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this module; the library never does.

What is computed (Sec. III.D, which points to the relative-binning method of
Zackay, Dai & Venumadhav 2018 for the details).  A fiducial template h0 is
fixed once, close to where the likelihood peaks.  Per detector, the data and
h0 are folded into a handful of sums per coarse frequency bin (the summary
data); the bins are wide where the waveform's phase changes slowly and narrow
where it changes fast, with one bin grid for all detectors.  For a template
h, only the ratio r_i = h_i / h0_i is needed, and only at the bin edges: it
is treated as a straight line across each bin.  The binned Z and <h|h> then
feed the same log L and marginalisation formulae as the full-band sums.  The
steps here:

1. Phase bound Phi(f) = sum_g sgn(g) (f / f*_g)^g over
   g in {-5/3, -2/3, 1, 5/3, 7/3}, f*_g = f_max for g > 0 else f_min; it is
   monotone increasing on the band.
2. Edges f_j = Phi^-1(Phi(f_min) + j [Phi(f_max) - Phi(f_min)] / N_b),
   j = 0..N_b, by monotone interpolation on the fine grid, snapped to the
   nearest fine-grid frequency (duplicates removed, so fewer bins can result).
   Rule 1 instead spaces the edges geometrically.
3. Summary data per detector i and bin b = [f_lo, f_hi) (the last bin also
   holds f_max), with bin centre f_c = (f_lo + f_hi) / 2:
   A0 = 4 df sum d* h0 / S,  A1 = 4 df sum d* h0 / S (f - f_c),
   B0 = 4 df sum |h0|^2 / S, B1 = 4 df sum |h0|^2 / S (f - f_c).
4. Evaluation: r_i at the edges, r0 = (r_lo + r_hi) / 2,
   r1 = (r_hi - r_lo) / (f_hi - f_lo);  Z_i = sum_b A0 r0 + A1 r1  and
   <h_i|h_i> = sum_b B0 |r0|^2 + 2 B1 Re(r0 conj(r1)) (the |r1|^2 term is
   dropped); then the marginalisation epilogue of the full-band likelihood.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.special import logsumexp

from . import detector, likelihood, waveform

GAMMAS = (-5.0 / 3.0, -2.0 / 3.0, 1.0, 5.0 / 3.0, 7.0 / 3.0)


def phase_bound(f: np.ndarray, f_min: float, f_max: float) -> np.ndarray:
    f = np.asarray(f, dtype=np.float64)
    out = np.zeros_like(f)
    for g in GAMMAS:
        fs = f_max if g > 0 else f_min
        out += math.copysign(1.0, g) * (f / fs) ** g
    return out


def bin_edges(freqs: np.ndarray, n_bins: int, rule: int = 0) -> np.ndarray:
    """Edge indices into the fine grid ``freqs`` (increasing, first 0, last N-1)."""
    f = np.asarray(freqs, dtype=np.float64)
    f_min, f_max = f[0], f[-1]
    if rule == 0:
        phi = phase_bound(f, f_min, f_max)
        targets = phi[0] + np.arange(n_bins + 1) * (phi[-1] - phi[0]) / n_bins
        fe = np.interp(targets, phi, f)
    elif rule == 1:
        fe = f_min * (f_max / f_min) ** (np.arange(n_bins + 1) / n_bins)
    else:
        raise ValueError("rule must be 0 or 1")
    idx = np.rint((fe - f_min) / (f[1] - f[0])).astype(np.int64)
    idx = np.clip(idx, 0, len(f) - 1)
    idx[0], idx[-1] = 0, len(f) - 1
    return np.unique(idx)


@dataclasses.dataclass
class HetData:
    edges: np.ndarray      # fine-grid indices [n_bins + 1]
    f_edges: np.ndarray    # [n_bins + 1]
    a0: np.ndarray         # complex [n_det, n_bins]
    a1: np.ndarray         # complex [n_det, n_bins]
    b0: np.ndarray         # real    [n_det, n_bins]
    b1: np.ndarray         # real    [n_det, n_bins]
    h0_edges: np.ndarray   # complex [n_det, n_bins + 1]
    theta0: np.ndarray


def setup(prob, theta0: np.ndarray, n_bins: int, rule: int = 0) -> HetData:
    """Bin edges and summary data for the reference parameters ``theta0``."""
    f = likelihood.freqs(prob)
    e = bin_edges(f, n_bins, rule)
    h0 = likelihood.strain(np.asarray(theta0, dtype=np.float64), prob)
    nb = len(e) - 1
    nd = h0.shape[0]
    a0 = np.zeros((nd, nb), dtype=np.complex128)
    a1 = np.zeros((nd, nb), dtype=np.complex128)
    b0 = np.zeros((nd, nb))
    b1 = np.zeros((nd, nb))
    for b in range(nb):
        lo, hi = e[b], e[b + 1]
        stop = hi + 1 if b == nb - 1 else hi
        sl = slice(lo, stop)
        fc = 0.5 * (f[lo] + f[hi])
        dfc = f[sl] - fc
        for i in range(nd):
            w = 4.0 * prob.df / prob.psd[i, sl]
            dh = np.conj(prob.data[i, sl]) * h0[i, sl] * w
            hh = np.abs(h0[i, sl]) ** 2 * w
            a0[i, b] = np.sum(dh)
            a1[i, b] = np.sum(dh * dfc)
            b0[i, b] = np.sum(hh)
            b1[i, b] = np.sum(hh * dfc)
    return HetData(edges=e, f_edges=f[e], a0=a0, a1=a1, b0=b0, b1=b1, h0_edges=h0[:, e],
                   theta0=np.array(theta0, dtype=np.float64))


def strain_at(theta: np.ndarray, prob, fe: np.ndarray) -> np.ndarray:
    """Projected templates h_i at the frequencies ``fe`` [n_det, len(fe)]."""
    hp, hc = waveform.polarizations(theta, fe)
    ra, dec, psi = float(theta[8]), float(theta[9]), float(theta[10])
    out = np.empty((prob.data.shape[0], len(fe)), dtype=np.complex128)
    for i in range(out.shape[0]):
        fp, fx = detector.antenna_pattern(prob.det_tensor[i], ra, dec, psi, prob.gmst)
        dt = detector.time_delay(prob.det_pos[i], ra, dec, prob.gmst)
        out[i] = (fp * hp + fx * hc) * np.exp(-2j * math.pi * fe * dt)
    return out


def overlaps(theta: np.ndarray, prob, het: HetData):
    """Per-detector binned (Z_i, <h_i|h_i>)."""
    h = strain_at(np.asarray(theta, dtype=np.float64), prob, het.f_edges)
    r = h / het.h0_edges
    r0 = 0.5 * (r[:, 1:] + r[:, :-1])
    r1 = (r[:, 1:] - r[:, :-1]) / np.diff(het.f_edges)[None, :]
    z = np.sum(het.a0 * r0 + het.a1 * r1, axis=1)
    hh = np.sum(het.b0 * np.abs(r0) ** 2 + 2.0 * het.b1 * (r0 * np.conj(r1)).real, axis=1)
    return z, hh


def loglike(theta: np.ndarray, prob, het: HetData, marg: int = likelihood.PLAIN, dd: float | None = None) -> float:
    if not likelihood.is_physical(theta, marg):
        return -math.inf
    if dd is None:
        dd = likelihood.data_inner(prob)
    th = np.array(theta, dtype=np.float64)
    if marg != likelihood.PLAIN:
        th[11] = 0.0
    if marg == likelihood.PHASE_DIST:
        th[6] = 1.0
    if marg == likelihood.PHASE_TIME:
        # the phase-marginal binned likelihood at every shift of the time grid
        # (template at t_c = t_j), averaged over the grid
        t = likelihood.time_grid(prob)
        vals = np.empty(t.size)
        for j, tj in enumerate(t):
            th[12] = tj
            z, hh = overlaps(th, prob, het)
            vals[j] = -0.5 * float(np.sum(hh)) + float(likelihood.log_i0(abs(complex(np.sum(z)))))
        return -0.5 * dd + float(logsumexp(vals)) - math.log(t.size)
    z, hh = overlaps(th, prob, het)
    hh_t = float(np.sum(hh))
    if marg == likelihood.PLAIN:
        return -0.5 * dd + float(np.sum(z.real)) - 0.5 * hh_t
    zt = abs(complex(np.sum(z)))
    if marg == likelihood.PHASE:
        return -0.5 * dd - 0.5 * hh_t + float(likelihood.log_i0(zt))
    d = np.asarray(prob.dist_grid, dtype=np.float64)
    terms = np.asarray(prob.dist_logw) - 0.5 * hh_t / (d * d) + likelihood.log_i0(zt / d)
    return -0.5 * dd + float(logsumexp(terms))


def loglike_many(thetas, prob, het: HetData, marg: int = likelihood.PLAIN) -> np.ndarray:
    dd = likelihood.data_inner(prob)
    return np.array([loglike(t, prob, het, marg, dd) for t in np.asarray(thetas, dtype=np.float64)])
