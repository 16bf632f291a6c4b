"""Maximum-likelihood search for the heterodyne fiducial, plain FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The GW170817 section takes the reference parameters of the relative binning
from a maximum-likelihood optimisation over priors narrowed to the event
(and its limitations section notes that a deployment must find them).  Here
the optimiser is differential evolution, DE/rand/1/bin (Storn & Price 1997),
maximising a log-likelihood over a box [lo, hi] inside the sampler's unit
cube:
  * member i of generation g draws its uniforms from Philox4x64-10, counter
    (g, i, j / 4, 0), key (seed, 2), word j % 4, mapped as the slice step's:
      u_0, u_1, u_2  three distinct partners r1, r2, r3, all different from
                     i: k_1 = floor(u_0 (P - 1)) is the k_1-th index of
                     {0..P-1} without i, k_2 = floor(u_1 (P - 2)) the k_2-th
                     without {i, r1}, k_3 = floor(u_2 (P - 3)) the k_3-th
                     without {i, r1, r2} (indices in increasing order);
      u_3            jrand = floor(11 u_3), the coordinate always crossed;
      u_4 .. u_14    coordinate j is crossed when u_(4+j) < CR;
  * mutant v = x_r1 + F (x_r2 - x_r3); trial t_j = v_j where crossed, else
    x_ij; a trial coordinate outside [lo_j, hi_j] is reflected into the box
    (lo - t -> lo + (lo - t), hi + e -> hi - e) and then clipped to it;
  * selection: the trial replaces x_i when f(t) >= f(x_i); a trial whose f
    is NaN never replaces, and one that is not NaN replaces an incumbent
    whose f is NaN.
Random numbers the method draws come from the published counter-based
generator, so that the device and this reference draw the same ones.
"""
from __future__ import annotations

import math

import numpy as np

from .sampler import philox4x64

N_DE_UNIFORMS = 15


def de_uniforms(seed: int, gen: int, member: int) -> np.ndarray:
    out = np.empty(N_DE_UNIFORMS)
    for j in range(N_DE_UNIFORMS):
        if j % 4 == 0:
            block = philox4x64((gen, member, j // 4, 0), (seed, 2))
        out[j] = ((block[j % 4] >> 11) + 0.5) * 2.0 ** -53
    return out


def kth_excluding(k: int, excluded) -> int:
    """The k-th (from 0) non-negative integer not in ``excluded``."""
    r = k
    for e in sorted(excluded):
        if r >= e:
            r += 1
    return r


def de_partners(i: int, pop: int, u) -> tuple[int, int, int]:
    r1 = kth_excluding(int(math.floor(u[0] * (pop - 1))), [i])
    r2 = kth_excluding(int(math.floor(u[1] * (pop - 2))), [i, r1])
    r3 = kth_excluding(int(math.floor(u[2] * (pop - 3))), [i, r1, r2])
    return r1, r2, r3


def de_trial(x: np.ndarray, i: int, u, f_scale: float, cr: float, lo, hi) -> np.ndarray:
    """Trial vector of member i (see the module docstring)."""
    pop, dim = x.shape
    r1, r2, r3 = de_partners(i, pop, u)
    jrand = int(math.floor(u[3] * dim))
    t = x[i].copy()
    for j in range(dim):
        if j == jrand or u[4 + j] < cr:
            v = x[r1, j] + f_scale * (x[r2, j] - x[r3, j])
            if v < lo[j]:
                v = lo[j] + (lo[j] - v)
            elif v > hi[j]:
                v = hi[j] - (v - hi[j])
            t[j] = min(hi[j], max(lo[j], v))
    return t


def de_search(objective, x0: np.ndarray, generations: int, seed: int, f_scale: float = 0.6, cr: float = 0.9,
              lo=None, hi=None):
    """Run the search from population x0 [P, 11]; objective maps [n, 11]
    points to [n] log-likelihoods.  Returns (population, values,
    smallest |f(t) - f(x_i)| of any selection, best index)."""
    x = np.array(x0, dtype=np.float64)
    pop, dim = x.shape
    lo = np.zeros(dim) if lo is None else np.asarray(lo, dtype=np.float64)
    hi = np.ones(dim) if hi is None else np.asarray(hi, dtype=np.float64)
    fx = np.asarray(objective(x), dtype=np.float64)
    margin = math.inf
    for g in range(generations):
        t = np.array([de_trial(x, i, de_uniforms(seed, g, i), f_scale, cr, lo, hi) for i in range(pop)])
        ft = np.asarray(objective(t), dtype=np.float64)
        for i in range(pop):
            if np.isfinite(ft[i]) and np.isfinite(fx[i]):
                margin = min(margin, abs(ft[i] - fx[i]))
            if ft[i] >= fx[i] or (np.isnan(fx[i]) and not np.isnan(ft[i])):
                x[i], fx[i] = t[i], ft[i]
    fb = np.where(np.isnan(fx), -np.inf, fx)
    return x, fx, margin, int(np.argmax(fb))


def conditional_peak(z1: complex, hh1: float):
    """(d_L, phi_c) maximising the plain likelihood of a template with overlap
    z1 and norm hh1 at d_L = 1 Mpc, phi_c = 0:  Re(z1 e^{i phi}) / d - hh1 / (2 d^2)
    peaks at phi = -arg z1 and d = hh1 / |z1|."""
    return hh1 / abs(z1), (-np.angle(z1)) % (2.0 * math.pi)
