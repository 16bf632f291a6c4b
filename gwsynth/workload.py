"""Seeded synthetic inputs with the shapes of the paper's BNS workloads.

The paper analyses 128 s of three-detector data over 20-2048 Hz with a BNS
prior (Sec. IV.A, injection catalogue, Table I).  Its PSD files, detector
network and catalogue are not available, so every input here is drawn from a
fixed seed instead:

* a uniform frequency grid f_k = (k0 + k) df with both ends of the band
  included, k0 = ceil(f_min T), k1 = floor(f_max T);
* an analytic aLIGO-like PSD fit (prefactor exposed as ``psd_scale``);
* three detectors at seeded Earth-surface positions with seeded arm azimuths;
* circular complex Gaussian noise with Re, Im ~ N(0, S / (4 df)) per bin;
* prior draws of the 13-column parameter vector;
* a luminosity-distance grid with log-weights of a d_L^2 prior (Sec. III.A);
* an uneven split of a batch into sub-batches (sizes 100-8000).

Parameter vector columns, FP64, fixed order:
    [Mc (Msun, detector frame), q = m2/m1 <= 1, chi1, chi2, Lambda1, Lambda2,
     d_L (Mpc), iota, ra, dec, psi, phi_c, t_c (s)]
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

PARAM_NAMES = ("mc", "q", "chi1", "chi2", "lambda1", "lambda2", "dl",
               "iota", "ra", "dec", "psi", "phic", "tc")
N_PARAMS = len(PARAM_NAMES)

# Seeds of every random stream; recorded in every result.
SEEDS = dict(detectors=1, injection=2, noise=3, prior=4, split=5,
             sampler=6, mlp=7)

EARTH_RADIUS_M = 6.371e6

# Uniform prior ranges used for draws (configuration of the synthetic runs).
PRIOR = dict(mc=(1.1, 1.4), q=(0.5, 1.0), chi=(-0.05, 0.05),
             lam=(0.0, 5000.0), dl=(10.0, 200.0), tc=(-0.1, 0.1))


@dataclasses.dataclass(frozen=True)
class FreqGrid:
    k0: int
    n_freq: int
    df: float

    @property
    def freqs(self) -> np.ndarray:
        return (self.k0 + np.arange(self.n_freq, dtype=np.float64)) * self.df


def freq_grid(duration: float, f_min: float, f_max: float) -> FreqGrid:
    """Uniform grid of a ``duration``-second segment, both band edges included."""
    k0 = int(math.ceil(f_min * duration - 1e-9))
    k1 = int(math.floor(f_max * duration + 1e-9))
    return FreqGrid(k0=k0, n_freq=k1 - k0 + 1, df=1.0 / duration)


def psd_fit(f: np.ndarray, scale: float = 1e-46) -> np.ndarray:
    """Analytic aLIGO-shaped one-sided PSD, x = f / 215 Hz."""
    x = np.asarray(f, dtype=np.float64) / 215.0
    x2 = x * x
    return scale * (x ** -4.14 - 5.0 / x2
                    + 111.0 * (1.0 - x2 + 0.5 * x2 * x2) / (1.0 + 0.5 * x2))


def _unit(v):
    return v / np.linalg.norm(v)


def detectors(seed: int = SEEDS["detectors"], n_det: int = 3):
    """Seeded detector network: positions [n_det, 3] (m) and tensors [n_det, 3, 3].

    Each detector sits at a random point on a sphere of Earth radius; its two
    orthogonal unit arms lie in the local tangent plane at a random azimuth and
    its tensor is D = (x x^T - y y^T) / 2.
    """
    rng = np.random.default_rng(seed)
    pos = np.zeros((n_det, 3))
    tens = np.zeros((n_det, 3, 3))
    for i in range(n_det):
        n = _unit(rng.normal(size=3))
        pos[i] = EARTH_RADIUS_M * n
        e1 = _unit(np.cross([0.0, 0.0, 1.0], n))
        e2 = np.cross(n, e1)
        az = rng.uniform(0.0, 2.0 * np.pi)
        ax = math.cos(az) * e1 + math.sin(az) * e2
        ay = np.cross(n, ax)
        tens[i] = 0.5 * (np.outer(ax, ax) - np.outer(ay, ay))
    return pos, tens


def gaussian_noise(seed: int, psd: np.ndarray, df: float) -> np.ndarray:
    """Complex noise with independent Re, Im ~ N(0, S / (4 df)) per bin."""
    rng = np.random.default_rng(seed)
    sig = np.sqrt(psd / (4.0 * df))
    return sig * rng.standard_normal(psd.shape) + 1j * sig * rng.standard_normal(psd.shape)


def prior_draws(seed: int, n: int) -> np.ndarray:
    """``n`` draws [n, 13] of the uniform / isotropic synthetic prior."""
    rng = np.random.default_rng(seed)
    th = np.empty((n, N_PARAMS))
    th[:, 0] = rng.uniform(*PRIOR["mc"], n)
    th[:, 1] = rng.uniform(*PRIOR["q"], n)
    th[:, 2] = rng.uniform(*PRIOR["chi"], n)
    th[:, 3] = rng.uniform(*PRIOR["chi"], n)
    th[:, 4] = rng.uniform(*PRIOR["lam"], n)
    th[:, 5] = rng.uniform(*PRIOR["lam"], n)
    th[:, 6] = rng.uniform(*PRIOR["dl"], n)
    th[:, 7] = np.arccos(rng.uniform(-1.0, 1.0, n))
    th[:, 8] = rng.uniform(0.0, 2.0 * np.pi, n)
    th[:, 9] = np.arcsin(rng.uniform(-1.0, 1.0, n))
    th[:, 10] = rng.uniform(0.0, np.pi, n)
    th[:, 11] = rng.uniform(0.0, 2.0 * np.pi, n)
    th[:, 12] = rng.uniform(*PRIOR["tc"], n)
    return th


_NEAR_SIGMA = np.array([2e-5, 0.01, 0.002, 0.002, 50.0, 50.0, 2.0,
                        0.02, 0.005, 0.005, 0.02, 0.05, 5e-5])


def near_posterior(seed: int, theta0: np.ndarray, n: int, scale: float = 1.0) -> np.ndarray:
    """``n`` small seeded Gaussian perturbations of ``theta0``, kept in the prior box."""
    rng = np.random.default_rng(seed)
    th = theta0[None, :] + scale * _NEAR_SIGMA[None, :] * rng.standard_normal((n, N_PARAMS))
    th[:, 0] = np.clip(th[:, 0], *PRIOR["mc"])
    th[:, 1] = np.clip(th[:, 1], PRIOR["q"][0], PRIOR["q"][1])
    th[:, 2:4] = np.clip(th[:, 2:4], *PRIOR["chi"])
    th[:, 4:6] = np.clip(th[:, 4:6], *PRIOR["lam"])
    th[:, 6] = np.clip(th[:, 6], *PRIOR["dl"])
    th[:, 7] = np.clip(th[:, 7], 0.0, np.pi)
    th[:, 8] = np.mod(th[:, 8], 2.0 * np.pi)
    th[:, 9] = np.clip(th[:, 9], -0.5 * np.pi, 0.5 * np.pi)
    th[:, 10] = np.mod(th[:, 10], np.pi)
    th[:, 11] = np.mod(th[:, 11], 2.0 * np.pi)
    th[:, 12] = np.clip(th[:, 12], *PRIOR["tc"])
    return th


def distance_grid(n: int = 1000, d_min: float = PRIOR["dl"][0], d_max: float = PRIOR["dl"][1]):
    """Uniform d_L grid (Mpc) and normalised log-weights of a d_L^2 prior.

    The weights are trapezoid-rule weights times d^2, normalised so that the
    discrete prior sums to one.
    """
    d = np.linspace(d_min, d_max, n)
    w = np.full(n, (d_max - d_min) / (n - 1))
    w[0] *= 0.5
    w[-1] *= 0.5
    p = w * d * d
    return d, np.log(p) - np.log(p.sum())


def uneven_split(seed: int, total: int, lo: int = 100, hi: int = 8000) -> np.ndarray:
    """Offsets [n_sub + 1] of an uneven split of ``total`` items.

    Sizes are drawn uniformly from {lo..hi} until they cover ``total``; the
    last one is cut to fit and merged into its neighbour if it falls below
    ``lo``.
    """
    rng = np.random.default_rng(seed)
    sizes = []
    acc = 0
    while acc < total:
        s = int(rng.integers(lo, hi + 1))
        s = min(s, total - acc)
        sizes.append(s)
        acc += s
    if len(sizes) > 1 and sizes[-1] < lo:
        sizes[-2] += sizes.pop()
    return np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)


# Workload shapes of the synthetic runs.
CONFIGS = {
    "cfg1": dict(duration=8.0, f_min=20.0, f_max=512.0, batch=1024, psd_scale=1e-46),
    "cfg2": dict(duration=128.0, f_min=20.0, f_max=2048.0, batch=4096, psd_scale=1e-46),
    "cfg3": dict(duration=128.0, f_min=20.0, f_max=2048.0, batch=65536, psd_scale=1e-46,
                 n_bins=500),
}


@dataclasses.dataclass
class Problem:
    """Everything the likelihood needs besides the parameter vector."""
    k0: int
    n_freq: int
    df: float
    data: np.ndarray        # complex128 [n_det, n_freq]
    psd: np.ndarray         # float64    [n_det, n_freq]
    det_tensor: np.ndarray  # float64    [n_det, 3, 3]
    det_pos: np.ndarray     # float64    [n_det, 3] (m)
    gmst: float
    dist_grid: np.ndarray   # float64    [n_dist] (Mpc)
    dist_logw: np.ndarray   # float64    [n_dist]

    @property
    def n_det(self) -> int:
        return self.data.shape[0]

    @property
    def freqs(self) -> np.ndarray:
        return (self.k0 + np.arange(self.n_freq, dtype=np.float64)) * self.df


def make_problem(duration: float, f_min: float, f_max: float, psd_scale: float = 1e-46,
                 noise_seed: int | None = SEEDS["noise"], det_seed: int = SEEDS["detectors"],
                 n_det: int = 3, n_dist: int = 1000, gmst: float = 0.0) -> Problem:
    """Noise-only problem (the caller adds an injected signal to ``data``)."""
    g = freq_grid(duration, f_min, f_max)
    f = g.freqs
    psd1 = psd_fit(f, psd_scale)
    psd = np.tile(psd1, (n_det, 1))
    if noise_seed is None:
        data = np.zeros((n_det, g.n_freq), dtype=np.complex128)
    else:
        data = gaussian_noise(noise_seed, psd, g.df)
    pos, tens = detectors(det_seed, n_det)
    dg, dw = distance_grid(n_dist)
    return Problem(k0=g.k0, n_freq=g.n_freq, df=g.df, data=data, psd=psd,
                   det_tensor=tens, det_pos=pos, gmst=gmst, dist_grid=dg, dist_logw=dw)
