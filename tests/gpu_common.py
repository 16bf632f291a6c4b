"""Shared set-up of the GPU parity tests: seeded problems with oracle-made
injections, handed identically to the oracle and to the HIP library."""
import functools
import os

import numpy as np

import gwsynth
from oracle import likelihood as L

N_PROC = max(1, min(16, len(os.sched_getaffinity(0))))


def with_injection(prob, theta_inj):
    prob.data = prob.data + L.strain(theta_inj, prob)
    prob.theta_inj = theta_inj
    return prob


def scale_to_snr(prob, theta, snr):
    """Rescale d_L of ``theta`` so that the network optimal SNR is ``snr``."""
    _, hh = L.overlap(theta, prob)
    th = theta.copy()
    th[6] *= np.sqrt(hh) / snr
    return th


@functools.lru_cache(maxsize=None)
def problem(name: str, loud: bool = False):
    cfg = gwsynth.CONFIGS[name]
    scale = 1e-49 if loud else cfg["psd_scale"]
    prob = gwsynth.make_problem(cfg["duration"], cfg["f_min"], cfg["f_max"], psd_scale=scale)
    th = gwsynth.prior_draws(gwsynth.SEEDS["injection"], 1)[0]
    if loud:
        th = scale_to_snr(prob, th, 24.0)
    return with_injection(prob, th)


def oracle_many(thetas, prob, marg):
    return L.loglike_many(thetas, prob, marg, processes=N_PROC)
