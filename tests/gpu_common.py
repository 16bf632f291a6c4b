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


_HET_POOL = None


def _het_init(prob, het):
    global _HET_POOL
    _HET_POOL = (prob, het)


def _het_eval(args):
    from oracle import heterodyne as H
    theta, marg, dd = args
    prob, het = _HET_POOL
    return H.loglike(theta, prob, het, marg, dd)


def oracle_het_many(thetas, prob, het, marg):
    """The heterodyne oracle over a process pool (same values as
    oracle.heterodyne.loglike_many, row by row)."""
    import multiprocessing as mp
    thetas = np.asarray(thetas, dtype=np.float64)
    dd = L.data_inner(prob)
    if N_PROC <= 1 or len(thetas) < 2:
        from oracle import heterodyne as H
        return H.loglike_many(thetas, prob, het, marg)
    with mp.get_context("fork").Pool(N_PROC, initializer=_het_init, initargs=(prob, het)) as pool:
        res = pool.map(_het_eval, [(t, marg, dd) for t in thetas],
                       chunksize=max(1, len(thetas) // (4 * N_PROC)))
    return np.array(res)
