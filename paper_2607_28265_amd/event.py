"""End-to-end analysis of one event, in the order of the GW170817 section.

The pipeline runs on the library's kernels:
  1. reference parameters for the relative binning from a maximum-likelihood
     search (``gw_fiducial_search``) over the prior, narrowed in chirp mass
     and coalescence time around a trigger, as a detection pipeline reports
     them;
  2. the heterodyne on the found parameters (5000 bins by default);
  3. nested sampling with the phase and coalescence time marginalised and d_L
     sampled, the sky in the detector frame (m = 512, k = 64, one sweep), the
     time window narrowed to +-0.03 s around the trigger as in that section;
  4. post-hoc (t_c, phi_c) for the weighted points (``gw_reconstruct``).
The event is a synthetic injection, since no detector strain is available
here: seeded noise at the analytic PSD plus the library's template of a prior
draw, with t_c within 10 ms of the trigger time 0 and the distance set for a
chosen network SNR.  Each stage is timed, and the weighted posterior mean and
standard deviation of each parameter (circular ones for the right ascension
and the phase) are reported next to the truth.

``python -m paper_2607_28265_amd.event --help`` lists the options.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import Context, _lib
from .nested import NestedSampler
from .prescreen import library_injection

MC_LO, MC_WIDTH = 1.1, 0.3  # chirp-mass prior [1.1, 1.4] Msun
TC_LO, TC_WIDTH = -0.1, 0.2  # t_c prior [-0.1, 0.1] s
# posterior summaries: name -> index into the parameter vector
REPORT = {"mc": 0, "q": 1, "lambda1": 4, "dl": 6, "iota": 7, "ra": 8, "dec": 9, "phic": 11, "tc": 12}
CIRCULAR = ("ra", "phic")


def weighted_stats(x, w):
    """Weighted mean and standard deviation."""
    w = np.asarray(w, dtype=np.float64) / np.sum(w)
    m = float(np.sum(w * x))
    return m, float(math.sqrt(max(float(np.sum(w * (x - m) ** 2)), 0.0)))


def weighted_circular_stats(x, w):
    """Weighted circular mean in [0, 2 pi) and circular standard deviation
    sqrt(-2 ln R), R the length of the mean resultant vector."""
    w = np.asarray(w, dtype=np.float64) / np.sum(w)
    c, s = float(np.sum(w * np.cos(x))), float(np.sum(w * np.sin(x)))
    r = math.hypot(c, s)
    return math.atan2(s, c) % (2.0 * math.pi), math.sqrt(-2.0 * math.log(r)) if r > 0.0 else math.inf


def make_event(seed: int = 2017, snr: float = 32.0, duration: float = 128.0, f_max: float = 2048.0,
               psd_scale: float = 1e-49):
    """(problem, truth): noise plus the library's template of a prior draw."""
    import gwsynth
    rng = np.random.default_rng(seed)
    prob = gwsynth.make_problem(duration, 20.0, f_max, psd_scale=psd_scale, noise_seed=int(rng.integers(1 << 62)))
    th = gwsynth.prior_draws(int(rng.integers(1 << 62)), 1)[0]
    th[11] = 2.0 * math.pi * rng.uniform()
    th[12] = 0.01 * (2.0 * rng.uniform() - 1.0)
    truth = library_injection(Context, prob, th, snr=snr)
    return prob, truth


def analyse(prob, trigger_mc: float, trigger_tc: float, truth=None, n_bins: int = 5000, pop: int = 8192,
            generations: int = 300, n_live: int = 512, n_delete: int = 64, seed: int = 17,
            mc_half_width: float = 0.002, tc_half_width: float = 0.005, time_window: float = 0.03,
            tm_split: int = 0) -> dict:
    """Run the four stages on ``prob``; ``truth``, when given, is only
    reported beside the posterior summaries."""
    import torch
    out = {}
    marg = _lib.GW_MARG_PHASE_TIME
    with Context(prob) as ctx:
        # 1. search box: the trigger's chirp mass and time, the rest of the prior whole
        lo, hi = np.zeros(11), np.ones(11)
        u_mc = (trigger_mc - MC_LO) / MC_WIDTH
        u_tc = (trigger_tc - TC_LO) / TC_WIDTH
        lo[0], hi[0] = max(0.0, u_mc - mc_half_width / MC_WIDTH), min(1.0, u_mc + mc_half_width / MC_WIDTH)
        lo[10], hi[10] = max(0.0, u_tc - tc_half_width / TC_WIDTH), min(1.0, u_tc + tc_half_width / TC_WIDTH)
        x = torch.from_numpy(lo + (hi - lo) * np.random.default_rng(seed).uniform(size=(pop, 11))).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fx, fid = _lib.gw_fiducial_search(ctx.handle, x, generations, seed=seed, lo=lo, hi=hi)
        torch.cuda.synchronize()
        out["search_s"] = time.perf_counter() - t0
        out["search_evals"] = pop * (generations + 1)
        out["fiducial"] = [float(v) for v in fid]
        # 2. heterodyne on the found point
        t0 = time.perf_counter()
        ctx.heterodyne_setup(fid, n_bins)
        _lib.gw_set_sky_frame(ctx.handle, 1, 0, 1, False)
        _lib.gw_set_time_window(ctx.handle, time_window)
        _lib.gw_set_het_tm_split(ctx.handle, tm_split)
        torch.cuda.synchronize()
        out["heterodyne_s"] = time.perf_counter() - t0
        # 3. nested sampling (phase and t_c marginalised, d_L sampled)
        ns = NestedSampler(ctx, n_live=n_live, n_delete=n_delete, seed=seed, like=_lib.GW_HET,
                           prec=_lib.GW_PREC_MIXED, marg=marg)
        res = ns.run()
        out.update(sampling_s=res["wall_s"], iterations=res["iterations"], n_evals=res["n_evals"],
                   log_z=res["log_z"], log_z_err=res["log_z_err"], ess=res["ess"])
        xs, w = ns.samples()
        # 4. post-hoc (t_c, phi_c) for the points that carry weight
        t0 = time.perf_counter()
        sel = np.nonzero(w > 1e-12 * w.max())[0]
        ths = _lib.gw_prior_transform(ctx.handle, torch.from_numpy(np.ascontiguousarray(xs[sel])).cuda(), marg=marg)
        uni = torch.from_numpy(np.random.default_rng(seed + 1).uniform(size=(sel.size, 2))).cuda()
        rec, _, _ = _lib.gw_reconstruct(ctx.handle, ths, uni, like=_lib.GW_HET, marg=marg)
        th = ths.cpu().numpy()
        rec = rec.cpu().numpy()
        out["reconstruction_s"] = time.perf_counter() - t0
        _lib.gw_set_sky_frame(ctx.handle, 0)
    th[:, 12], th[:, 11] = rec[:, 0], rec[:, 1]
    ws = w[sel]
    out["n_posterior_points"] = int(sel.size)
    out["posterior"] = {}
    for name, j in REPORT.items():
        circ = name in CIRCULAR
        m, sd = (weighted_circular_stats if circ else weighted_stats)(th[:, j], ws)
        row = {"mean": m, "sd": sd}
        if truth is not None:
            t = float(truth[j])
            d = (m - t + math.pi) % (2.0 * math.pi) - math.pi if circ else m - t
            row["truth"] = t
            row["pull"] = d / sd if 0.0 < sd < math.inf else None
        out["posterior"][name] = row
    out["total_s"] = out["search_s"] + out["heterodyne_s"] + out["sampling_s"] + out["reconstruction_s"]
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description="Analyse one synthetic event end to end.")
    ap.add_argument("--seed", type=int, default=2017)
    ap.add_argument("--snr", type=float, default=32.0)
    ap.add_argument("--n-bins", type=int, default=5000)
    ap.add_argument("--n-live", type=int, default=512)
    ap.add_argument("--n-delete", type=int, default=64)
    ap.add_argument("--pop", type=int, default=8192)
    ap.add_argument("--generations", type=int, default=300)
    ap.add_argument("--time-window", type=float, default=0.03)
    ap.add_argument("--sampler-seeds", default="17", help="comma list: one run per seed on the same event")
    ap.add_argument("--tm-split", type=int, default=0, help="edge chunks of the time marginal's edge moments (0: auto)")
    a = ap.parse_args(argv)
    prob, truth = make_event(a.seed, a.snr)
    rng = np.random.default_rng(a.seed + 5)
    # a trigger's chirp mass and time: the truth with a pipeline's scatter
    trig_mc = float(truth[0] + 5e-4 * rng.standard_normal())
    trig_tc = float(truth[12] + 1e-3 * rng.standard_normal())
    for seed in (int(v) for v in a.sampler_seeds.split(",")):
        res = analyse(prob, trig_mc, trig_tc, truth, n_bins=a.n_bins, pop=a.pop, generations=a.generations,
                      n_live=a.n_live, n_delete=a.n_delete, seed=seed, time_window=a.time_window,
                      tm_split=a.tm_split)
        res["seed"] = seed
        res["truth"] = [float(v) for v in truth]
        res["trigger"] = {"mc": trig_mc, "tc": trig_tc}
        print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
