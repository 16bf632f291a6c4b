"""Injection campaign and P-P calibration of the sampler.

Section on injection tests and P-P calibration, and the table of sampler
configurations.  For each injection:
  * the true parameters are drawn from the recovery prior: a uniform point of
    the sampler's unit cube, with d_L ~ d^2 on the distance grid's range and
    phi_c uniform on [0, 2 pi) for the marginalised pair;
  * the data are seeded Gaussian noise plus the library's own template of the
    true parameters (``gw_template``);
  * nested sampling runs in the configuration under test, and the credible
    level of each sampled coordinate is the posterior mass below the truth,
    taken with the nested-sampling weights directly;
  * the marginalised d_L and phi_c are drawn post-hoc for the weighted points
    (``gw_reconstruct``) and get credible levels the same way.  The grid
    quantises these, so they are reported but left out of the KS tests.
Each sampled coordinate is summarised by the KS p-value of its credible levels
against U(0, 1), and all of them together by Fisher's combined p-value.

Configurations: ``baseline`` (the seven Gibbs blocks, one sweep per
replacement), ``highres`` (three sweeps), and ``nss`` (the unblocked nested
slice sampler: one block of all 11 coordinates, 3 x 11 joint slice steps per
replacement); ``joint`` puts the masses, spins and tidal parameters in one
block.  With ``marg = GW_MARG_PHASE_TIME`` coordinate 10 is d_L (t_c
marginalised, as in the GW170817 configuration); the post-hoc pair is then
(t_c, phi_c), and the injections draw t_c uniformly over the marginal's grid.

Run ``python -m paper_2607_28265_amd.pp --help`` for the command line.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import sys
import time

import numpy as np

from . import Context, _lib
from .nested import BLOCKS, N_DIM, UNBLOCKED, NestedSampler

# ``joint``: the masses, spins and tidal parameters in one block (a different
# decomposition of the same space, one sweep per replacement)
JOINT_INTRINSIC = ((0, 1, 2, 3, 4, 5), (6,), (7, 8), (9,), (10,))
CONFIGS = {"baseline": (BLOCKS, 1), "highres": (BLOCKS, 3), "nss": (UNBLOCKED, 3 * N_DIM),
           "joint": (JOINT_INTRINSIC, 1)}
C_SI = 299792458.0  # m / s
PARAMS = ("mc", "q", "chi1", "chi2", "lambda1", "lambda2", "iota", "ra", "dec", "psi", "tc")
LO = np.array([1.1, 0.5, -0.05, -0.05, 0.0, 0.0])
HI = np.array([1.4, 1.0, 0.05, 0.05, 5000.0, 5000.0])


@dataclasses.dataclass
class SkyFrame:
    """The detector sky frame of ``gw_set_sky_frame`` in numpy: baseline n of
    detectors a -> b, e1 the Earth's axis made orthogonal to n (x when
    |n_z| > 0.99), e2 = n x e1; with det_time, coordinate 10 is the arrival
    time at detector a."""
    det_pos: np.ndarray
    gmst: float = 0.0
    a: int = 0
    b: int = 1
    det_time: bool = False

    def __post_init__(self):
        n = np.asarray(self.det_pos[self.b], float) - np.asarray(self.det_pos[self.a], float)
        n = n / np.linalg.norm(n)
        ref = np.array([1.0, 0.0, 0.0]) if abs(n[2]) > 0.99 else np.array([0.0, 0.0, 1.0])
        e1 = ref - (ref @ n) * n
        e1 = e1 / np.linalg.norm(e1)
        self.n, self.e1, self.e2 = n, e1, np.cross(n, e1)
        self.ra_m = np.asarray(self.det_pos[self.a], float)

    def direction(self, u7: float, u8: float) -> np.ndarray:
        zen = math.acos(1.0 - 2.0 * u8)
        kap = 2.0 * math.pi * u7
        return math.cos(zen) * self.n + math.sin(zen) * (math.cos(kap) * self.e1 + math.sin(kap) * self.e2)

    def cube(self, ra: float, dec: float):
        """(u7, u8, s) of a sky position."""
        phi = ra - self.gmst
        s = np.array([math.cos(dec) * math.cos(phi), math.cos(dec) * math.sin(phi), math.sin(dec)])
        return (math.atan2(s @ self.e2, s @ self.e1) % (2.0 * math.pi)) / (2.0 * math.pi), 0.5 * (1.0 - s @ self.n), s


def to_cube(theta, d_lo: float, d_hi: float, time_marg: bool, frame: SkyFrame | None = None) -> np.ndarray:
    """Unit-cube coordinates of a parameter vector (inverse of the prior
    transform); coordinate 10 is t_c (or the arrival time at the frame's first
    detector), or d_L when t_c is marginalised."""
    th = np.asarray(theta, dtype=np.float64)
    u = np.empty(N_DIM)
    u[:6] = (th[:6] - LO) / (HI - LO)
    u[6] = 0.5 * (1.0 - math.cos(th[7]))
    if frame is None:
        u[7] = th[8] / (2.0 * math.pi)
        u[8] = 0.5 * (math.sin(th[9]) + 1.0)
    else:
        u[7], u[8], s = frame.cube(th[8], th[9])
    u[9] = th[10] / math.pi
    if time_marg:
        u[10] = (th[6] ** 3 - d_lo ** 3) / (d_hi ** 3 - d_lo ** 3)
    elif frame is not None and frame.det_time:
        u[10] = (th[12] - float(s @ frame.ra_m) / C_SI + 0.1) / 0.2
    else:
        u[10] = (th[12] + 0.1) / 0.2
    return u


def draw_truth(rng, d_lo: float, d_hi: float, time_marg: bool, frame: SkyFrame | None = None,
               t_span: float = 0.1) -> np.ndarray:
    """One parameter vector from the recovery prior: a uniform cube point
    through the prior transform (in the given sky frame), d_L ~ d^2 and phi_c
    uniform; with the time marginal, t_c uniform on [-t_span, t_span] (the
    span of the marginal's grid) instead of from the cube."""
    u = rng.uniform(size=N_DIM)
    th = np.zeros(13)
    th[:6] = LO + (HI - LO) * u[:6]
    th[7] = math.acos(1.0 - 2.0 * u[6])
    if frame is None:
        th[8] = 2.0 * math.pi * u[7]
        th[9] = math.asin(2.0 * u[8] - 1.0)
    else:
        s = frame.direction(u[7], u[8])
        th[9] = math.asin(max(-1.0, min(1.0, float(s[2]))))
        th[8] = (math.atan2(float(s[1]), float(s[0])) + frame.gmst) % (2.0 * math.pi)
    th[10] = math.pi * u[9]
    th[6] = (d_lo ** 3 + rng.uniform() * (d_hi ** 3 - d_lo ** 3)) ** (1.0 / 3.0)
    th[11] = 2.0 * math.pi * rng.uniform()
    th[12] = t_span * (2.0 * rng.uniform() - 1.0) if time_marg else -0.1 + 0.2 * u[10]
    if frame is not None and frame.det_time and not time_marg:
        th[12] += float(s @ frame.ra_m) / C_SI
    return th


def weighted_level(samples, weights, truth: float) -> float:
    """Posterior mass strictly below the truth."""
    s = np.asarray(samples, dtype=np.float64)
    w = np.asarray(weights, dtype=np.float64)
    return float(w[s < truth].sum() / w.sum())


def ks_pvalue(levels) -> float:
    from scipy import stats
    return float(stats.kstest(np.asarray(levels, dtype=np.float64), "uniform").pvalue)


def fisher_pvalue(pvalues) -> float:
    from scipy import stats
    return float(stats.combine_pvalues(np.asarray(pvalues, dtype=np.float64), method="fisher").pvalue)


@dataclasses.dataclass
class Campaign:
    """Fixed parts of a campaign: the noise-free problem (grid, PSD,
    detectors, distance grid) and a context that makes templates."""
    base: object
    config: str = "baseline"
    like: int = _lib.GW_HET
    marg: int = _lib.GW_MARG_PHASE_DIST
    prec: int = _lib.GW_PREC_MIXED
    n_live: int = 512
    n_delete: int = 64
    n_bins: int = 500
    seed: int = 2026
    n_phase: int = 2048
    recon_floor: float = 1e-12  # points below this fraction of the largest weight are not reconstructed
    sky_frame: bool = False     # sample the sky about the baseline of detectors 0 -> 1
    det_time: bool = False      # ... and the arrival time at detector 0
    sweeps: int = 0             # Gibbs sweeps per replacement (0: the configuration's own M)

    def __post_init__(self):
        if self.config not in CONFIGS:
            raise ValueError(f"config must be one of {sorted(CONFIGS)}")
        self.time_marg = self.marg == _lib.GW_MARG_PHASE_TIME
        self.d_lo = float(self.base.dist_grid[0])
        self.d_hi = float(self.base.dist_grid[-1])
        self.frame = SkyFrame(self.base.det_pos, self.base.gmst, det_time=self.det_time) if self.sky_frame else None
        self._tctx = Context(dataclasses.replace(self.base, data=np.zeros_like(self.base.data)))
        step, n_t, _, _ = _lib.gw_time_grid_info(self._tctx.handle)
        self.t_span = step * (n_t - 1) / 2  # the time marginal's grid spans [-t_span, t_span]

    def close(self):
        self._tctx.close()

    def make_data(self, i: int):
        """(truth, problem, noise seed) of injection i: seeded noise plus the template."""
        import torch
        from gwsynth import gaussian_noise
        rng = np.random.default_rng([self.seed, i])
        th = draw_truth(rng, self.d_lo, self.d_hi, self.time_marg, self.frame, self.t_span)
        h = self._tctx.template(torch.from_numpy(th[None, :].copy()).cuda()).cpu().numpy()[0]  # complex
        noise_seed = int(rng.integers(1 << 62))
        noise = gaussian_noise(noise_seed, self.base.psd, self.base.df)
        prob = dataclasses.replace(self.base, data=noise + h)
        return th, prob, noise_seed

    def run_injection(self, i: int, keep: bool = False) -> dict:
        import torch
        th, prob, _ = self.make_data(i)
        blocks, sweeps = CONFIGS[self.config]
        if self.sweeps > 0:
            sweeps = self.sweeps
        t0 = time.perf_counter()
        with Context(prob) as ctx:
            if self.like == _lib.GW_HET:
                ctx.heterodyne_setup(th, self.n_bins)  # fiducial at the true parameters
            if self.frame is not None:
                _lib.gw_set_sky_frame(ctx.handle, 1, 0, 1, self.det_time)
            ns = NestedSampler(ctx, n_live=self.n_live, n_delete=self.n_delete, seed=self.seed * 1000 + i,
                               blocks=blocks, sweeps=sweeps, like=self.like, prec=self.prec, marg=self.marg)
            res = ns.run()
            x, w = ns.samples()
            truth = to_cube(th, self.d_lo, self.d_hi, self.time_marg, self.frame)
            levels = [weighted_level(x[:, j], w, truth[j]) for j in range(N_DIM)]
            # post-hoc draws of the marginalised pair for the weighted points:
            # (d_L, phi_c), or (t_c, phi_c) when t_c is marginalised
            sel = np.nonzero(w > self.recon_floor * w.max())[0]
            xs = torch.from_numpy(np.ascontiguousarray(x[sel])).cuda()
            ths = _lib.gw_prior_transform(ctx.handle, xs, marg=self.marg)
            rng = np.random.default_rng([self.seed, i, 7])
            uni = torch.from_numpy(rng.uniform(size=(sel.size, 2))).cuda()
            recon, _, _ = _lib.gw_reconstruct(ctx.handle, ths, uni, like=self.like, marg=self.marg, prec=self.prec,
                                              n_phase=self.n_phase)
            recon = recon.cpu().numpy()
            torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        out = dict(index=i, levels=levels, log_z=res["log_z"], log_z_err=res["log_z_err"],
                   iterations=res["iterations"], n_evals=res["n_evals"], sampling_s=res["wall_s"], wall_s=wall,
                   ess=res["ess"], truth=th.tolist())
        ws = w[sel]
        if self.time_marg:
            out["level_tc"] = weighted_level(recon[:, 0], ws, th[12])
        else:
            out["level_dl"] = weighted_level(recon[:, 0], ws, th[6])
        out["level_phic"] = weighted_level(recon[:, 1], ws, th[11])
        out["n_recon"] = int(sel.size)
        if keep:
            out["x"], out["w"], out["sel"], out["recon"] = x, w, sel, recon
        return out

    def summarise(self, runs) -> dict:
        names = list(PARAMS)
        if self.frame is not None:
            names[7], names[8] = "sky_azimuth", "sky_zenith"
            if self.det_time:
                names[10] = "t_det0"
        if self.time_marg:
            names[10] = "dl"
        lv = np.array([r["levels"] for r in runs])
        ks = {n: ks_pvalue(lv[:, j]) for j, n in enumerate(names)}
        out = dict(config=self.config, sweeps=self.sweeps or CONFIGS[self.config][1],
                   like="het" if self.like == _lib.GW_HET else "full",
                   sky_frame="detector" if self.frame is not None else "equatorial", det_time=self.det_time,
                   marg="phase+time" if self.time_marg else "phase+distance", n_injections=len(runs),
                   ks_pvalues=ks, fisher_p=fisher_pvalue(list(ks.values())),
                   median_sampling_s=float(np.median([r["sampling_s"] for r in runs])),
                   median_evals=float(np.median([r["n_evals"] for r in runs])))
        if not self.time_marg:
            sampled = [v for n, v in ks.items() if n not in ("tc", "t_det0")]
            out["fisher_p_without_tc"] = fisher_pvalue(sampled)
            out["ks_reconstructed"] = {"dl": ks_pvalue([r["level_dl"] for r in runs]),
                                       "phic": ks_pvalue([r["level_phic"] for r in runs])}
        else:
            out["ks_reconstructed"] = {"tc": ks_pvalue([r["level_tc"] for r in runs]),
                                       "phic": ks_pvalue([r["level_phic"] for r in runs])}
        return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--n", type=int, default=100, help="injections")
    ap.add_argument("--config", default="baseline", choices=sorted(CONFIGS))
    ap.add_argument("--like", default="het", choices=["het", "full"])
    ap.add_argument("--marg", default="dist", choices=["dist", "time"])
    ap.add_argument("--duration", type=float, default=128.0)
    ap.add_argument("--fmax", type=float, default=2048.0)
    ap.add_argument("--psd-scale", type=float, default=1e-49)
    ap.add_argument("--n-live", type=int, default=512)
    ap.add_argument("--n-delete", type=int, default=64)
    ap.add_argument("--n-bins", type=int, default=500)
    ap.add_argument("--seed", type=int, default=2026)
    ap.add_argument("--sky-frame", action="store_true", help="sample the sky about the baseline of detectors 0, 1")
    ap.add_argument("--det-time", action="store_true", help="with --sky-frame: sample the arrival time at detector 0")
    ap.add_argument("--sweeps", type=int, default=0, help="Gibbs sweeps per replacement (default: the config's)")
    ap.add_argument("--out", default=None, help="JSON file for the per-injection records and the summary")
    a = ap.parse_args(argv)
    import gwsynth
    base = gwsynth.make_problem(a.duration, 20.0, a.fmax, psd_scale=a.psd_scale, noise_seed=None)
    camp = Campaign(base, config=a.config, like=_lib.GW_HET if a.like == "het" else _lib.GW_FULL,
                    marg=_lib.GW_MARG_PHASE_TIME if a.marg == "time" else _lib.GW_MARG_PHASE_DIST,
                    n_live=a.n_live, n_delete=a.n_delete, n_bins=a.n_bins, seed=a.seed, sky_frame=a.sky_frame,
                    det_time=a.det_time, sweeps=a.sweeps)
    runs = []
    try:
        for i in range(a.n):
            r = camp.run_injection(i)
            runs.append(r)
            print(f"injection {i}: {r['iterations']} it, {r['n_evals']} evals, sampling {r['sampling_s']:.2f} s, "
                  f"levels " + " ".join(f"{v:.2f}" for v in r["levels"]), flush=True)
    finally:
        camp.close()
    summ = camp.summarise(runs)
    print(json.dumps(summ), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(dict(summary=summ, runs=runs, args=vars(a)), f)
    return 0


if __name__ == "__main__":
    sys.exit(main())
