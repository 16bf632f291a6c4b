#!/usr/bin/env python3
"""Throughput of the batched full-band gravitational-wave likelihood on one MI355X.

One step = one batch of 4096 proposals through the whole full-band path
(prologue -> fused phase/projection/overlap kernel -> FP64 epilogue with the
phase and distance marginalisations) on the 128 s, 20-2048 Hz, three-detector
grid (259,585 bins per detector).  Inputs are resident in HBM before timing.
The measured form is the mixed-precision one (FP64 phase, FP32 hardware
sin/cos, FP64 sums); the plain FP64 form is timed alongside for the speedup.

Prints one JSON line (see the keys below).  --gpus above 1 is refused: this
build measures one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "logL evals/sec (full-band & heterodyned) vs FP64 plain at |dlogL|<1e-3"

# Algorithmic FP64 flops per (proposal, frequency bin) of the fused kernel, FMA
# counted as 2.  FP64 form: TaylorF2 phase by Horner in f^(1/3) (11 FMA + 1 mul
# = 23), reduction to a fraction of a cycle (1), detector-0 complex MAC (4 FMA
# = 8), two detectors' rotation-Horner steps (2 x (2 mul + 6 FMA) = 28), and
# the FP64 sin/cos polynomial (47): 107.  Mixed form: the phase comes from a
# cubic recurrence in runs of bins (gw_full_phase_runs): a recurrence bin
# costs 3 additions, a directly evaluated one (the first four of a run, and
# every bin below the lowest level) the phase without its constant and
# linear terms (9 FMA + 3 mul = 21), the linear term (1 mul + 1 FMA = 3), the
# difference update (3) and the sum (1); both then add 1 + 8 + 28.  The FP32
# sin/cos of the mixed form are not counted as FP64 flops.
FLOPS_PER_BIN = {"fp64": 107.0, "mixed_recurrence": 40.0, "mixed_direct": 65.0}


def mixed_flops_per_bin(gw, ctx, n_freq):
    """Average mixed-form flops per bin over the band.  Runs are aligned
    blocks, and a chunk that starts inside one also re-evaluates the run's
    first bins, which adds under 0.2 % at 128 chunks and is not counted."""
    k_min, lens = gw.gw_full_phase_runs(ctx.handle)
    direct, k = 0, n_freq - 1
    while k >= 0:
        run, s = 0, 0
        for km, ln in zip(k_min, lens):
            if k & ~(ln - 1) >= km:
                run, s = ln, k & ~(ln - 1)
                break
        if run == 0:  # every lower bin is evaluated directly
            direct += k + 1
            break
        direct += min(min(s + run - 1, n_freq - 1) - s + 1, 4)
        k = s - 1
    return (FLOPS_PER_BIN["mixed_recurrence"] * (n_freq - direct) + FLOPS_PER_BIN["mixed_direct"] * direct) / n_freq
PEAK_FP64_TFLOPS = 78.6  # MI355X FP64 vector, dense

# HBM bytes per launch from two rocprofv3 PMC runs (FETCH_SIZE, WRITE_SIZE)
# scaled by what the same counters read for a plain 256 MiB device copy
# (FETCH_SIZE x 1.99982, WRITE_SIZE x 1.000): k_full<3, 1, false> at
# 4096 x 259,585, and k_wmom<3> at 4096 rows on 2048 cached slots (12 orders).
# Valid only for the kernel sources they were taken on (hash below; retaken
# when those files change, or carried over after checking that the compiled
# code of both kernels is unchanged).
TRAFFIC = {"sources_sha256": "78485f89754a80c14c8330dda9495618a08f1c73a5db95363cacc7f73b1b324d",
           "k_full": {"read_bytes": 22404.2 * 1.99982 * 1024, "write_bytes": 49152.0 * 1024},
           "k_wmom": {"read_bytes": 320487.9 * 1.99982 * 1024, "write_bytes": 23040.0 * 1024}}
TRAFFIC_SOURCES = ("paper_2607_28265_amd/csrc/gw_full.hip", "paper_2607_28265_amd/csrc/gw_device.h")


def traffic_bytes(kernel="k_full"):
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != TRAFFIC["sources_sha256"]:
        return None
    return TRAFFIC[kernel]["read_bytes"] + TRAFFIC[kernel]["write_bytes"]


_T0 = time.perf_counter()


def log(msg):
    """Progress on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench {time.perf_counter() - _T0:7.1f} s] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--legs", default="full,cfg1,het,tmarg,recon,mlp,cache,fiducial,nested,nested_tmarg,nested_full,"
                                      "prescreen",
                    help="comma list of legs to run: full (always timed), cfg1, het, tmarg, recon, mlp, cache, fiducial, "
                         "nested, nested_tmarg, nested_full, prescreen, copy")
    return ap.parse_args()


def make_problem_gpu(gw, torch):
    """Full-band problem: seeded noise plus an injection made by the library."""
    import numpy as np
    import gwsynth
    cfg = gwsynth.CONFIGS["cfg2"]
    prob = gwsynth.make_problem(cfg["duration"], cfg["f_min"], cfg["f_max"], psd_scale=cfg["psd_scale"])
    th_inj = gwsynth.prior_draws(gwsynth.SEEDS["injection"], 1)
    noise_only = gw.Context(prob)
    h = noise_only.template(torch.from_numpy(th_inj).cuda())[0].cpu().numpy()
    noise_only.close()
    prob.data = prob.data + h
    return prob, th_inj[0]


def time_steps(ctx, theta, out, steps, warmup, prec, marg, torch, gw, profile=False):
    for _ in range(warmup):
        ctx.loglike(theta, marg=marg, prec=prec, out=out)
    torch.cuda.synchronize()
    if profile:
        gw._lib.gw_profile_read(ctx.handle)
        gw._lib.gw_profile_enable(ctx.handle, True)
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.loglike(theta, marg=marg, prec=prec, out=out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern = None
    if profile:
        ms, nl = gw._lib.gw_profile_read(ctx.handle)
        gw._lib.gw_profile_enable(ctx.handle, False)
        kern = ms / max(nl, 1)
    return (t1 - t0), kern


# Algorithmic FP64 flops per (row, edge) of the heterodyned contraction
# k_het<3, PREC>, FMA = 2: the edge's TaylorF2 phase (11 FMA + 1 mul = 23)
# minus the fiducial's (1); per detector the delay term of detectors 1 and 2
# (1 FMA + 1 sub = 3 each), the phasor (mixed: the reduction to a fraction of
# a cycle (1) and the Newton normalisation of the FP32 pair (7); FP64: the
# software sin/cos, 47), the summed-by-parts weight product (4 FMA = 8) and
# the norm term (1 mul + 2 FMA = 5).  Mixed: 24 + 3 (8 + 8 + 5) + 2 x 3 = 93;
# FP64: 24 + 3 (47 + 13) + 6 = 210.
HET_FLOPS_PER_EDGE = {"mixed": 93.0, "fp64": 210.0}


def het_leg(gw, torch, prob, th_inj, steps, warmup):
    """Heterodyned form: bins of equal maximum phase change from the 128 s
    segment (500, the workload, and 5000, the paper's count), 65,536
    proposals in uneven sub-batches of 100-8000, one graph replay per batch,
    launch shape from the library's autotuner on this batch."""
    import numpy as np
    import gwsynth
    from paper_2607_28265_amd import autotune
    n = 65536
    th = np.concatenate([gwsynth.prior_draws(gwsynth.SEEDS["prior"], n // 2),
                         gwsynth.near_posterior(41, th_inj, n // 2, scale=0.5)])
    off = gwsynth.uneven_split(gwsynth.SEEDS["split"], n)
    subs = torch.from_numpy(np.stack([off[:-1], np.diff(off)], axis=1).astype(np.int64)).cuda()
    theta = torch.from_numpy(th).cuda()
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    res = {}
    with gw.Context(prob) as ctx:
        for n_bins in (500, 5000):
            ctx.heterodyne_setup(th_inj, n_bins)
            nb_res = {}
            for name, prec in (("mixed", gw.GW_PREC_MIXED), ("fp64", gw.GW_PREC_FP64)):
                shape, tune_ms = autotune.tune(ctx, theta, gw.GW_HET, gw.GW_MARG_PHASE_DIST, prec, reps=3,
                                               use_cache=False)
                for _ in range(warmup):
                    ctx.loglike_uneven(theta, subs, marg=gw.GW_MARG_PHASE_DIST, prec=prec, out=out)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(steps):
                    ctx.loglike_uneven(theta, subs, marg=gw.GW_MARG_PHASE_DIST, prec=prec, out=out)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                gw._lib.gw_profile_read(ctx.handle)
                gw._lib.gw_profile_enable(ctx.handle, True)
                for _ in range(3):
                    ctx.loglike_uneven(theta, subs, marg=gw.GW_MARG_PHASE_DIST, prec=prec, out=out,
                                       use_graph=False)
                ms, nl = gw._lib.gw_profile_read(ctx.handle)
                gw._lib.gw_profile_enable(ctx.handle, False)
                k_ms = ms / max(nl, 1)
                flops = HET_FLOPS_PER_EDGE[name] * n * (n_bins + 1)
                ach = flops / (k_ms * 1e-3) / 1e12
                nb_res[name] = {"value": n * steps / dt, "ms_per_batch": dt / steps * 1e3, "kernel_ms": k_ms,
                                "autotuned_shape": list(shape), "autotune_ms_per_call": tune_ms,
                                "roofline": {"kernel": f"k_het<3,{1 if name == 'mixed' else 0}>", "bound": "alu",
                                             "achieved": ach, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                                             "frac": ach / PEAK_FP64_TFLOPS, "flops_per_launch": flops,
                                             "flops_per_row_edge": HET_FLOPS_PER_EDGE[name], "traffic": None}}
            nb_res["n_bins"] = n_bins
            res[f"bins_{n_bins}"] = nb_res
            ctx.set_het_shape(4, 0, 0)
        # phase+time marginal on 500 and 5000 bins and the same proposals
        delta, n_t, p_len, blk = gw.gw_time_grid_info(ctx.handle)
        L = p_len * 4
        K = tgrid_orders(L, (n_t - 1) // 2)
        for n_bins in (500, 5000):
            ctx.heterodyne_setup(th_inj, n_bins)
            tm = {}
            for name, prec in (("mixed", gw.GW_PREC_MIXED), ("fp64", gw.GW_PREC_FP64)):
                run = lambda: ctx.loglike(theta, gw.GW_HET, gw.GW_MARG_PHASE_TIME, prec, out=out)
                for _ in range(2):
                    run()
                torch.cuda.synchronize()
                reps = max(3, steps // 2)
                t0 = time.perf_counter()
                for _ in range(reps):
                    run()
                torch.cuda.synchronize()
                dt = (time.perf_counter() - t0) / reps
                mom_ms, n_mom = time_kernel(gw, torch, ctx, run, reps, 1)
                grid_ms, n_grid = time_kernel(gw, torch, ctx, run, reps, 2)
                rows_per_launch = n * reps / max(n_grid, 1)
                gflops = tgrid_flops_per_row(K, L) * rows_per_launch
                tm[name] = {"value": n / dt, "ms_per_batch": dt * 1e3,
                            "moments_ms_per_batch": mom_ms * n_mom / reps,
                            "k_tgrid_ms_per_batch": grid_ms * n_grid / reps,
                            "k_tgrid_roofline": {"bound": "alu", "achieved": gflops / (grid_ms * 1e-3) / 1e12,
                                                 "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                                                 "frac": gflops / (grid_ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
                                                 "rows_per_launch": rows_per_launch}}
            res[f"time_marginal_{n_bins}_bins"] = tm
        n_graphs, inst_ms = gw._lib.gw_graph_info(ctx.handle)
    res.update({"unit": "logL evals/s", "batch": n, "n_sub": int(subs.shape[0]),
                "graph_instantiate_ms": inst_ms,
                "workload": "heterodyned: 500 and 5000 bins of equal maximum phase change from the 128 s segment, "
                            "65,536 proposals (half prior, half near-posterior) in uneven sub-batches of "
                            "100-8000, one graph replay per batch, autotuned launch shape, phase+distance "
                            "marginalised"})
    return res


def cfg1_leg(gw, torch, steps, warmup):
    """Plain FP64 batch likelihood (no marginalisation): T = 8 s, 20-512 Hz,
    3937 bins x 3 detectors, 1024 prior draws; the mixed form beside it."""
    import gwsynth
    cfg = gwsynth.CONFIGS["cfg1"]
    prob = gwsynth.make_problem(cfg["duration"], cfg["f_min"], cfg["f_max"], psd_scale=cfg["psd_scale"])
    th_inj = gwsynth.prior_draws(gwsynth.SEEDS["injection"], 1)
    noise_only = gw.Context(prob)
    prob.data = prob.data + noise_only.template(torch.from_numpy(th_inj).cuda())[0].cpu().numpy()
    noise_only.close()
    n = 1024
    theta = torch.from_numpy(gwsynth.prior_draws(gwsynth.SEEDS["prior"], n)).cuda()
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    res = {}
    with gw.Context(prob) as ctx:
        for name, prec in (("fp64", gw.GW_PREC_FP64), ("mixed", gw.GW_PREC_MIXED)):
            dt, k_ms = time_steps(ctx, theta, out, steps, warmup, prec, gw.GW_MARG_NONE, torch, gw, profile=True)
            fpb = FLOPS_PER_BIN["fp64"] if name == "fp64" else mixed_flops_per_bin(gw, ctx, int(prob.n_freq))
            ach = fpb * n * prob.n_freq / (k_ms * 1e-3) / 1e12
            res[name] = {"value": n * steps / dt, "ms_per_batch": dt / steps * 1e3, "kernel_ms": k_ms,
                         "roofline": {"kernel": f"k_full<3,{0 if name == 'fp64' else 1}>", "bound": "alu",
                                      "achieved": ach, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                                      "frac": ach / PEAK_FP64_TFLOPS, "flops_per_bin": fpb}}
    res.update({"unit": "logL evals/s", "batch": n, "n_freq": int(prob.n_freq),
                "workload": "plain FP64 batch likelihood: T=8 s, 20-512 Hz, df=1/8 Hz (3937 bins x 3 detectors), "
                            "1024 prior draws, no marginalisation"})
    return res


def prescreen_leg(gw, torch, reps):
    """Learned prescreen on the full-band grid with the phase+distance marginal:
    a nested-sampling run (1000 live points, 125 deletions, heterodyned
    likelihood, SNR-24 injection at the 1e-49 PSD) is stopped in its
    posterior-bulk phase; the network is trained on the sampler's recent dead
    points, its live set and one exactly evaluated batch of 65,536 slice
    proposals; a fresh batch of 65,536 proposals is then evaluated exactly with
    and without the prescreen (full band, mixed form)."""
    import numpy as np
    import gwsynth
    from paper_2607_28265_amd import prescreen as P
    from paper_2607_28265_amd.nested import NestedSampler
    cfg = gwsynth.CONFIGS["cfg2"]
    prob = gwsynth.make_problem(cfg["duration"], cfg["f_min"], cfg["f_max"], psd_scale=1e-49)
    th = gwsynth.prior_draws(gwsynth.SEEDS["injection"], 1)[0]
    th_inj = P.library_injection(gw.Context, prob, th, snr=24.0)
    n = 65536
    stage = 180
    res = {}
    with gw.Context(prob) as ctx:
        ctx.heterodyne_setup(th_inj, 500)
        ns = NestedSampler(ctx, n_live=1000, n_delete=125, seed=gwsynth.SEEDS["sampler"], like=gw.GW_HET,
                           prec=gw.GW_PREC_MIXED)
        t0 = time.perf_counter()
        while ns.iteration < stage and not ns.converged(ns.logl.cpu().numpy()):
            ns.step()
        t_ns = time.perf_counter() - t0
        live_x = ns.x.cpu().numpy()
        lstar = float(np.sort(ns.logl.cpu().numpy())[ns.k - 1])
        xp, yp = P.sampler_pairs(ns, last_iters=30)
        mixed, full, pd = gw.GW_PREC_MIXED, gw.GW_FULL, gw.GW_MARG_PHASE_DIST

        def exact(xd, out=None):
            thd = gw.gw_prior_transform(ctx.handle, xd)
            return ctx.loglike(thd, like=full, marg=pd, prec=mixed, out=out)

        xa = P.slice_candidates(live_x, n, seed=1)
        ya = exact(torch.from_numpy(xa).cuda()).cpu().numpy()
        pre = P.Prescreen(ctx, seed=gwsynth.SEEDS["mlp"])
        tr = pre.train(np.concatenate([xp, xa]), np.concatenate([yp, ya]), live_x, lstar, epochs=40, batch=1024)
        margin = pre.set_margin(lstar)
        xb = torch.from_numpy(P.slice_candidates(live_x, n, seed=2)).cuda()
        out = torch.empty(n, dtype=torch.float64, device="cuda")
        exact(xb, out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            exact(xb, out)
        torch.cuda.synchronize()
        t_plain = (time.perf_counter() - t0) / reps
        truth = out.cpu().numpy()
        pre.screen(xb, lstar, audit_frac=0.01, seed=3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            logl, flags, pred, ne = pre.screen(xb, lstar, audit_frac=0.01, seed=3)
        torch.cuda.synchronize()
        t_screen = (time.perf_counter() - t0) / reps
        pred_out = torch.empty(n, dtype=torch.float64, device="cuda")
        pre.mlp.forward(xb, out=pred_out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            pre.mlp.forward(xb, out=pred_out)
        torch.cuda.synchronize()
        t_mlp = (time.perf_counter() - t0) / reps
        logl, flags, pred = logl.cpu().numpy(), flags.cpu().numpy(), pred.cpu().numpy()
        ev = (flags & 1) != 0
        acc_true = truth > lstar
        acc_kept = ev & (logl > lstar)
        aud = (flags & 4) != 0
        near = np.abs(truth - lstar) < 10.0
        err = pred - truth
        confirm_dl = float(np.max(np.abs(logl[ev] - truth[ev]))) if ev.any() else 0.0
        mlp_flops = 2.0 * (11 * 256 + 2 * 256 * 256 + 256) * n
        res = {
            "unit": "accepted proposals/s",
            "value": float(acc_kept.sum()) / t_screen,
            "value_without_prescreen": float(acc_true.sum()) / t_plain,
            "gain": (float(acc_kept.sum()) / t_screen) / (float(acc_true.sum()) / t_plain),
            "candidates": n, "accepted_true": int(acc_true.sum()), "accepted_kept": int(acc_kept.sum()),
            "exact_evals_with": int(ne), "exact_evals_without": n,
            "false_negatives": int((acc_true & ~ev).sum()),
            "audit": {"audited": int(aud.sum()), "audited_accepted": int((aud & (logl > lstar)).sum()),
                      "frac": 0.01},
            "ms_with": t_screen * 1e3, "ms_without": t_plain * 1e3,
            "mlp_rmse_near": float(np.sqrt(np.mean(err[near] ** 2))), "mlp_maxerr_near": float(np.max(np.abs(err[near]))),
            "n_near": int(near.sum()), "margin": margin, "logl_star": lstar,
            "confirm_max_dlogl_vs_unscreened": confirm_dl,
            "mlp_inference": {"ms": t_mlp * 1e3, "rows": n, "tflops": mlp_flops / t_mlp / 1e12,
                              "peak_bf16_tflops": 2500.0, "frac": mlp_flops / t_mlp / 1e12 / 2500.0},
            "training": {"steps": tr.steps, "wall_s": tr.wall_s, "pairs": tr.n_train, "holdout_rmse": tr.rmse_holdout,
                         "loss_first": tr.loss_first, "loss_last": tr.loss_last},
            "ns_stage": {"iterations": ns.iteration, "wall_s": t_ns, "n_evals": ns.n_evals},
            "workload": "learned prescreen: 65,536 first-shrink slice proposals around the live set of a "
                        "heterodyned nested-sampling run stopped at iteration 180 (1000 live, 125 deletions, "
                        "SNR 24 at the 1e-49 PSD); exact confirmation on the 128 s full-band grid, mixed form",
        }
        pre.close()
    return res


def nested_leg(gw, torch):
    """End-to-end nested sampling: 1000 live points, 125 deletions per
    iteration, 11 dimensions in 7 Gibbs blocks, heterodyned (500 bins)
    phase+distance-marginalised likelihood in the mixed form, dlogz 0.1, on the
    SNR-24 injection at the 1e-49 PSD; wall time excludes problem set-up.  The
    oracle's own run of the same settings (stored by the test suite's golden
    script) is quoted beside it."""
    import numpy as np
    import gwsynth
    from paper_2607_28265_amd import prescreen as P
    from paper_2607_28265_amd.nested import NestedSampler
    cfg = gwsynth.CONFIGS["cfg2"]
    prob = gwsynth.make_problem(cfg["duration"], cfg["f_min"], cfg["f_max"], psd_scale=1e-49)
    th = gwsynth.prior_draws(gwsynth.SEEDS["injection"], 1)[0]
    th_inj = P.library_injection(gw.Context, prob, th, snr=24.0)
    with gw.Context(prob) as ctx:
        ctx.heterodyne_setup(th_inj, 500)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ns = NestedSampler(ctx, n_live=1000, n_delete=125, seed=gwsynth.SEEDS["sampler"], like=gw.GW_HET,
                           prec=gw.GW_PREC_MIXED)
        r = ns.run()
        wall = time.perf_counter() - t0
        # the same run with the sky sampled about the baseline of detectors 0
        # and 1, then also with the arrival time at detector 0 as coordinate 10
        frames = {}
        for name, det_time in (("detector_frame", False), ("detector_frame_and_time", True)):
            gw.gw_set_sky_frame(ctx.handle, 1, 0, 1, det_time)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            rf = NestedSampler(ctx, n_live=1000, n_delete=125, seed=gwsynth.SEEDS["sampler"], like=gw.GW_HET,
                               prec=gw.GW_PREC_MIXED).run()
            frames[name] = {"wall_s": time.perf_counter() - t1, "log_z": rf["log_z"], "log_z_err": rf["log_z_err"],
                            "iterations": rf["iterations"], "n_evals": rf["n_evals"], "ess": rf["ess"]}
        gw.gw_set_sky_frame(ctx.handle, 0)
        # three sweeps per replacement (the High-Res setting), the setting of
        # the oracle's reference run: its evidence is compared with the
        # oracle's (runs with one sweep do not decorrelate on this problem)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        r3 = NestedSampler(ctx, n_live=1000, n_delete=125, seed=gwsynth.SEEDS["sampler"], like=gw.GW_HET,
                           prec=gw.GW_PREC_MIXED, sweeps=3).run()
        m3 = {"wall_s": time.perf_counter() - t1, "log_z": r3["log_z"], "log_z_err": r3["log_z_err"],
              "iterations": r3["iterations"], "n_evals": r3["n_evals"], "ess": r3["ess"]}
    out = {"wall_s": wall, "log_z": r["log_z"], "log_z_err": r["log_z_err"], "iterations": r["iterations"],
           "n_evals": r["n_evals"], "evals_per_s": r["n_evals"] / wall, "ess": r["ess"], "sky_frames": frames,
           "three_sweeps": m3}
    gold = os.path.join(ROOT, "tests", "golden", "ns_cfg2.json")
    if os.path.exists(gold):
        with open(gold) as f:
            g = json.load(f)
        out["oracle_run"] = {"log_z": g["log_z"], "log_z_err": g["log_z_err"], "iterations": g["iterations"],
                             "n_evals": g["n_evals"], "sweeps": g.get("sweeps", 1),
                             "cpu_wall_s_single_process": g["cpu_wall_s"]}
        if g.get("sweeps", 1) == 3:
            m3["log_z_minus_oracle_in_sigma"] = (r3["log_z"] - g["log_z"]) / math.hypot(r3["log_z_err"],
                                                                                     g["log_z_err"])
    out["workload"] = ("nested sampling: 1000 live points, 125 deletions per iteration, 7 Gibbs blocks over 11 "
                       "dimensions, heterodyned 500-bin likelihood (mixed form), dlogz 0.1, SNR-24 injection")
    return out


def nested_tmarg_leg(gw, torch):
    """Heterodyned nested sampling at 5000 bins in the detector sky frame with
    t_c and phi_c marginalised and d_L sampled (the paper's GW170817
    configuration), against the same run with phi_c and d_L marginalised and
    t_c sampled: 512 live points, 64 deletions, one sweep, mixed form, the
    SNR-24 injection of the 128 s grid.  The cost per iteration is the figure
    of merit (the two runs integrate the same likelihood over different
    coordinates)."""
    import gwsynth
    from paper_2607_28265_amd import prescreen as P
    from paper_2607_28265_amd.nested import NestedSampler
    cfg = gwsynth.CONFIGS["cfg2"]
    prob = gwsynth.make_problem(cfg["duration"], cfg["f_min"], cfg["f_max"], psd_scale=1e-49)
    th = gwsynth.prior_draws(gwsynth.SEEDS["injection"], 1)[0]
    th_inj = P.library_injection(gw.Context, prob, th, snr=24.0)
    out = {}
    with gw.Context(prob) as ctx:
        ctx.heterodyne_setup(th_inj, 5000)
        gw.gw_set_sky_frame(ctx.handle, 1, 0, 1, False)
        for name, marg in (("phase_time", gw.GW_MARG_PHASE_TIME), ("phase_distance", gw.GW_MARG_PHASE_DIST)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ns = NestedSampler(ctx, n_live=512, n_delete=64, seed=gwsynth.SEEDS["sampler"], like=gw.GW_HET,
                               prec=gw.GW_PREC_MIXED, marg=marg)
            r = ns.run()
            wall = time.perf_counter() - t0
            ns.close()
            out[name] = {"wall_s": wall, "log_z": r["log_z"], "log_z_err": r["log_z_err"],
                         "iterations": r["iterations"], "n_evals": r["n_evals"],
                         "ms_per_iteration": 1e3 * wall / max(1, r["iterations"])}
        gw.gw_set_sky_frame(ctx.handle, 0)
    out["time_over_distance_per_iteration"] = (out["phase_time"]["ms_per_iteration"]
                                               / out["phase_distance"]["ms_per_iteration"])
    out["workload"] = ("nested sampling, heterodyned 5000-bin likelihood (mixed form) in the detector sky frame: "
                       "512 live points, 64 deletions, one sweep, dlogz 0.1, SNR-24 injection on the 128 s grid; "
                       "phase+time marginal (d_L sampled, 3273 grid points) against phase+distance marginal "
                       "(t_c sampled)")
    return out


def cache_leg(gw, torch, prob, steps, warmup, mixed_value):
    """Waveform cache (the sampler's fast/slow split): 4096 rows on 2048
    cached waveforms of the 128 s grid (two rows per slot, as the sampler's
    two bracket ends), moved in sky position, t_c, psi, iota and d_L (kind 1:
    the cached waveform re-summed with new delays) or in psi, iota and d_L
    only (kind 2: cached overlaps reprojected), against the slow update that
    generates and stores the 2048 waveforms."""
    import numpy as np
    import gwsynth
    n_slots, n = 2048, 4096
    base = gwsynth.prior_draws(gwsynth.SEEDS["prior"], n_slots)
    rows = np.repeat(np.arange(n_slots), 2)
    rng = np.random.default_rng(51)
    res = {}
    with gw.Context(prob) as ctx:
        cache = gw.WaveformCache(ctx.handle, n_slots)
        slots_b = torch.arange(n_slots, dtype=torch.int32, device="cuda")
        tb = torch.from_numpy(base).cuda()
        lb = torch.empty(n_slots, dtype=torch.float64, device="cuda")
        for _ in range(max(1, warmup // 2)):
            cache.update(tb, slots_b, prec=gw.GW_PREC_MIXED, out=lb)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = max(3, steps // 5)
        for _ in range(reps):
            cache.update(tb, slots_b, prec=gw.GW_PREC_MIXED, out=lb)
        torch.cuda.synchronize()
        dt_up = (time.perf_counter() - t0) / reps
        res["update"] = {"value": n_slots / dt_up, "ms_per_call": dt_up * 1e3, "rows": n_slots}
        slots = torch.from_numpy(rows.astype(np.int32)).cuda()
        for kind in (1, 2):
            th = base[rows].copy()
            th[:, 7] = np.clip(th[:, 7] + 0.05 * rng.standard_normal(n), 0.01, np.pi - 0.01)
            th[:, 10] = np.mod(th[:, 10] + 0.1 * rng.standard_normal(n), np.pi)
            if kind == 1:
                th[:, 8] = np.mod(th[:, 8] + 0.02 * rng.standard_normal(n), 2 * np.pi)
                th[:, 9] = np.clip(th[:, 9] + 0.02 * rng.standard_normal(n), -1.5, 1.5)
                th[:, 12] += 1e-3 * rng.standard_normal(n)
            tt = torch.from_numpy(th).cuda()
            out = torch.empty(n, dtype=torch.float64, device="cuda")
            for _ in range(warmup):
                cache.loglike(tt, slots, kind, prec=gw.GW_PREC_MIXED, out=out)
            torch.cuda.synchronize()
            if kind == 1:
                gw._lib.gw_profile_read(ctx.handle)
                gw._lib.gw_profile_enable(ctx.handle, True)
            t0 = time.perf_counter()
            for _ in range(steps):
                cache.loglike(tt, slots, kind, prec=gw.GW_PREC_MIXED, out=out)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            r = {"value": n / dt, "ms_per_call": dt * 1e3, "speedup_vs_full_mixed": n / dt / mixed_value}
            if kind == 1:
                ms, nl = gw._lib.gw_profile_read(ctx.handle)
                gw._lib.gw_profile_enable(ctx.handle, False)
                k_ms = ms / max(nl, 1)
                # moment cache: blocks of B bins (256 at df = 1/128 Hz), 12 Chebyshev moments per block and
                # detector, FP32 complex; algorithmic bytes = each used slot's moments once
                blk = 4
                while blk < 512 and math.pi * prob.df * (2 * blk) * 0.25 <= 1.61:
                    blk *= 2
                n_blk = -(-prob.n_freq // blk)
                nbytes = n_slots * n_blk * 3 * 12 * 8
                # per row, block and detector: 12 weighted moments (2 FMA each) + block factor and rotation
                # (8 flop-pairs)
                flops = n * n_blk * 3 * (12 * 2 + 8) * 2
                r["kernel"] = "k_wmom<3>"
                r["kernel_ms"] = k_ms
                r["moment_block_bins"] = blk
                r["roofline"] = {"bound": "hbm", "achieved": nbytes / (k_ms * 1e-3) / 1e9, "peak": 8000.0,
                                 "unit": "GB/s", "frac": nbytes / (k_ms * 1e-3) / 1e9 / 8000.0,
                                 "traffic": traffic_bytes("k_wmom"), "bytes_per_launch": nbytes,
                                 "fp64_tflops": flops / (k_ms * 1e-3) / 1e12,
                                 "fp64_frac": flops / (k_ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS}
            res[f"kind{kind}"] = r
        cache.close()
    res["unit"] = "logL evals/s"
    res["workload"] = ("waveform cache on the 128 s grid: 2048 cached waveforms (block moments), 4096 rows (two "
                       "per slot); kind 1 = sky/t_c/psi/iota/d_L moves on the cached moments, kind 2 = "
                       "psi/iota/d_L moves on the cached overlaps; phase+distance marginalised")
    return res


def tgrid_orders(L, jmax):
    """Expansion orders the library takes for a grid (12 when the dropped
    Chebyshev terms' bound 2 (phi/2)^12 / 12! at phi = pi jmax / L is at most
    2e-11, else 16)."""
    phi = math.pi * jmax / L
    b = 2.0
    for i in range(1, 13):
        b *= 0.5 * phi / i
    return 12 if b <= 2e-11 else 16


# k_tmom (mixed, ND = 3), FP64 flops per (row, bin) on the recurrence path, from
# the source: phase recurrence 3, cycle reduction 1, detector sums 3 x 4 FMA,
# two delay rotations 2 x 6, y = g s 6, and K moment updates of 2 FMA each.
def tmom_flops_per_bin(K):
    return 3 + 1 + 24 + 12 + 6 + 4 * K


# k_tgrid, FP64 flops per row: K transforms of L points at the conventional
# 5 L log2 L, plus the weighted accumulation (2 FMA per point and order); the
# grid epilogue (ln I0, log-sum-exp) is not counted.
def tgrid_flops_per_row(K, L):
    return K * (5 * L * math.log2(L) + 4 * L)


def time_kernel(gw, torch, ctx, fn, steps, mode):
    gw._lib.gw_profile_read(ctx.handle)
    gw._lib.gw_profile_enable(ctx.handle, mode)
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    ms, nl = gw._lib.gw_profile_read(ctx.handle)
    gw._lib.gw_profile_enable(ctx.handle, 0)
    return ms / max(nl, 1), nl


def tmarg_leg(gw, torch, ctx, theta, steps, warmup, mixed_value):
    """Phase + coalescence-time marginal on the same 4096 proposals of the
    128 s band: grid t_j = j / 16384 s over |t| <= 0.1 s (3273 points, R = 4),
    block moments of 512 bins (K Chebyshev orders) and K FFTs of 4096 points
    per proposal; k_tmom and k_tgrid timed separately with HIP events."""
    n = theta.shape[0]
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    delta, n_t, p_len, blk = gw.gw_time_grid_info(ctx.handle)
    R = 4
    L = p_len * R
    jmax = (n_t - 1) // 2
    K = tgrid_orders(L, jmax)
    res = {}
    for name, prec in (("mixed", gw.GW_PREC_MIXED), ("fp64", gw.GW_PREC_FP64)):
        run = lambda: ctx.loglike(theta, gw.GW_FULL, gw.GW_MARG_PHASE_TIME, prec, out=out)
        for _ in range(warmup):
            run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            run()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        mom_ms, _ = time_kernel(gw, torch, ctx, run, steps, 1)
        grid_ms, _ = time_kernel(gw, torch, ctx, run, steps, 2)
        r = {"value": n / dt, "ms_per_batch": dt * 1e3, "k_tmom_ms": mom_ms, "k_tgrid_ms": grid_ms}
        gflops = tgrid_flops_per_row(K, L) * n
        r["k_tgrid_roofline"] = {"bound": "alu", "achieved": gflops / (grid_ms * 1e-3) / 1e12,
                                 "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                                 "frac": gflops / (grid_ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
                                 "flops_per_row": tgrid_flops_per_row(K, L)}
        if name == "mixed":
            mflops = tmom_flops_per_bin(K) * n * prob_n_freq(ctx)
            r["k_tmom_roofline"] = {"bound": "alu", "achieved": mflops / (mom_ms * 1e-3) / 1e12,
                                    "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                                    "frac": mflops / (mom_ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
                                    "flops_per_bin": tmom_flops_per_bin(K)}
        res[name] = r
    res["cost_vs_distance_marginal_mixed"] = mixed_value / res["mixed"]["value"]
    res.update({"unit": "logL evals/s", "batch": n, "grid_points": n_t, "delta_s": delta, "blocks_P": p_len,
                "fft_len": L, "orders": K, "block_bins": blk,
                "workload": "phase+time marginal on the 128 s full band, 4096 prior draws, t_c grid of a quarter "
                            "of the segment's sampling interval over +-0.1 s"})
    return res


def prob_n_freq(ctx):
    return int(ctx.n_freq)


def nested_full_leg(gw, torch):
    """Nested sampling on the full band (128 s, 259,585 bins per detector,
    mixed form), settings as the heterodyned run, with and without the
    waveform cache of the fast blocks."""
    import gwsynth
    from paper_2607_28265_amd import prescreen as P
    from paper_2607_28265_amd.nested import NestedSampler
    cfg = gwsynth.CONFIGS["cfg2"]
    prob = gwsynth.make_problem(cfg["duration"], cfg["f_min"], cfg["f_max"], psd_scale=1e-49)
    th = gwsynth.prior_draws(gwsynth.SEEDS["injection"], 1)[0]
    th_inj = P.library_injection(gw.Context, prob, th, snr=24.0)
    out = {}
    pre_cfg = dict(start=100, every=50, audit=0.01)
    with gw.Context(prob) as ctx:
        for name, cache, pre in (("no_cache", False, None), ("cache", True, None), ("prescreen", False, pre_cfg)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ns = NestedSampler(ctx, n_live=1000, n_delete=125, seed=gwsynth.SEEDS["sampler"], like=gw.GW_FULL,
                               prec=gw.GW_PREC_MIXED, cache=cache, prescreen=pre)
            r = ns.run()
            wall = time.perf_counter() - t0
            ns.close()
            d = {"wall_s": wall, "log_z": r["log_z"], "log_z_err": r["log_z_err"], "iterations": r["iterations"],
                 "n_evals": r["n_evals"], "accepted_proposals": r["moves"],
                 "accepted_proposals_per_s": r["moves"] / wall}
            if cache:
                d["evals_full_cachedwaveform_cachedsums"] = r["eval_kinds"]
            if pre is not None:
                p = r["prescreen"]
                d["prescreen"] = {"settings": pre, "screened": p["screened"], "audited": p["audited"],
                                  "audited_inside_false_negatives": p["audited_inside"],
                                  "trainings": p["trainings"], "train_s": p["train_s"], "margin_last": p["margin"],
                                  "accepted_proposals_per_s_excluding_training":
                                      r["moves"] / max(wall - p["train_s"], 1e-9)}
            out[name] = d
    out["workload"] = ("nested sampling on the full band: 1000 live points, 125 deletions, 7 Gibbs blocks, "
                       "128 s at 259,585 bins per detector, mixed form, phase+distance marginalised, dlogz 0.1, "
                       "SNR-24 injection; without and with the waveform cache, and with the learned prescreen in "
                       "the sweeps (trained on the run's dead and live points from iteration 100, every 50)")
    return out


def recon_leg(gw, torch, ctx, theta, steps, warmup, dt_like):
    """Post-hoc reconstruction of (d_L, phi_c) for the 4096 proposals of the
    128 s band (mixed form): the likelihood pass that stages each overlap,
    then one wave per sample draws on the 1000-point distance grid and the
    2048-point phase grid."""
    import numpy as np
    n = theta.shape[0]
    uni = torch.from_numpy(np.random.default_rng(8).uniform(size=(n, 2))).cuda()
    for _ in range(warmup):
        gw.gw_reconstruct(ctx.handle, theta, uni, like=gw.GW_FULL, marg=gw.GW_MARG_PHASE_DIST, prec=gw.GW_PREC_MIXED)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        gw.gw_reconstruct(ctx.handle, theta, uni, like=gw.GW_FULL, marg=gw.GW_MARG_PHASE_DIST, prec=gw.GW_PREC_MIXED)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    return {"value": n / dt, "unit": "samples/s", "ms_per_batch": dt * 1e3, "batch": n,
            "draw_ms_over_likelihood": dt * 1e3 - dt_like * 1e3,
            "workload": "post-hoc d_L and phi_c for 4096 samples of the 128 s band (likelihood pass included), "
                        "1000 distance nodes, 2048 phase nodes"}


def fiducial_leg(gw, torch, pop=8192, gens=300):
    """Maximum-likelihood fiducial search on the loud 128 s injection: a box
    narrowed in chirp mass (+-0.002 Msun) and t_c (+-5 ms) around the event,
    all other coordinates over their whole prior range; then the heterodyne
    (500 bins) from the found point against the one from the true point, on
    2048 draws near the posterior."""
    import numpy as np
    import gwsynth
    from paper_2607_28265_amd import prescreen as P
    from paper_2607_28265_amd.pp import to_cube
    cfg = gwsynth.CONFIGS["cfg2"]
    prob = gwsynth.make_problem(cfg["duration"], cfg["f_min"], cfg["f_max"], psd_scale=1e-49)
    th = gwsynth.prior_draws(gwsynth.SEEDS["injection"], 1)[0]
    th_inj = P.library_injection(gw.Context, prob, th, snr=24.0)
    u_inj = to_cube(th_inj, 10.0, 200.0, False)
    lo, hi = np.zeros(11), np.ones(11)
    lo[0], hi[0] = max(0.0, u_inj[0] - 0.002 / 0.3), min(1.0, u_inj[0] + 0.002 / 0.3)
    lo[10], hi[10] = max(0.0, u_inj[10] - 0.005 / 0.2), min(1.0, u_inj[10] + 0.005 / 0.2)
    out = {}
    with gw.Context(prob) as ctx:
        x = torch.from_numpy(lo + (hi - lo) * np.random.default_rng(12).uniform(size=(pop, 11))).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fx, best = gw.gw_fiducial_search(ctx.handle, x, gens, seed=13, lo=lo, hi=hi, prec=gw.GW_PREC_MIXED)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ti = torch.from_numpy(th_inj[None, :].copy()).cuda()
        f_inj = float(ctx.loglike(ti, gw.GW_FULL, gw.GW_MARG_PHASE_DIST, gw.GW_PREC_FP64).item())
        near = torch.from_numpy(gwsynth.near_posterior(14, th_inj, 2048, scale=0.5)).cuda()
        full = ctx.loglike(near, gw.GW_FULL, gw.GW_MARG_PHASE_DIST, gw.GW_PREC_FP64)
        errs = {}
        for name, fid in (("found", best), ("true", th_inj)):
            ctx.heterodyne_setup(fid, 500)
            het = ctx.loglike(near, gw.GW_HET, gw.GW_MARG_PHASE_DIST, gw.GW_PREC_FP64)
            errs[name] = float(torch.max(torch.abs(het - full)).item())
        out = {"wall_s": wall, "pop": pop, "generations": gens, "evals": pop * (gens + 1),
               "evals_per_s": pop * (gens + 1) / wall, "best_logl": float(fx.max().item()), "injection_logl": f_inj,
               "best_minus_injection": float(fx.max().item()) - f_inj,
               "het500_max_abs_err_near_posterior": errs,
               "found_minus_true": {"mc": float(best[0] - th_inj[0]), "tc_ms": float(1e3 * (best[12] - th_inj[12]))},
               "workload": "differential evolution (DE/rand/1/bin, F 0.6, CR 0.9) on the full-band phase+distance "
                           "marginal of the 128 s SNR-24 injection; box: chirp mass +-0.002 Msun, t_c +-5 ms, "
                           "the rest of the unit cube free"}
    return out


def copy_leg(torch, reps=5, mib=256):
    """A plain device copy of known size, the reference for the HBM byte
    counters (FETCH_SIZE, WRITE_SIZE) of the kernels above."""
    a = torch.ones(mib * (1 << 20) // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    return {"bytes_read_per_copy": a.numel() * 8, "bytes_written_per_copy": a.numel() * 8, "reps": reps}


def mlp_leg(gw, torch, ctx, reps):
    """BF16 inference of the prescreen network (11 -> 256 -> 256 -> 256 -> 1,
    GELU; random weights) on 65,536 unit-cube rows, the kernel timed with HIP
    events on the stream it runs on."""
    import numpy as np
    n = 65536
    rng = np.random.default_rng(17)
    x = torch.from_numpy(rng.random((n, 11))).cuda()
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    net = gw.Mlp(ctx, seed=7)
    try:
        net.set_scaling(np.full(11, 0.5), np.full(11, 0.29), 0.0, 1.0)
        for _ in range(3):
            net.forward(x, out=out)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            net.forward(x, out=out)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
    finally:
        net.close()
    flops = 2.0 * (11 * 256 + 2 * 256 * 256 + 256) * n
    return {"rows": n, "ms_per_call": ms, "tflops": flops / (ms * 1e-3) / 1e12, "peak_bf16_tflops": 2500.0,
            "frac": flops / (ms * 1e-3) / 1e12 / 2500.0,
            "workload": "prescreen network inference, 65,536 rows, BF16 matrix cores with FP32 accumulation"}


def cpu_baseline(gw, torch, batch: int, n_target_cpu_s: float = 16.0):
    """The FP64 oracle on the host cores, on a bounded sample of the headline
    workload (the first rows of its batch), timed; then the same rows' GPU
    values, taken from a full headline batch in the headline launch
    configuration on a context built from the oracle's data, are compared with
    the oracle's: dlogL = GPU - oracle.  The data differ from the headline
    problem's only in who made the injection (the oracle's template here, the
    library's there; both the same TaylorF2 of the same parameters).  Config 1
    (8 s, no marginalisation, all 1024 draws) is compared the same way."""
    import numpy as np
    import gwsynth
    from oracle import likelihood as L
    cores = len(os.sched_getaffinity(0))

    def oracle_problem(name):
        cfg = gwsynth.CONFIGS[name]
        prob = gwsynth.make_problem(cfg["duration"], cfg["f_min"], cfg["f_max"], psd_scale=cfg["psd_scale"])
        th_inj = gwsynth.prior_draws(gwsynth.SEEDS["injection"], 1)[0]
        prob.data = prob.data + L.strain(th_inj, prob)
        return prob, th_inj

    def stats(got, ref):
        d = np.abs(got - ref)
        return {"max": float(d.max()), "p99": float(np.quantile(d, 0.99)), "n": int(d.size)}

    prob, th_inj = oracle_problem("cfg2")
    t0 = time.perf_counter()
    L.loglike(th_inj, prob, L.PHASE_DIST)
    one = time.perf_counter() - t0
    n = int(max(cores, min(64 * cores, n_target_cpu_s / max(one, 1e-3))))
    th = gwsynth.prior_draws(gwsynth.SEEDS["prior"], max(n, batch))
    t0 = time.perf_counter()
    ref = L.loglike_many(th[:n], prob, L.PHASE_DIST, processes=cores)
    dt = time.perf_counter() - t0
    out = {"value": n / dt, "unit": "logL evals/s", "cores": cores, "kind": "oracle",
           "sample": f"the first {n} of the 4096 prior draws of the 128 s full-band workload, phase+distance "
                     f"marginalised, NumPy FP64 oracle over a {cores}-process pool ({dt:.1f} s wall)"}
    dl = {}
    theta = torch.from_numpy(th[:batch]).cuda()
    with gw.Context(prob) as ctx:
        for name, prec in (("mixed", gw.GW_PREC_MIXED), ("fp64", gw.GW_PREC_FP64)):
            got = ctx.loglike(theta, marg=gw.GW_MARG_PHASE_DIST, prec=prec).cpu().numpy()
            dl[name] = stats(got[:n], ref)
    dl["rows"] = f"the first {n} rows of the 4096-row headline batch (evaluated as a whole batch)"
    prob1, _ = oracle_problem("cfg1")
    th1 = gwsynth.prior_draws(gwsynth.SEEDS["prior"], 1024)
    ref1 = L.loglike_many(th1, prob1, L.PLAIN, processes=cores)
    cfg1 = {}
    with gw.Context(prob1) as ctx:
        t1 = torch.from_numpy(th1).cuda()
        for name, prec in (("fp64", gw.GW_PREC_FP64), ("mixed", gw.GW_PREC_MIXED)):
            cfg1[name] = stats(ctx.loglike(t1, marg=gw.GW_MARG_NONE, prec=prec).cpu().numpy(), ref1)
    cfg1["rows"] = "all 1024 prior draws of the 8 s workload, no marginalisation"
    dl["cfg1_plain"] = cfg1
    return out, dl


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported; the benchmark runs on a single GPU "
              "(the batch shards by proposal across GPUs with no exchange but the logL gather).",
              file=sys.stderr, flush=True)
        sys.exit(2)
    import numpy as np
    import torch
    import gwsynth
    import paper_2607_28265_amd as gw

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    prob, th_inj = make_problem_gpu(gw, torch)
    n = args.batch
    th = gwsynth.prior_draws(gwsynth.SEEDS["prior"], n)
    theta = torch.from_numpy(th).cuda()
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    marg = gw.GW_MARG_PHASE_DIST
    with gw.Context(prob) as ctx:
        dt_mix, k_mix = time_steps(ctx, theta, out, args.steps, args.warmup, gw.GW_PREC_MIXED, marg, torch, gw,
                                   profile=True)
        mix = out.clone()
        fp_steps = max(5, args.steps // 2)
        dt_fp, k_fp = time_steps(ctx, theta, out, fp_steps, 2, gw.GW_PREC_FP64, marg, torch, gw, profile=True)
        fp = out.clone()
        dlogl = float(torch.max(torch.abs(mix - fp)).item())
        fpb_mixed = mixed_flops_per_bin(gw, ctx, int(prob.n_freq))
        tm = None
        if "tmarg" in set(args.legs.split(",")):
            tm = tmarg_leg(gw, torch, ctx, theta, max(5, args.steps // 2), 2, n * args.steps / dt_mix)
        rc = None
        if "recon" in set(args.legs.split(",")):
            rc = recon_leg(gw, torch, ctx, theta, max(5, args.steps // 2), 2, dt_mix / args.steps)
        ml = None
        if "mlp" in set(args.legs.split(",")):
            ml = mlp_leg(gw, torch, ctx, max(10, args.steps))
    value = n * args.steps / dt_mix
    fp_value = n * fp_steps / dt_fp
    units = n * prob.n_freq
    ach = fpb_mixed * units / (k_mix * 1e-3) / 1e12
    ach_fp = FLOPS_PER_BIN["fp64"] * units / (k_fp * 1e-3) / 1e12
    res = {
        "metric": METRIC,
        "value": value,
        "unit": "logL evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt_mix / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {"workload": "full-band BNS likelihood: TaylorF2 3.5PN aligned-spin+tidal, 3 detectors, "
                               "T=128 s, 20-2048 Hz, df=1/128 Hz (259,585 bins/detector), batch 4096 prior "
                               "draws, phase+distance marginalised; mixed form (FP64 phase by a cubic "
                               "recurrence in runs of bins, FP32 sin/cos, FP64 sums)",
                   "batch": n, "n_freq": int(prob.n_freq), "n_det": 3, "marg": "phase+distance",
                   "prec": "mixed"},
        "roofline": {"bound": "alu", "achieved": ach, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": ach / PEAK_FP64_TFLOPS, "traffic": traffic_bytes(), "traffic_unit": "bytes/launch",
                     "hbm_gbs": (traffic_bytes() / (k_mix * 1e-3) / 1e9) if traffic_bytes() else None,
                     "hbm_peak_gbs": 8000.0,
                     "kernel": "k_full<3,1> (mixed)", "kernel_ms": k_mix,
                     "flops_per_launch": fpb_mixed * units, "flops_per_bin": fpb_mixed},
        "fp64_plain": {"value": fp_value, "ms_per_step": dt_fp / fp_steps * 1e3, "kernel_ms": k_fp,
                       "roofline_frac": ach_fp / PEAK_FP64_TFLOPS},
        "speedup_vs_fp64": value / fp_value,
        "mixed_vs_fp64_max_dlogl": dlogl,
    }
    legs = set(args.legs.split(","))
    log(f"full-band legs done: {value:.4g} evals/s mixed")
    if "het" in legs:
        res["heterodyned"] = het_leg(gw, torch, prob, th_inj, max(5, args.steps // 2), 2)
        log("heterodyned leg done")
    if tm is not None:
        res["time_marginal"] = tm
    if rc is not None:
        res["reconstruction"] = rc
    if ml is not None:
        res["mlp_inference"] = ml
    if "cache" in legs:
        res["waveform_cache"] = cache_leg(gw, torch, prob, args.steps, args.warmup, value)
        log("cache leg done")
    if "fiducial" in legs:
        res["fiducial_search"] = fiducial_leg(gw, torch)
        log("fiducial leg done")
    if "nested" in legs:
        res["nested_sampling"] = nested_leg(gw, torch)
        log("nested-sampling leg done")
    if "nested_tmarg" in legs:
        res["nested_sampling_time_marginal"] = nested_tmarg_leg(gw, torch)
        log("time-marginal nested-sampling leg done")
    if "nested_full" in legs:
        res["nested_sampling_full_band"] = nested_full_leg(gw, torch)
        log("full-band nested-sampling leg done")
    if "prescreen" in legs:
        res["prescreen"] = prescreen_leg(gw, torch, 10)
        log("prescreen leg done")
    if "copy" in legs:
        res["copy_calibration"] = copy_leg(torch)
    if "cfg1" in legs:
        res["cfg1_plain_fp64"] = cfg1_leg(gw, torch, args.steps, args.warmup)
        log("config-1 leg done")
    if not args.no_cpu_baseline:
        res["cpu_baseline"], res["dlogl_vs_oracle"] = cpu_baseline(gw, torch, n)
        log("cpu baseline done")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
