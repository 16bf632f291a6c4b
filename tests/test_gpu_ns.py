"""End-to-end nested sampling on the GPU (heterodyned likelihood, phase and
distance marginalised) against the oracle's own run on the same seeded
problem, sampler settings and seeds (stored by tests/golden/make_ns_golden.py,
which calls only the oracle; three Gibbs sweeps per replacement, the setting
at which runs with different random numbers agree).  The two runs are
separate stochastic estimates once a near tie resolves differently, so log Z
is compared within three combined standard errors sqrt(H/m); a checkpoint
taken mid-run and resumed must reproduce the uninterrupted run exactly.
"""
import json
import math
import os

import numpy as np
import pytest

from tests.gpu_common import problem

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
HERE = os.path.dirname(os.path.abspath(__file__))
# RMS of log Z(screened) - log Z(unscreened) over runs that share a seed (cfg2,
# heterodyned, mixed, three sweeps; see test_prescreened_run_evidence_matches_oracle)
SCREEN_SPREAD = 0.34


def golden(name):
    with open(os.path.join(HERE, "golden", f"ns_{name}.json")) as f:
        return json.load(f)


def run(name, prec, max_iter=100000, checkpoint_at=None, path=None, async_sweep=True):
    import paper_2607_28265_amd as gw
    from paper_2607_28265_amd.nested import NestedSampler
    g = golden(name)
    prob = problem(name, loud=True)
    with gw.Context(prob) as ctx:
        ctx.heterodyne_setup(prob.theta_inj, g["n_bins"])
        ns = NestedSampler(ctx, n_live=g["n_live"], n_delete=g["n_delete"], seed=g["seed"], dlogz=g["dlogz"],
                           like=gw.GW_HET, prec=prec, async_sweep=async_sweep, sweeps=g.get("sweeps", 1))
        if checkpoint_at is not None:
            ns.run(max_iter=checkpoint_at)
            ns.save(path)
            ns2 = NestedSampler(ctx, n_live=g["n_live"], n_delete=g["n_delete"], seed=g["seed"], dlogz=g["dlogz"],
                                like=gw.GW_HET, prec=prec, sweeps=g.get("sweeps", 1))
            ns2.load(path)
            ns = ns2
        return ns.run(max_iter=max_iter)


@pytest.mark.parametrize("name", ["cfg1", "cfg2"])
def test_log_evidence_matches_oracle_run(name):
    import paper_2607_28265_amd as gw
    g = golden(name)
    for prec in (gw.GW_PREC_FP64, gw.GW_PREC_MIXED):
        r = run(name, prec)
        sig = math.hypot(r["log_z_err"], g["log_z_err"])
        print(f"{name} prec {prec}: GPU logZ {r['log_z']:.3f} +- {r['log_z_err']:.3f} ({r['iterations']} it, "
              f"{r['n_evals']} evals, {r['wall_s']:.2f} s); oracle {g['log_z']:.3f} +- {g['log_z_err']:.3f} "
              f"({g['iterations']} it, {g['n_evals']} evals, {g['cpu_wall_s']:.0f} s)")
        assert abs(r["log_z"] - g["log_z"]) < 3.0 * sig
        assert abs(r["iterations"] - g["iterations"]) <= 0.15 * g["iterations"]
        assert abs(r["h"] - g["h"]) < 0.25 * g["h"]


def test_checkpoint_resume_is_exact(tmp_path):
    import paper_2607_28265_amd as gw
    path = str(tmp_path / "ns.npz")
    a = run("cfg1", gw.GW_PREC_MIXED, max_iter=90)
    b = run("cfg1", gw.GW_PREC_MIXED, max_iter=90, checkpoint_at=40, path=path)
    assert a["iterations"] == b["iterations"] == 90
    assert a["log_z"] == b["log_z"] and a["n_evals"] == b["n_evals"]


def test_async_sweep_equals_block_by_block():
    # one slice_sweep call per sweep or one slice_step call per block: the
    # same chains, so the same run
    import paper_2607_28265_amd as gw
    a = run("cfg1", gw.GW_PREC_MIXED, max_iter=60, async_sweep=True)
    b = run("cfg1", gw.GW_PREC_MIXED, max_iter=60, async_sweep=False)
    print(f"async {a['wall_s']:.2f} s, block by block {b['wall_s']:.2f} s")
    assert a["iterations"] == b["iterations"] == 60
    assert a["log_z"] == b["log_z"] and a["n_evals"] == b["n_evals"] and a["h"] == b["h"]


def test_prescreened_run_evidence_matches_oracle():
    # The learned prescreen inside the sampler's sweeps (trained on the
    # candidates the run evaluated exactly and its live set, from iteration
    # 60, retrained every 40): every accepted point keeps an exact log L, and
    # the evidence stays near the oracle's unscreened run.  The audit
    # measures how often a screened-out candidate was in fact inside, and
    # widens the margin when that is often.
    #
    # The two runs draw the same random numbers until the screen first
    # rejects a candidate (iteration 60 of about 230), then go separate ways,
    # so their difference is the scatter of the remaining iterations, which
    # sqrt(H / m) understates: consecutive points of a slice chain are
    # correlated.  Measured on the GPU at these settings: ten unscreened runs
    # with seeds 6..15 spread with standard deviation 0.84 in log Z (sqrt(H /
    # m) = 0.16), and 21 screened runs differ from the unscreened run of the
    # same seed by 0.34 RMS, with no sign of a bias.  The bound is three
    # times that RMS.
    import paper_2607_28265_amd as gw
    from paper_2607_28265_amd.nested import NestedSampler
    g = golden("cfg2")
    prob = problem("cfg2", loud=True)
    with gw.Context(prob) as ctx:
        ctx.heterodyne_setup(prob.theta_inj, g["n_bins"])
        ns = NestedSampler(ctx, n_live=g["n_live"], n_delete=g["n_delete"], seed=g["seed"], dlogz=g["dlogz"],
                           like=gw.GW_HET, prec=gw.GW_PREC_MIXED, sweeps=g.get("sweeps", 1),
                           prescreen=dict(start=60, every=40, audit=0.02))
        r = ns.run()
        ns.close()
    p = r["prescreen"]
    print(f"prescreened run: logZ {r['log_z']:.3f} +- {r['log_z_err']:.3f} ({r['iterations']} it, {r['n_evals']} "
          f"exact evals, {r['wall_s']:.2f} s); screened {p['screened']}, audited {p['audited']} of which inside "
          f"{p['audited_inside']}; {p['trainings']} trainings in {p['train_s']:.2f} s, margin {p['margin']:.3f}; "
          f"oracle {g['log_z']:.3f} +- {g['log_z_err']:.3f}", flush=True)
    assert p["screened"] > 0 and p["audited"] > 0
    assert p["audited_inside"] <= 0.2 * p["audited"] + 1
    assert abs(r["log_z"] - g["log_z"]) < 3.0 * SCREEN_SPREAD
