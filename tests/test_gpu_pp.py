"""GPU injection campaign (P-P test machinery) against the oracle.

A small campaign on the 8 s, 20-512 Hz grid checks every step that the
campaign adds to the sampler:
  * the injected data equal the seeded noise plus the oracle's template of the
    true parameters;
  * the true parameters' unit-cube coordinates map back to them through the
    oracle's prior transform;
  * the credible levels, the KS and Fisher p-values, and the levels of the
    post-hoc d_L and phi_c all equal the oracle's statistics on the same
    samples and weights.
"""
import math

import numpy as np
import pytest

import gwsynth
from oracle import likelihood as L
from oracle import pp as OPP
from oracle import sampler as S

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def campaign():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_2607_28265_amd import pp
    base = gwsynth.make_problem(8.0, 20.0, 512.0, psd_scale=1e-49, noise_seed=None)
    camp = pp.Campaign(base, config="baseline", n_live=128, n_delete=16, n_bins=200, seed=11)
    yield pp, camp, base
    camp.close()


def test_injection_data_and_truth(campaign):
    pp, camp, base = campaign
    for i in range(3):
        th, prob, nseed = camp.make_data(i)
        h = L.strain(th, base)
        want = gwsynth.gaussian_noise(nseed, base.psd, base.df) + h
        assert np.max(np.abs(prob.data - want)) < 1e-9 * np.max(np.abs(h))
        u = pp.to_cube(th, camp.d_lo, camp.d_hi, False)
        assert np.all((u >= 0) & (u <= 1))
        back = S.prior_transform(u)
        keep = [0, 1, 2, 3, 4, 5, 7, 8, 9, 10, 12]  # all but d_L and phi_c
        assert np.allclose(back[keep], th[keep], rtol=1e-12, atol=1e-12)
        assert base.dist_grid[0] <= th[6] <= base.dist_grid[-1] and 0 <= th[11] < 2 * math.pi


def test_campaign_statistics_match_oracle(campaign):
    pp, camp, base = campaign
    runs = []
    for i in range(4):
        r = camp.run_injection(i, keep=True)
        truth = pp.to_cube(np.array(r["truth"]), camp.d_lo, camp.d_hi, False)
        for j in range(11):
            assert r["levels"][j] == OPP.credible_level(r["x"][:, j], r["w"], truth[j])
        ws = r["w"][r["sel"]]
        assert r["level_dl"] == OPP.credible_level(r["recon"][:, 0], ws, r["truth"][6])
        assert r["level_phic"] == OPP.credible_level(r["recon"][:, 1], ws, r["truth"][11])
        assert np.all(np.isin(r["recon"][:, 0], base.dist_grid))
        assert math.isfinite(r["log_z"]) and r["iterations"] > 10
        print(f"injection {i}: {r['iterations']} it, {r['n_evals']} evals, levels "
              + " ".join(f"{v:.2f}" for v in r["levels"]), flush=True)
        runs.append(r)
    summ = camp.summarise(runs)
    lv = np.array([r["levels"] for r in runs])
    for j, name in enumerate(pp.PARAMS):
        assert summ["ks_pvalues"][name] == OPP.ks_pvalue(lv[:, j])
    assert summ["fisher_p"] == OPP.fisher_combined(list(summ["ks_pvalues"].values()))
    assert summ["ks_reconstructed"]["dl"] == OPP.ks_pvalue([r["level_dl"] for r in runs])


def test_unblocked_configuration_runs(campaign):
    pp, camp, base = campaign
    from paper_2607_28265_amd import pp as ppm
    c2 = ppm.Campaign(base, config="nss", n_live=64, n_delete=8, n_bins=200, seed=11)
    try:
        r = c2.run_injection(0)
    finally:
        c2.close()
    assert math.isfinite(r["log_z"]) and all(0.0 <= v <= 1.0 for v in r["levels"])
