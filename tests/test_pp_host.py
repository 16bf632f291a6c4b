"""Host logic of the injection-campaign driver against the oracle (no GPU):
the driver's unit-cube inverse and truth draws in both sky frames, and its
credible levels and p-values on synthetic samples; the event pipeline's
weighted posterior summary."""
import math

import numpy as np

import gwsynth
from oracle import pp as OPP
from oracle import sampler as S
from paper_2607_28265_amd import pp


def test_to_cube_inverts_the_oracle_transform():
    pos, _ = gwsynth.detectors()
    rng = np.random.default_rng(1)
    keep = [0, 1, 2, 3, 4, 5, 7, 8, 9, 10]  # not d_L (marginalised)
    for det_time in (False, True):
        frame = pp.SkyFrame(pos, 0.4, det_time=det_time)
        for u in rng.uniform(0.01, 0.99, size=(50, 11)):
            th = S.prior_transform_frame(u, pos, 0.4, det_time=det_time)
            assert np.allclose(pp.to_cube(th, 10.0, 200.0, False, frame)[keep], u[keep], atol=1e-10)
            tt = S.prior_transform_frame(u, pos, 0.4, d_range=(10.0, 200.0))
            assert np.allclose(pp.to_cube(tt, 10.0, 200.0, True, pp.SkyFrame(pos, 0.4)), u, atol=1e-10)
    for u in rng.uniform(0.01, 0.99, size=(50, 11)):
        assert np.allclose(pp.to_cube(S.prior_transform(u), 10.0, 200.0, False)[keep], u[keep], atol=1e-12)


def test_truth_draws_follow_the_transform():
    pos, _ = gwsynth.detectors()
    for frame in (None, pp.SkyFrame(pos, 0.4), pp.SkyFrame(pos, 0.4, det_time=True)):
        rng = np.random.default_rng(2)
        for _ in range(30):
            th = pp.draw_truth(rng, 10.0, 200.0, False, frame)
            u = pp.to_cube(th, 10.0, 200.0, False, frame)
            assert np.all((u > -1e-12) & (u < 1 + 1e-12))
            if frame is None:
                back = S.prior_transform(u)
            else:
                back = S.prior_transform_frame(u, pos, 0.4, det_time=frame.det_time)
            keep = [0, 1, 2, 3, 4, 5, 7, 8, 9, 10, 12]
            d = np.abs(back[keep] - th[keep])
            d[7] = min(d[7], 2 * math.pi - d[7])
            assert np.all(d < 1e-10)
            assert 10.0 <= th[6] <= 200.0 and 0.0 <= th[11] < 2 * math.pi


def test_levels_and_pvalues_match_oracle():
    rng = np.random.default_rng(3)
    x = rng.normal(size=500)
    w = rng.uniform(size=500)
    for t in (-1.0, 0.0, 0.3, 2.5):
        assert pp.weighted_level(x, w, t) == OPP.credible_level(x, w, t)
    q = rng.uniform(size=40)
    assert pp.ks_pvalue(q) == OPP.ks_pvalue(q)
    assert pp.fisher_pvalue([0.2, 0.5, 0.01]) == OPP.fisher_combined([0.2, 0.5, 0.01])


def test_event_weighted_stats():
    from paper_2607_28265_amd.event import weighted_stats
    rng = np.random.default_rng(4)
    x, w = rng.normal(size=200), rng.uniform(size=200)
    m, sd = weighted_stats(x, w)
    assert abs(m - np.average(x, weights=w)) < 1e-12
    assert abs(sd - math.sqrt(np.cov(x, aweights=w, ddof=0))) < 1e-12


def test_event_circular_stats():
    from paper_2607_28265_amd.event import weighted_circular_stats
    # two points either side of 0: the mean is 0, not pi
    m, sd = weighted_circular_stats(np.array([0.1, 2 * math.pi - 0.1]), np.array([1.0, 1.0]))
    assert min(m, 2 * math.pi - m) < 1e-12 and abs(sd - math.sqrt(-2 * math.log(math.cos(0.1)))) < 1e-12
    # a narrow wrapped normal: circular sd close to sigma
    rng = np.random.default_rng(8)
    x = (3.0 + 0.05 * rng.standard_normal(20000)) % (2 * math.pi)
    m, sd = weighted_circular_stats(x, np.ones_like(x))
    assert abs(m - 3.0) < 2e-3 and abs(sd - 0.05) < 2e-3
