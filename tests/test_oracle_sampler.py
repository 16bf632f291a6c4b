"""Pins of the sampler oracle: Philox against NumPy's Philox, the prior
transform, slice-step invariance and nested sampling on a Gaussian with a
known evidence."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import sampler as S


def test_philox_matches_numpy():
    # NumPy's Philox bit generator is Philox4x64-10; it increments the counter
    # before producing a block, so its first block is ours at counter + 1.
    def inc(c):  # 256-bit counter increment with carry
        v = sum(int(w) << (64 * i) for i, w in enumerate(c)) + 1
        return [(v >> (64 * i)) & (2 ** 64 - 1) for i in range(4)]

    for key, ctr in [(0, [0, 0, 0, 0]), (0x1234567890ABCDEF, [5, 7, 9, 11]), (2 ** 64 - 1, [2 ** 64 - 2, 3, 0, 1])]:
        bg = np.random.Philox(key=np.array([key, 0], dtype=np.uint64), counter=np.array(ctr, dtype=np.uint64))
        raw = [int(v) for v in bg.random_raw(8)]
        c1 = inc(ctr)
        assert S.philox4x64(c1, (key, 0)) == raw[:4]
        assert S.philox4x64(inc(c1), (key, 0)) == raw[4:]


def test_philox_uniforms_range_and_uniformity():
    u = np.concatenate([S.philox_uniforms(7, 3, c, 64) for c in range(64)])
    assert np.all((u > 0) & (u < 1))
    assert stats.kstest(u, "uniform").pvalue > 1e-3


def test_prior_transform():
    th = S.prior_transform(np.zeros(11))
    assert np.allclose(th[:6], [1.1, 0.5, -0.05, -0.05, 0, 0])
    assert th[7] == 0.0 and th[8] == 0.0 and abs(th[9] + math.pi / 2) < 1e-15 and th[12] == -0.1
    th = S.prior_transform(np.ones(11))
    assert np.allclose(th[:6], [1.4, 1.0, 0.05, 0.05, 5000, 5000])
    assert abs(th[7] - math.pi) < 1e-15 and abs(th[9] - math.pi / 2) < 1e-15
    # isotropic inclination and declination: cos(iota), sin(dec) uniform
    u = np.random.default_rng(0).uniform(size=(4000, 11))
    t = np.array([S.prior_transform(x) for x in u])
    assert stats.kstest(np.cos(t[:, 7]), "uniform", args=(-1, 2)).pvalue > 1e-3
    assert stats.kstest(np.sin(t[:, 9]), "uniform", args=(-1, 2)).pvalue > 1e-3


def test_slice_step_keeps_uniform_on_a_ball():
    # P17: uniform on a ball (the constrained prior of logL = -|x - c|^2) is
    # invariant under the slice step; radial CDF (r / R)^d and a marginal stay
    # uniform after many updates.
    d, n, rad = 3, 1500, 0.3
    rng = np.random.default_rng(1)
    c = np.full(d, 0.5)
    g = rng.normal(size=(n, d))
    x = c + rad * (g / np.linalg.norm(g, axis=1, keepdims=True)) * rng.uniform(size=(n, 1)) ** (1 / d)
    loglike = lambda p: -float(np.sum((p - c) ** 2))
    lstar = -rad * rad
    chol = np.linalg.cholesky(np.cov(x, rowvar=False))
    logl = np.array([loglike(p) for p in x])
    for step in range(6):
        for i in range(n):
            uni = S.philox_uniforms(11, step, i, S.N_UNIFORM_FIXED + 100)
            x[i], logl[i], _, st, _ = S.slice_chain(x[i], logl[i], lstar, (0, 1, 2), chol, uni, loglike, w=0.5)
            assert st == 0
    r = np.linalg.norm(x - c, axis=1) / rad
    assert np.all(r < 1)
    assert stats.kstest(r ** d, "uniform").pvalue > 1e-3
    # marginal of a uniform ball along one axis: density ~ 1 - s^2 on [-1, 1]
    s = (x[:, 0] - c[0]) / rad
    cdf = lambda v: 0.5 + 0.75 * (v - v ** 3 / 3)
    assert stats.kstest(s, cdf).pvalue > 1e-3


def test_unblocked_slice_step_keeps_uniform_on_an_11_ball():
    # P17 for one block holding every coordinate (the unblocked nested slice
    # sampler): 6 Box-Muller pairs give the direction, the bracket offset is
    # uniform 12 and the shrink draws follow.  Uniform on an 11-ball stays
    # uniform: radial CDF r^11, one coordinate (s + 1) / 2 ~ Beta(6, 6).
    d, n, rad = 11, 600, 0.3
    assert S.n_direction_uniforms(d) == 12 and S.n_fixed_uniforms(d) == 13
    assert S.n_fixed_uniforms(4) == S.N_UNIFORM_FIXED == S.n_fixed_uniforms(1)
    rng = np.random.default_rng(2)
    c = np.full(d, 0.5)
    g = rng.normal(size=(n, d))
    x = c + rad * (g / np.linalg.norm(g, axis=1, keepdims=True)) * rng.uniform(size=(n, 1)) ** (1 / d)
    loglike = lambda p: -float(np.sum((p - c) ** 2))
    lstar = -rad * rad
    chol = np.linalg.cholesky(np.cov(x, rowvar=False))
    logl = np.array([loglike(p) for p in x])
    block = tuple(range(d))
    for step in range(5):
        for i in range(n):
            uni = S.philox_uniforms(12, step, i, S.n_fixed_uniforms(d) + 100)
            x[i], logl[i], _, st, _ = S.slice_chain(x[i], logl[i], lstar, block, chol, uni, loglike, w=0.5)
            assert st == 0
    r = np.linalg.norm(x - c, axis=1) / rad
    assert np.all(r < 1)
    assert stats.kstest(r ** d, "uniform").pvalue > 1e-3
    s = (x[:, 3] - c[3]) / rad
    assert stats.kstest((s + 1) / 2, stats.beta(6, 6).cdf).pvalue > 1e-3


def test_slice_step_block_moves_only_block():
    x0 = np.full(11, 0.5)
    uni = S.philox_uniforms(3, 0, 0, S.N_UNIFORM_FIXED + 100)
    x, v, ne, st, _ = S.slice_chain(x0, 0.0, -1.0, (7, 8), 0.1 * np.eye(2), uni, lambda p: 0.0)
    assert st == 0 and ne >= 1
    mask = np.ones(11, bool)
    mask[[7, 8]] = False
    assert np.array_equal(x[mask], x0[mask]) and not np.array_equal(x[[7, 8]], x0[[7, 8]])


@pytest.mark.slow
def test_nested_sampling_gaussian_evidence():
    # P16: a normalised Gaussian likelihood well inside the unit cube has
    # Z = 1 (log Z = 0) under the uniform prior; the estimate must fall within
    # 3 sigma, sigma = sqrt(H / m).
    d, sig = 6, 0.06
    mu = np.full(d, 0.5)

    def loglike(x):
        return float(-0.5 * np.sum(((x - mu) / sig) ** 2) - d * math.log(sig * math.sqrt(2 * math.pi)))

    blocks = ((0, 1), (2,), (3, 4), (5,))
    res = S.nested_sampling(loglike, n_live=150, n_delete=20, seed=5, dlogz=0.1, blocks=blocks, n_dim=d,
                            max_shrink=60)
    assert abs(res["log_z"]) < 3 * res["log_z_err"] + 0.05, res["log_z"]
    assert res["h"] > 5


def test_time_marginal_transform_samples_a_d_squared_prior():
    # coordinate 10 carries d_L with density proportional to d^2 on [10, 200]:
    # KS test against the CDF (d^3 - 10^3) / (200^3 - 10^3); the other columns
    # are those of the default transform, and t_c is zero
    from scipy import stats
    rng = np.random.default_rng(4)
    u = rng.uniform(size=(4000, 11))
    th = np.array([S.prior_transform_time(x, 10.0, 200.0) for x in u])
    cdf = lambda d: (d ** 3 - 1e3) / (200.0 ** 3 - 1e3)
    assert stats.kstest(th[:, 6], cdf).pvalue > 1e-3
    assert np.all(th[:, 12] == 0.0)
    ref = np.array([S.prior_transform(x) for x in u[:10]])
    assert np.array_equal(np.delete(th[:10], [6, 12], axis=1), np.delete(ref, [6, 12], axis=1))
    assert S.prior_transform_time(np.zeros(11), 10.0, 200.0)[6] == pytest.approx(10.0, rel=1e-15)
    assert S.prior_transform_time(np.ones(11), 10.0, 200.0)[6] == pytest.approx(200.0, rel=1e-15)


def test_detector_frame_sky_is_isotropic_and_keeps_the_baseline_delay():
    # The detector sky frame (zenith and azimuth about the baseline of
    # detectors 0 and 1): uniform u gives an isotropic sky (sin dec and ra
    # uniform); the delay between the two detectors depends on the zenith
    # only, -|r_1 - r_0| cos(zenith) / c, whatever the azimuth; u_zen = 0
    # points along the baseline.  Delays come from the detector module's own
    # (ra, dec) path, with a non-zero GMST.
    from oracle import detector as D
    import gwsynth
    pos, _ = gwsynth.detectors()
    gmst = 1.234
    rng = np.random.default_rng(3)
    u = rng.uniform(size=(4000, 2))
    rd = np.array([S.detector_frame_sky(a, b, pos, gmst)[:2] for a, b in u])
    assert stats.kstest(np.sin(rd[:, 1]), "uniform", args=(-1, 2)).pvalue > 1e-3
    assert stats.kstest(rd[:, 0], "uniform", args=(0, 2 * math.pi)).pvalue > 1e-3
    base = np.linalg.norm(pos[1] - pos[0])
    for uz in (0.1, 0.37, 0.5, 0.93):
        want = -base * (1 - 2 * uz) / S.C_SI
        for ua in rng.uniform(size=5):
            ra, dec, _ = S.detector_frame_sky(ua, uz, pos, gmst)
            got = D.time_delay(pos[1], ra, dec, gmst) - D.time_delay(pos[0], ra, dec, gmst)
            assert abs(got - want) < 1e-15
    n, _, _ = S.sky_frame_basis(pos)
    for ua in (0.0, 0.3, 0.8):
        _, _, s = S.detector_frame_sky(ua, 0.0, pos, gmst)
        assert np.allclose(s, n, rtol=0, atol=1e-15)


def test_detector_frame_time():
    # with det_time, coordinate 10 is the arrival time at detector 0:
    # t_c + dt_0(ra, dec) equals -0.1 + 0.2 u_10; the other columns are those
    # of the plain transform, apart from the sky
    from oracle import detector as D
    import gwsynth
    pos, _ = gwsynth.detectors()
    rng = np.random.default_rng(4)
    for u in rng.uniform(size=(20, 11)):
        th = S.prior_transform_frame(u, pos, 0.7, det_time=True)
        ta = th[12] + D.time_delay(pos[0], th[8], th[9], 0.7)
        assert abs(ta - (-0.1 + 0.2 * u[10])) < 1e-15
        plain = S.prior_transform(u)
        keep = [0, 1, 2, 3, 4, 5, 6, 7, 10, 11]
        assert np.array_equal(th[keep], plain[keep])
        tt = S.prior_transform_frame(u, pos, 0.7, d_range=(10.0, 200.0))
        assert np.array_equal(tt[[6, 12]], S.prior_transform_time(u, 10.0, 200.0)[[6, 12]])
