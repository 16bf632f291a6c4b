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
    # uniform 12, the stepping-out split uniform 13, and the shrink draws follow.  Uniform on an 11-ball stays
    # uniform: radial CDF r^11, one coordinate (s + 1) / 2 ~ Beta(6, 6).
    d, n, rad = 11, 600, 0.3
    assert S.n_direction_uniforms(d) == 12 and S.n_fixed_uniforms(d) == 14
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


def test_stepping_out_budget_split_keeps_uniform_when_caps_bind():
    # Stepping out with a budget m = 2 max_out + 1 split at random between the
    # ends (Neal 2003, Sec. 4.1) gives every point of the final bracket the
    # same chance of producing it, so the move leaves the constrained uniform
    # invariant even when the cap binds on every move (here: a region 0.6 wide,
    # w = 0.3, max_out = 1).  Capping each end at max_out on its own does not:
    # in this set-up its histogram after 10 steps fails the same test
    # (p ~ 2e-6, mass drawn towards the middle).
    lo, hi, w, n = 0.2, 0.8, 0.3, 6000
    rng = np.random.default_rng(5)
    x = rng.uniform(lo, hi, size=n)
    loglike = lambda p: 0.0 if lo < p[0] < hi else -1.0
    for _ in range(10):
        for i in range(n):
            uni = rng.uniform(size=S.N_UNIFORM_FIXED + 100)
            xi, _, _, st, _ = S.slice_chain(np.array([x[i]]), 0.0, -0.5, (0,), np.eye(1), uni, loglike, w=w,
                                            max_out=1)
            assert st == 0
            x[i] = xi[0]
    h, _ = np.histogram(x, bins=12, range=(lo, hi))
    assert stats.chisquare(h).pvalue > 1e-3


def test_stepping_out_budget_split():
    # J = floor(m V) steps below and m - 1 - J above, m = 2 max_out + 1: a
    # region wider than the whole budget shows the split in the bracket the
    # evaluations trace out.
    seen = []
    for v, j_lo in ((0.0, 0), (0.2, 1), (0.999, 4)):
        uni = np.zeros(S.N_UNIFORM_FIXED + 1)
        uni[:4] = [0.5, 0.0, 0.5, 0.25]  # direction +1 along the single coordinate
        uni[S.N_UNIFORM_FIXED - 2] = 0.5  # bracket offset
        uni[S.N_UNIFORM_FIXED - 1] = v
        uni[S.N_UNIFORM_FIXED] = 0.5  # the shrink draw lands on the start
        pts = []

        def loglike(p):
            pts.append(float(p[0]))
            return 0.0

        S.slice_chain(np.array([0.5]), 0.0, -1.0, (0,), np.eye(1), uni, loglike, w=0.01, max_out=2)
        below = sum(1 for t in pts[:-1] if t < 0.5)
        above = sum(1 for t in pts[:-1] if t > 0.5)
        seen.append((below, above))
        assert below == j_lo and above == 4 - j_lo, (v, pts)
    assert len(set(seen)) == 3


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


def test_prescreen_rule_special_cases():
    # The screen only decides which candidates get an exact log L.  With the
    # exact log L as the prediction and no margin it drops only candidates
    # outside the constraint, so the chain is unchanged; a screen that
    # predicts every candidate outside but audits all of them is unchanged
    # too; one that audits none evaluates nothing and the chain keeps its
    # point at the shrink cap.
    c = np.full(3, 0.5)
    loglike = lambda p: -float(np.sum((p - c) ** 2))
    lstar = -0.04
    chol = 0.2 * np.eye(3)
    rng = np.random.default_rng(4)
    for trial in range(40):
        x0 = c + 0.1 * rng.uniform(-1, 1, size=3)
        uni = rng.uniform(size=S.N_UNIFORM_FIXED + 50)
        ref = S.slice_chain(x0, loglike(x0), lstar, (0, 1, 2), chol, uni, loglike, w=0.3, max_out=2, max_shrink=50)
        st = {}
        exact = S.slice_chain(x0, loglike(x0), lstar, (0, 1, 2), chol, uni, loglike, w=0.3, max_out=2,
                              max_shrink=50, screen=lambda x, kind, i: (loglike(x), 1.0), screen_margin=0.0,
                              audit_frac=0.0, stats=st)
        assert np.array_equal(exact[0], ref[0]) and exact[1] == ref[1] and exact[3] == ref[3]
        assert exact[2] + st.get("screened", 0) == ref[2]  # the screened candidates were the rejected ones
        st = {}
        aud = S.slice_chain(x0, loglike(x0), lstar, (0, 1, 2), chol, uni, loglike, w=0.3, max_out=2,
                            max_shrink=50, screen=lambda x, kind, i: (-math.inf, 0.5), audit_frac=0.75, stats=st)
        assert np.array_equal(aud[0], ref[0]) and aud[1:4] == ref[1:4]
        assert st["audited"] == ref[2] and st["audited_inside"] >= (1 if ref[3] == 0 else 0)
        none = S.slice_chain(x0, loglike(x0), lstar, (0, 1, 2), chol, uni, loglike, w=0.3, max_out=2,
                             max_shrink=50, screen=lambda x, kind, i: (-math.inf, 0.5), audit_frac=0.25)
        assert np.array_equal(none[0], x0) and none[2] == 0 and none[3] == 1


def test_prescreen_audit_indices():
    # The screen sees each test's kind (0 lower end, 1 upper end, 2 shrink
    # draw) and its index within the block, in the order of the tests.
    seen = []

    def screen(x, kind, i):
        seen.append((kind, i))
        return 0.0, 1.0

    uni = np.full(S.N_UNIFORM_FIXED + 5, 0.5)
    uni[S.N_UNIFORM_FIXED - 1] = 0.3  # budget split: J = floor(5 * 0.3) = 1 below, 3 above
    S.slice_chain(np.array([0.5]), 0.0, -1.0, (0,), np.eye(1), uni, lambda p: 0.0, w=0.01, max_out=2,
                  max_shrink=5, screen=screen, screen_margin=10.0)
    assert seen == [(0, 0), (1, 0), (1, 1), (1, 2), (2, 0)]
