"""GPU phase+time marginal (GW_MARG_PHASE_TIME, full band and heterodyned)
against the oracle's grid sums over time shifts, on the same seeded problems.

The oracle sums I0(|Z(t_j)|) over the grid by direct summation of every
shifted overlap; the library evaluates the same grid with block moments and
FFTs.  FP64 must agree to 1e-6 in log L; the mixed form (FP32 hardware
sin/cos in the phasors) to 1e-4 at SNR 24.
"""
import numpy as np
import pytest

import gwsynth
from oracle import likelihood as L
from tests.gpu_common import oracle_het_many, oracle_many, problem

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def near(prob, n, seed, scale):
    rng = np.random.default_rng(seed)
    th = np.tile(prob.theta_inj, (n, 1))
    th[:, 0] *= 1 + scale * 1e-4 * rng.standard_normal(n)
    th[:, 1] = np.clip(th[:, 1] + scale * 0.01 * rng.standard_normal(n), 0.5, 1.0)
    th[:, 6] *= np.exp(scale * 0.1 * rng.standard_normal(n))
    th[:, 7:11] += scale * 0.02 * rng.standard_normal((n, 4))
    th[:, 12] = rng.uniform(-0.2, 0.2, n)  # ignored by the time marginal
    return th


def run(gw, ctx, th, prec):
    out = ctx.loglike(torch.from_numpy(th).cuda(), gw.GW_FULL, gw.GW_MARG_PHASE_TIME, prec)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("loud", [False, True])
def test_cfg1_against_oracle(loud):
    import paper_2607_28265_amd as gw
    prob = problem("cfg1", loud=loud)
    th = np.concatenate([gwsynth.prior_draws(gwsynth.SEEDS["prior"], 96), near(prob, 32, 3, 1.0)])
    ref = oracle_many(th, prob, L.PHASE_TIME)
    with gw.Context(prob) as ctx:
        delta, n_t, p_len, blk = gw.gw_time_grid_info(ctx.handle)
        t = L.time_grid(prob)
        assert n_t == t.size and delta == pytest.approx(t[1] - t[0], rel=1e-15)
        for prec, tol in ((gw.GW_PREC_FP64, 1e-6), (gw.GW_PREC_MIXED, 1e-4)):
            got = run(gw, ctx, th, prec)
            err = np.max(np.abs(got - ref))
            print(f"cfg1 loud={loud} prec {prec}: grid {n_t} points, FFT {p_len}, {blk}-bin blocks; "
                  f"max |dlogL| {err:.2e}")
            assert err < tol


def test_cfg2_sampled_against_oracle():
    import paper_2607_28265_amd as gw
    prob = problem("cfg2", loud=True)
    th = np.concatenate([near(prob, 3, 5, 0.3), gwsynth.prior_draws(gwsynth.SEEDS["prior"], 2)])
    ref = oracle_many(th, prob, L.PHASE_TIME)
    with gw.Context(prob) as ctx:
        for prec, tol in ((gw.GW_PREC_FP64, 1e-6), (gw.GW_PREC_MIXED, 1e-4)):
            got = run(gw, ctx, th, prec)
            err = np.max(np.abs(got - ref))
            print(f"cfg2 prec {prec}: max |dlogL| {err:.2e}, logL {ref.min():.1f} .. {ref.max():.1f}")
            assert err < tol


def test_one_point_window_is_phase_marginal():
    import paper_2607_28265_amd as gw
    prob = problem("cfg1", loud=True)
    th = near(prob, 16, 9, 1.0)
    with gw.Context(prob) as ctx:
        gw.gw_set_time_window(ctx.handle, 0.0)
        assert gw.gw_time_grid_info(ctx.handle)[1] == 1
        got = run(gw, ctx, th, gw.GW_PREC_FP64)
        th0 = th.copy()
        th0[:, 12] = 0.0
        ref = ctx.loglike(torch.from_numpy(th0).cuda(), gw.GW_FULL, gw.GW_MARG_PHASE, gw.GW_PREC_FP64)
        torch.cuda.synchronize()
        assert np.max(np.abs(got - ref.cpu().numpy())) < 1e-8
        with pytest.raises(gw.GwError):
            gw.gw_set_time_window(ctx.handle, 10.0)  # more than 2048 grid points
        with pytest.raises(gw.GwError):
            gw.gw_set_time_window(ctx.handle, -1.0)


def test_unphysical_rows():
    import paper_2607_28265_amd as gw
    prob = problem("cfg1")
    th = gwsynth.prior_draws(gwsynth.SEEDS["prior"], 4)
    th[1, 1] = 1.5  # q > 1
    th[2, 6] = -1.0  # d_L <= 0 (d_L is used by this mode)
    with gw.Context(prob) as ctx:
        got = run(gw, ctx, th, gw.GW_PREC_FP64)
        assert np.isneginf(got[1]) and np.isneginf(got[2]) and np.all(np.isfinite(got[[0, 3]]))
        ctx.heterodyne_setup(prob.theta_inj, 100)
        got = ctx.loglike(torch.from_numpy(th).cuda(), gw.GW_HET, gw.GW_MARG_PHASE_TIME, gw.GW_PREC_FP64)
        got = got.cpu().numpy()
        assert np.isneginf(got[1]) and np.isneginf(got[2]) and np.all(np.isfinite(got[[0, 3]]))


@pytest.mark.parametrize("loud", [False, True])
def test_heterodyned_against_oracle(loud):
    # the binned phase-marginal likelihood at every grid shift, log-mean-exp:
    # the oracle evaluates its own binned likelihood at each t_c = t_j
    import paper_2607_28265_amd as gw
    from oracle import heterodyne as H
    prob = problem("cfg1", loud=loud)
    het = H.setup(prob, prob.theta_inj, 200)
    th = np.concatenate([gwsynth.prior_draws(gwsynth.SEEDS["prior"], 8), near(prob, 16, 13, 1.0)])
    dd = L.data_inner(prob)
    ref = np.array([H.loglike(t, prob, het, L.PHASE_TIME, dd) for t in th])
    with gw.Context(prob) as ctx:
        ctx.heterodyne_setup(prob.theta_inj, 200)
        for prec, tol in ((gw.GW_PREC_FP64, 1e-7), (gw.GW_PREC_MIXED, 1e-4)):
            got = ctx.loglike(torch.from_numpy(th).cuda(), gw.GW_HET, gw.GW_MARG_PHASE_TIME, prec)
            torch.cuda.synchronize()
            err = np.max(np.abs(got.cpu().numpy() - ref))
            print(f"heterodyned loud={loud} prec {prec}: max |dlogL| {err:.2e}")
            assert err < tol


@pytest.mark.timeout(600)
@pytest.mark.parametrize("nb", [500, 5000])
def test_heterodyned_cfg2_against_oracle(nb):
    # the 128 s segment (SNR 24) with 500 bins (the benchmark's heterodyned
    # workload) and 5000 (the paper's count, Sec. III.D): 16 rows alone (a
    # sampler-round batch, products split over edge chunks) and the same rows
    # at the head of a 65,536-row batch (the benchmark's launch, unsplit)
    import paper_2607_28265_amd as gw
    from oracle import heterodyne as H
    prob = problem("cfg2", loud=True)
    het = H.setup(prob, prob.theta_inj, nb)
    th = np.concatenate([near(prob, 8, 31, 0.3), gwsynth.prior_draws(gwsynth.SEEDS["prior"], 8)])
    ref = oracle_het_many(th, prob, het, L.PHASE_TIME)
    big = np.concatenate([th, gwsynth.prior_draws(37, 65536 - len(th))])
    with gw.Context(prob) as ctx:
        ctx.heterodyne_setup(prob.theta_inj, nb)
        for prec, tol in ((gw.GW_PREC_FP64, 1e-6), (gw.GW_PREC_MIXED, 1e-4)):
            for name, rows in (("16 rows", th), ("65,536 rows", big)):
                got = ctx.loglike(torch.from_numpy(rows).cuda(), gw.GW_HET, gw.GW_MARG_PHASE_TIME, prec)
                got = got[:len(th)].cpu().numpy()
                err = np.max(np.abs(got - ref))
                print(f"heterodyned 128 s, {nb} bins, {name}, prec {prec}: max |dlogL| {err:.2e}, "
                      f"logL {ref.min():.1f} .. {ref.max():.1f}", flush=True)
                assert err < tol


@pytest.mark.timeout(600)
def test_heterodyned_narrow_window_against_oracle(monkeypatch):
    # the event analysis' +-0.03 s window at 5000 bins: a shorter transform
    # and wide frequency blocks, hundreds of edges in the lowest ones, so the
    # edge moments of a sampler-round batch come from chunks that cut blocks
    # into many pieces, added by the fix-up pass
    import paper_2607_28265_amd as gw
    from oracle import heterodyne as H
    prob = problem("cfg2", loud=True)
    monkeypatch.setattr(L, "TIME_WINDOW", 0.03)
    het = H.setup(prob, prob.theta_inj, 5000)
    th = np.concatenate([near(prob, 8, 41, 0.3), gwsynth.prior_draws(gwsynth.SEEDS["prior"], 8)])
    ref = oracle_het_many(th, prob, het, L.PHASE_TIME)
    with gw.Context(prob) as ctx:
        gw.gw_set_time_window(ctx.handle, 0.03)
        _, n_t, _, _ = gw.gw_time_grid_info(ctx.handle)
        assert n_t == L.time_grid(prob).size
        ctx.heterodyne_setup(prob.theta_inj, 5000)
        for prec, tol in ((gw.GW_PREC_FP64, 1e-6), (gw.GW_PREC_MIXED, 1e-4)):
            got = ctx.loglike(torch.from_numpy(th).cuda(), gw.GW_HET, gw.GW_MARG_PHASE_TIME, prec).cpu().numpy()
            err = np.max(np.abs(got - ref))
            print(f"heterodyned 128 s, 5000 bins, window 0.03 s ({n_t} points), prec {prec}: max |dlogL| {err:.2e}",
                  flush=True)
            assert err < tol


def test_heterodyned_split_matches_unsplit():
    # few rows split the edge sum of the products into up to 32 chunks; a
    # large batch keeps one chunk: the same rows agree to rounding
    import paper_2607_28265_amd as gw
    prob = problem("cfg1", loud=True)
    th = np.concatenate([gwsynth.prior_draws(gwsynth.SEEDS["prior"], 8), near(prob, 16, 21, 1.0)])
    big = np.concatenate([th, gwsynth.prior_draws(7, 16384 - len(th))])
    with gw.Context(prob) as ctx:
        ctx.heterodyne_setup(prob.theta_inj, 200)
        for prec, tol in ((gw.GW_PREC_FP64, 1e-9), (gw.GW_PREC_MIXED, 1e-6)):
            small = ctx.loglike(torch.from_numpy(th).cuda(), gw.GW_HET, gw.GW_MARG_PHASE_TIME, prec).cpu().numpy()
            large = ctx.loglike(torch.from_numpy(big).cuda(), gw.GW_HET, gw.GW_MARG_PHASE_TIME, prec).cpu().numpy()
            err = np.max(np.abs(small - large[:len(th)]))
            print(f"prec {prec}: split vs unsplit max |dlogL| {err:.2e}")
            assert err < tol


@pytest.mark.parametrize("factor", [1, 8])
def test_oversampling_factors_against_oracle(factor, monkeypatch):
    # the grid's oversampling (points per sampling interval) on both sides
    import paper_2607_28265_amd as gw
    from oracle import heterodyne as H
    prob = problem("cfg1", loud=True)
    th = np.concatenate([gwsynth.prior_draws(gwsynth.SEEDS["prior"], 8), near(prob, 16, 4, 1.0)])
    monkeypatch.setattr(L, "TIME_OVERSAMPLE", factor)
    ref = oracle_many(th, prob, L.PHASE_TIME)
    het = H.setup(prob, prob.theta_inj, 200)
    dd = L.data_inner(prob)
    ref_het = np.array([H.loglike(t, prob, het, L.PHASE_TIME, dd) for t in th[:6]])
    with gw.Context(prob) as ctx:
        gw.gw_set_time_oversample(ctx.handle, factor)
        delta, n_t, _, _ = gw.gw_time_grid_info(ctx.handle)
        t = L.time_grid(prob)
        assert n_t == t.size and delta == pytest.approx(t[1] - t[0], rel=1e-15)
        err = np.max(np.abs(run(gw, ctx, th, gw.GW_PREC_FP64) - ref))
        ctx.heterodyne_setup(prob.theta_inj, 200)
        got = ctx.loglike(torch.from_numpy(th[:6]).cuda(), gw.GW_HET, gw.GW_MARG_PHASE_TIME, gw.GW_PREC_FP64)
        err_het = np.max(np.abs(got.cpu().numpy() - ref_het))
        print(f"oversampling {factor}: {n_t} points, full band {err:.2e}, heterodyned {err_het:.2e}")
        assert err < 1e-6 and err_het < 1e-6
        with pytest.raises(gw.GwError):
            gw.gw_set_time_oversample(ctx.handle, 3)


def test_odd_power_fft_length(monkeypatch):
    # a 0.05 s window gives 103 points per sub-grid and an FFT of 128 points
    # (radix-4 stages and one radix-2 stage); the default grids use 256 and
    # 1024 (radix-4 only)
    import paper_2607_28265_amd as gw
    prob = problem("cfg1", loud=True)
    th = np.concatenate([gwsynth.prior_draws(gwsynth.SEEDS["prior"], 8), near(prob, 16, 6, 1.0)])
    monkeypatch.setattr(L, "TIME_WINDOW", 0.05)
    ref = oracle_many(th, prob, L.PHASE_TIME)
    with gw.Context(prob) as ctx:
        gw.gw_set_time_window(ctx.handle, 0.05)
        delta, n_t, p_len, blk = gw.gw_time_grid_info(ctx.handle)
        assert p_len == 128 and n_t == L.time_grid(prob).size
        err = np.max(np.abs(run(gw, ctx, th, gw.GW_PREC_FP64) - ref))
        print(f"window 0.05 s: FFT {p_len}, {n_t} points, max |dlogL| {err:.2e}")
        assert err < 1e-6


@pytest.mark.parametrize("nsk", [1, 2, 8, 32, 256])
def test_heterodyned_fixed_splits_agree(nsk):
    # every split of the edge sum gives the same grid sums up to summation
    # order, for a sampler-sized batch (and the default split on the same rows)
    import paper_2607_28265_amd as gw
    prob = problem("cfg1", loud=True)
    th = np.concatenate([gwsynth.prior_draws(gwsynth.SEEDS["prior"], 64), near(prob, 64, 23, 1.0)])
    with gw.Context(prob) as ctx:
        ctx.heterodyne_setup(prob.theta_inj, 200)
        t = torch.from_numpy(th).cuda()
        for prec, tol in ((gw.GW_PREC_FP64, 1e-9), (gw.GW_PREC_MIXED, 1e-6)):
            base = ctx.loglike(t, gw.GW_HET, gw.GW_MARG_PHASE_TIME, prec).cpu().numpy()
            gw.gw_set_het_tm_split(ctx.handle, nsk)
            try:
                got = ctx.loglike(t, gw.GW_HET, gw.GW_MARG_PHASE_TIME, prec).cpu().numpy()
            finally:
                gw.gw_set_het_tm_split(ctx.handle, 0)
            fin = np.isfinite(base)
            assert fin.sum() > 100 and np.array_equal(np.isfinite(got), fin)
            err = np.max(np.abs(got[fin] - base[fin]))
            print(f"split {nsk} prec {prec}: max |dlogL| vs default {err:.2e}", flush=True)
            assert err < tol
        for bad in (3, 512):
            with pytest.raises(gw.GwError):
                gw.gw_set_het_tm_split(ctx.handle, bad)
