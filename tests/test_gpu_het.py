"""GPU parity of the heterodyned likelihood and of the uneven work-list /
hipGraph path against the FP64 heterodyne oracle.

Tolerances as for the full band: 1e-6 absolute for the FP64 form, 1e-3 for the
mixed form.  Edge indices are integer work and must match exactly.
"""
import numpy as np
import pytest

import gwsynth
from oracle import heterodyne as H
from oracle import likelihood as L
from tests.gpu_common import oracle_het_many, problem

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = {0: 1e-6, 1: 1e-3}
MARGS = (L.PLAIN, L.PHASE, L.PHASE_DIST)


@pytest.fixture(scope="module")
def gw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_2607_28265_amd as gw
    return gw


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("name,nb,rule", [("cfg1", 64, 0), ("cfg1", 300, 1), ("cfg2", 500, 0), ("cfg2", 5000, 0),
                                          ("cfg2", 500, 1)])
def test_edges_match_oracle(gw, name, nb, rule):
    prob = problem(name)
    with gw.Context(prob) as ctx:
        fe = ctx.heterodyne_setup(prob.theta_inj, nb, rule)
    want = prob.freqs[H.bin_edges(prob.freqs, nb, rule)]
    assert np.array_equal(fe, want)


@pytest.fixture(scope="module")
def cfg1_het(gw):
    prob = problem("cfg1", loud=True)
    het = H.setup(prob, prob.theta_inj, 200)
    ctx = gw.Context(prob)
    ctx.heterodyne_setup(prob.theta_inj, 200)
    th = np.concatenate([gwsynth.near_posterior(31, prob.theta_inj, 512, scale=0.7),
                         gwsynth.prior_draws(32, 512)])
    ref = {m: H.loglike_many(th, prob, het, m) for m in MARGS}
    yield prob, het, ctx, th, ref
    ctx.close()


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("marg", MARGS)
def test_cfg1_het_parity(cfg1_het, marg, prec):
    prob, het, ctx, th, ref = cfg1_het
    got = ctx.loglike(_t(th), like=1, marg=marg, prec=prec).cpu().numpy()
    err = np.abs(got - ref[marg])
    w = int(np.argmax(err))
    print(f"het cfg1 marg={marg} prec={prec}: max|dlogL|={err.max():.3e} p99={np.quantile(err, 0.99):.3e} "
          f"worst row {w} ({'near' if w < 512 else 'prior'}) logL={ref[marg][w]:.3f}", flush=True)
    assert np.all(np.isfinite(got))
    assert err.max() < TOL[prec]


def test_het_reference_point_equals_full_band(cfg1_het):
    # r = 1 at theta0: the binned sums regroup the full-band sums.
    prob, het, ctx, th, ref = cfg1_het
    t0 = _t(prob.theta_inj[None, :])
    for marg in MARGS:
        a = ctx.loglike(t0, like=1, marg=marg).cpu().numpy()[0]
        b = ctx.loglike(t0, like=0, marg=marg).cpu().numpy()[0]
        assert abs(a - b) < 1e-6, (marg, a, b)


def test_het_before_setup_is_estate(gw):
    prob = problem("cfg1")
    with gw.Context(prob) as ctx:
        with pytest.raises(gw.GwError) as e:
            ctx.loglike(_t(prob.theta_inj[None, :]), like=1)
        assert e.value.status == gw._lib.GW_ESTATE


def test_uneven_edge_cases(cfg1_het, gw):
    prob, het, ctx, th, ref = cfg1_het
    t = _t(th)
    # gaps, an empty sub-batch, a count past the end, a negative offset
    subs = _t(np.array([[0, 10], [20, 0], [30, 70], [1000, 100], [-5, 3], [500, 1]], dtype=np.int64))
    for use_graph in (False, True):
        out = ctx.loglike_uneven(t, subs, marg=L.PHASE, use_graph=use_graph).cpu().numpy()
        covered = np.zeros(len(th), bool)
        covered[0:10] = covered[30:100] = covered[1000:1024] = covered[500] = True
        assert np.all(np.isnan(out[~covered]))
        assert np.max(np.abs(out[covered] - ref[L.PHASE][covered])) < TOL[0]
    empty = _t(np.zeros((0, 2), dtype=np.int64))
    out = ctx.loglike_uneven(t, empty, marg=L.PHASE)
    assert torch.all(torch.isnan(out))


@pytest.mark.parametrize("wpb,grid,ech", [(1, 0, 0), (2, 37, 3), (4, 1, 1), (4, 1024, 0), (4, 4096, 16),
                                          (2, 0, 200)])
def test_het_shapes_agree(cfg1_het, wpb, grid, ech):
    # ech 200 exceeds the 200-bin grid's useful range only at the margin: it
    # is clamped to the bin count (one bin per chunk)
    prob, het, ctx, th, ref = cfg1_het
    ctx.set_het_shape(wpb, grid, ech)
    try:
        for prec in (0, 1):
            got = ctx.loglike(_t(th), like=1, marg=L.PHASE_DIST, prec=prec).cpu().numpy()
            assert np.max(np.abs(got - ref[L.PHASE_DIST])) < TOL[prec]
    finally:
        ctx.set_het_shape(4, 0, 0)


def _cfg3_inputs(n=65536):
    # 65,536 proposals: half prior draws, half near the posterior, split into
    # uneven sub-batches of 100-8000; 4096 of them (2048 from each half) are
    # compared with the oracle
    prob = problem("cfg2", loud=True)
    th = np.concatenate([gwsynth.prior_draws(gwsynth.SEEDS["prior"], n // 2),
                         gwsynth.near_posterior(41, prob.theta_inj, n // 2, scale=0.5)])
    off = gwsynth.uneven_split(gwsynth.SEEDS["split"], n)
    subs = np.stack([off[:-1], np.diff(off)], axis=1).astype(np.int64)
    rng = np.random.default_rng(42)
    idx = np.sort(np.concatenate([rng.choice(n // 2, 2048, replace=False),
                                  n // 2 + rng.choice(n // 2, 2048, replace=False)]))
    return prob, th, subs, idx


@pytest.fixture(scope="module", params=[500, 5000])
def cfg3(gw, request):
    # 128 s full-band segment at PSD scale 1e-49 (SNR 24 injection), bins of
    # equal maximum phase change: 500 (the workload) and 5000 (the paper's
    # Sec. III.D count)
    nb = request.param
    prob, th, subs, idx = _cfg3_inputs()
    het = H.setup(prob, prob.theta_inj, nb)
    ctx = gw.Context(prob)
    ctx.heterodyne_setup(prob.theta_inj, nb)
    yield prob, het, ctx, th, subs, idx
    ctx.close()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("marg", MARGS)
def test_cfg3_uneven_graph(cfg3, marg):
    prob, het, ctx, th, subs, idx = cfg3
    ref = oracle_het_many(th[idx], prob, het, marg)
    t = _t(th)
    s = _t(subs)
    nb = len(het.edges) - 1
    for prec in (0, 1):
        got = ctx.loglike_uneven(t, s, marg=marg, prec=prec, use_graph=True).cpu().numpy()
        assert np.all(np.isfinite(got))
        err = np.abs(got[idx] - ref)
        print(f"het cfg3 {nb} bins marg={marg} prec={prec}: {len(idx)} rows max|dlogL|={err.max():.3e} "
              f"p99={np.quantile(err, 0.99):.3e} (n_sub={len(subs)})", flush=True)
        assert err.max() < TOL[prec]
        eager = ctx.loglike(t, like=1, marg=marg, prec=prec).cpu().numpy()
        assert np.array_equal(got, eager)


def test_cfg3_graph_replays(cfg3, gw):
    # One instantiated graph replayed for different layouts, with eager work
    # and synchronisations in between; every replay matches the eager result.
    prob, het, ctx, th, subs, idx = cfg3
    t = _t(th)
    eager = ctx.loglike(t, like=1, marg=L.PHASE, prec=1).cpu().numpy()
    n = len(th)
    for seed in range(4):
        off = gwsynth.uneven_split(100 + seed, n)
        s = np.stack([off[:-1], np.diff(off)], axis=1).astype(np.int64)
        out = ctx.loglike_uneven(t, _t(s), marg=L.PHASE, prec=1, use_graph=True)
        torch.cuda.synchronize()
        ctx.loglike(t[:100], like=0, marg=L.PHASE)  # eager work in between
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), eager)
    n_graphs, inst_ms = gw.gw_graph_info(ctx.handle)
    print(f"graphs={n_graphs} instantiate={inst_ms:.3f} ms", flush=True)
    assert n_graphs >= 1


def test_autotune_keeps_results(cfg1_het, gw, tmp_path, monkeypatch):
    prob, het, ctx, th, ref = cfg1_het
    monkeypatch.setenv("GW_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    from paper_2607_28265_amd import autotune
    t = _t(th)
    try:
        for like in (1, 0):
            shape, ms = autotune.tune(ctx, t, like, L.PHASE, 1, reps=1)
            assert ms is not None and ms > 0
            shape2, ms2 = autotune.tune(ctx, t, like, L.PHASE, 1)
            assert tuple(shape2) == tuple(shape) and ms2 is None
            got = ctx.loglike(t, like=like, marg=L.PHASE, prec=1).cpu().numpy()
            want = ref[L.PHASE] if like == 1 else np.array([L.loglike(x, prob, L.PHASE) for x in th[:64]])
            assert np.max(np.abs(got[:len(want)] - want)) < TOL[1]
    finally:
        ctx.set_het_shape(4, 0, 0)
        ctx.set_full_shape(0, 0)
