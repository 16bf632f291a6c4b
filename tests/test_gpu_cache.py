"""Fast/slow waveform cache of slice_sweep (full band) against the oracle.

With use_cache a sweep evaluates projection-only blocks (iota, psi) from the
chain's cached sums z_i, extrinsic blocks (sky position, t_c) from its cached
intrinsic waveform (block moments, FP32), and every other block in full; the
waveform is rebuilt when a chain enters an extrinsic block after a slow move.  The oracle has no cache: its slice chain
evaluates the exact full-band likelihood at every candidate, with the same
Philox numbers (block b of the sweep uses counter + b).  Moves must agree
exactly (likelihood calls, capped blocks), the point to 1e-12 and log L to
1e-5 (the moments are rounded to FP32, about 3e-8 relative).  A
chain that came within 1e-5 of log L* anywhere in the oracle run is a near tie
and is only checked for validity.
"""
import numpy as np
import pytest

from oracle import likelihood as L
from oracle import sampler as S
from tests.gpu_common import problem

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TIE = 1e-5


def to_unit(th):
    lo = np.array([1.1, 0.5, -0.05, -0.05, 0.0, 0.0])
    hi = np.array([1.4, 1.0, 0.05, 0.05, 5000.0, 5000.0])
    u = np.empty(11)
    u[:6] = (th[:6] - lo) / (hi - lo)
    u[6] = (1 - np.cos(th[7])) / 2
    u[7] = th[8] / (2 * np.pi)
    u[8] = (np.sin(th[9]) + 1) / 2
    u[9] = th[10] / np.pi
    u[10] = (th[12] + 0.1) / 0.2
    return u


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_2607_28265_amd as gw
    prob = problem("cfg1", loud=True)
    ctx = gw.Context(prob)
    dd = L.data_inner(prob)

    def loglike_u(u):
        return L.loglike(S.prior_transform(u), prob, L.PHASE_DIST, dd)

    k = 40
    u0 = to_unit(prob.theta_inj)
    rng = np.random.default_rng(11)
    x = np.clip(u0 + 0.01 * rng.standard_normal((k, 11)), 0.001, 0.999)
    logl = np.array([loglike_u(p) for p in x])
    yield gw, ctx, prob, loglike_u, x, logl
    ctx.close()


def gpu_sweep(gw, ctx, x, logl, lstar, blocks, chols, seed, counter, use_cache, prec=0, like=None, max_out=4,
              max_shrink=60):
    k = len(x)
    xt = torch.from_numpy(x.copy()).cuda()
    lt = torch.from_numpy(logl.copy()).cuda()
    ne = torch.zeros(k, dtype=torch.int32, device="cuda")
    st = torch.zeros(k, dtype=torch.int32, device="cuda")
    kinds = gw.slice_sweep(ctx.handle, xt, lt, lstar, blocks, chols, seed=seed, counter=counter, w=1.0,
                           max_out=max_out, max_shrink=max_shrink, like=gw.GW_FULL if like is None else like,
                           marg=gw.GW_MARG_PHASE_DIST, prec=prec, n_evals=ne, status=st, use_cache=use_cache)
    torch.cuda.synchronize()
    return xt.cpu().numpy(), lt.cpu().numpy(), ne.cpu().numpy(), st.cpu().numpy(), kinds


def oracle_sweep(x0, l0, lstar, blocks, chols, seed, counter, c, loglike_u, max_out=4, max_shrink=60):
    x, l = x0.copy(), l0
    ne = st = 0
    margin = np.inf
    for b, (blk, ch) in enumerate(zip(blocks, chols)):
        uni = S.philox_uniforms(seed, counter + b, c, S.N_UNIFORM_FIXED + max_shrink)
        x, l, n1, s1, m1 = S.slice_chain(x, l, lstar, blk, ch, uni, loglike_u, 1.0, max_out, max_shrink)
        ne += n1
        st += s1
        margin = min(margin, m1)
    return x, l, ne, st, margin


CASES = {
    "psi": [S.BLOCKS[5]],
    "iota": [S.BLOCKS[3]],
    "sky": [S.BLOCKS[4]],
    "tc": [S.BLOCKS[6]],
    "all": list(S.BLOCKS),
}


@pytest.mark.parametrize("case", list(CASES))
def test_cached_sweep_matches_oracle(setup, case):
    gw, ctx, prob, loglike_u, x, logl = setup
    blocks = CASES[case]
    chols = [S.block_cholesky(x, b) for b in blocks]
    lstar = float(np.quantile(logl, 0.25))
    keep = logl > lstar
    xs, ls = x[keep], logl[keep]
    seed, counter = 41, 9000
    gx, gl, gne, gst, kinds = gpu_sweep(gw, ctx, xs, ls, lstar, blocks, chols, seed, counter, True)
    k = len(xs)
    # every evaluation is counted once by kind; the k seeding evaluations are full ones
    assert kinds[0] + kinds[1] + kinds[2] == int(gne.sum()) + k
    if case in ("psi", "iota"):
        assert kinds[0] == k and kinds[1] == 0 and kinds[2] > 0
    elif case in ("sky", "tc"):
        # the waveform is built after each chain's first round in the block,
        # whose (at most two) candidates evaluate in full
        assert k < kinds[0] <= 3 * k and kinds[2] == 0 and kinds[1] > 0
    else:
        assert min(kinds) > 0
    n_cmp = 0
    for c in range(k):
        ox, ol, one, ost, margin = oracle_sweep(xs[c], ls[c], lstar, blocks, chols, seed, counter, c, loglike_u)
        assert gl[c] > lstar or gst[c] > 0
        if margin < TIE:
            continue
        n_cmp += 1
        assert gne[c] == one and gst[c] == ost, (c, gne[c], one, gst[c], ost)
        assert np.max(np.abs(gx[c] - ox)) < 1e-12
        assert abs(gl[c] - ol) < 1e-5, (c, gl[c], ol)
    print(f"{case}: {n_cmp}/{k} chains compared; evaluations full/cached waveform/cached sums = {kinds}")
    assert n_cmp >= k - 3


def test_cache_off_equals_plain_sweep(setup):
    # use_cache = 0 takes the plain full-band path: same moves as block-by-block steps
    gw, ctx, prob, loglike_u, x, logl = setup
    blocks = list(S.BLOCKS)
    chols = [S.block_cholesky(x, b) for b in blocks]
    lstar = float(np.quantile(logl, 0.3))
    keep = logl > lstar
    a = gpu_sweep(gw, ctx, x[keep], logl[keep], lstar, blocks, chols, 5, 123, False)
    xb = torch.from_numpy(x[keep].copy()).cuda()
    lb = torch.from_numpy(logl[keep].copy()).cuda()
    for b, (blk, ch) in enumerate(zip(blocks, chols)):
        gw.slice_step(ctx.handle, xb, lb, lstar, blk, ch, seed=5, counter=123 + b, w=1.0, max_out=4, max_shrink=60,
                      like=gw.GW_FULL, marg=gw.GW_MARG_PHASE_DIST, prec=0)
    torch.cuda.synchronize()
    assert a[4] is None
    assert np.array_equal(a[0], xb.cpu().numpy()) and np.array_equal(a[1], lb.cpu().numpy())


def test_cache_graph_replay_equals_eager(setup):
    gw, ctx, prob, loglike_u, x, logl = setup
    blocks = list(S.BLOCKS)
    chols = [S.block_cholesky(x, b) for b in blocks]
    lstar = float(np.quantile(logl, 0.2))
    keep = logl > lstar
    outs = []
    for g in (False, True, True):
        k = int(keep.sum())
        xt = torch.from_numpy(x[keep].copy()).cuda()
        lt = torch.from_numpy(logl[keep].copy()).cuda()
        ne = torch.zeros(k, dtype=torch.int32, device="cuda")
        kinds = gw.slice_sweep(ctx.handle, xt, lt, lstar, blocks, chols, seed=8, counter=70, w=1.0, max_out=4,
                               max_shrink=60, like=gw.GW_FULL, marg=gw.GW_MARG_PHASE_DIST, prec=1, n_evals=ne,
                               use_graph=g, use_cache=True)
        torch.cuda.synchronize()
        outs.append((xt.cpu().numpy(), lt.cpu().numpy(), ne.cpu().numpy(), kinds))
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1])
        assert np.array_equal(o[2], outs[0][2]) and o[3] == outs[0][3]


def test_cache_argument_errors(setup):
    gw, ctx, prob, loglike_u, x, logl = setup
    xt = torch.from_numpy(x.copy()).cuda()
    lt = torch.from_numpy(logl.copy()).cuda()
    with pytest.raises(gw.GwError):  # the cache is for the full band only
        gw.slice_sweep(ctx.handle, xt, lt, float(logl.min()) - 1, [S.BLOCKS[5]], [np.eye(1)], like=gw.GW_HET,
                       use_cache=True)


def test_cached_sweep_large_grid_against_plain():
    # 128 s, 259,585 bins per detector: the cached and plain sweeps make the
    # same moves except near ties, and the final log L agree to the mixed
    # form's tolerance; a few chains' final log L against the oracle
    import paper_2607_28265_amd as gw
    prob = problem("cfg2", loud=True)
    with gw.Context(prob) as ctx:
        u0 = to_unit(prob.theta_inj)
        rng = np.random.default_rng(3)
        k = 96
        x = np.clip(u0 + 0.003 * rng.standard_normal((k, 11)), 0.001, 0.999)
        xt = torch.from_numpy(x).cuda()
        th = gw.gw_prior_transform(ctx.handle, xt)
        lt = ctx.loglike(th, gw.GW_FULL, gw.GW_MARG_PHASE_DIST, gw.GW_PREC_FP64)
        torch.cuda.synchronize()
        logl = lt.cpu().numpy()
        lstar = float(np.quantile(logl, 0.25))
        keep = logl > lstar
        xs, ls = x[keep], logl[keep]
        blocks = list(S.BLOCKS)
        chols = [S.block_cholesky(xs, b) for b in blocks]
        a = gpu_sweep(gw, ctx, xs, ls, lstar, blocks, chols, 77, 400, True, prec=1)
        b = gpu_sweep(gw, ctx, xs, ls, lstar, blocks, chols, 77, 400, False, prec=1)
        same = (a[2] == b[2]) & (a[3] == b[3]) & np.all(a[0] == b[0], axis=1)
        print(f"cfg2: {int(same.sum())}/{len(xs)} chains with identical moves; kinds {a[4]}")
        assert same.mean() >= 0.9
        assert np.max(np.abs(a[1][same] - b[1][same])) < 1e-3
        assert np.all(a[1] > lstar) and np.all(b[1] > lstar)
        dd = L.data_inner(prob)
        for c in np.flatnonzero(same)[:4]:
            ol = L.loglike(S.prior_transform(a[0][c]), prob, L.PHASE_DIST, dd)
            assert abs(a[1][c] - ol) < 1e-3, (c, a[1][c], ol)


# -- the cache as a library object (gw_wcache_*) -----------------------------

def _base_thetas(prob, n, seed):
    rng = np.random.default_rng(seed)
    th = np.tile(prob.theta_inj, (n, 1))
    th[:, 0] *= 1 + 2e-4 * rng.standard_normal(n)
    th[:, 1] = np.clip(th[:, 1] + 0.02 * rng.standard_normal(n), 0.5, 1.0)
    th[:, 2:4] = np.clip(th[:, 2:4] + 0.01 * rng.standard_normal((n, 2)), -0.05, 0.05)
    th[:, 4:6] = np.clip(th[:, 4:6] + 100 * rng.standard_normal((n, 2)), 0, 5000)
    th[:, 11] = 0.0
    return th


def _moved(base, kind, rng):
    th = base.copy()
    m = len(th)
    th[:, 6] *= np.exp(0.2 * rng.standard_normal(m))           # d_L
    th[:, 7] = np.clip(th[:, 7] + 0.1 * rng.standard_normal(m), 0.01, np.pi - 0.01)  # iota
    th[:, 10] = np.mod(th[:, 10] + 0.2 * rng.standard_normal(m), np.pi)           # psi
    if kind == 1:
        th[:, 8] = np.mod(th[:, 8] + 0.05 * rng.standard_normal(m), 2 * np.pi)     # ra
        th[:, 9] = np.clip(th[:, 9] + 0.05 * rng.standard_normal(m), -1.5, 1.5)   # dec
        th[:, 12] += 2e-4 * rng.standard_normal(m)                                 # t_c
    return th


@pytest.mark.parametrize("name,marg", [("cfg1", 2), ("cfg1", 1), ("cfg1", 0), ("cfg2", 2)])
def test_wcache_slow_and_fast_match_oracle(name, marg):
    import paper_2607_28265_amd as gw
    from tests.gpu_common import oracle_many
    prob = problem(name, loud=True)
    n_slots, per = (24, 4) if name == "cfg1" else (6, 3)
    base = _base_thetas(prob, n_slots, 21)
    rng = np.random.default_rng(22)
    with gw.Context(prob) as ctx:
        cache = gw.WaveformCache(ctx.handle, n_slots)
        slots = torch.arange(n_slots, dtype=torch.int32, device="cuda")
        l_slow = cache.update(torch.from_numpy(base).cuda(), slots, marg=marg).cpu().numpy()
        o_slow = oracle_many(base, prob, marg)
        assert np.max(np.abs(l_slow - o_slow)) < 1e-6
        for kind in (1, 2):
            rows = np.repeat(np.arange(n_slots), per)
            th = _moved(base[rows], kind, rng)
            got = cache.loglike(torch.from_numpy(th).cuda(), torch.from_numpy(rows.astype(np.int32)).cuda(), kind,
                                marg=marg).cpu().numpy()
            ref = oracle_many(th, prob, marg)
            err = np.max(np.abs(got - ref))
            print(f"{name} marg {marg} kind {kind}: {len(th)} rows, max |dlogL| {err:.2e}, "
                  f"logL range {ref.min():.1f} .. {ref.max():.1f}")
            # FP32 waveform: ~3e-8 relative per bin, unbiased; FP64 otherwise
            assert err < (1e-5 if kind == 1 else 1e-6)
        cache.close()


def test_wcache_slot_rules():
    import paper_2607_28265_amd as gw
    from tests.gpu_common import oracle_many
    prob = problem("cfg1", loud=True)
    base = _base_thetas(prob, 3, 31)
    rng = np.random.default_rng(32)
    with gw.Context(prob) as ctx:
        cache = gw.WaveformCache(ctx.handle, 2)
        # slot 0 named twice: the later row (base[1]) wins; slot 5 is out of range
        l = cache.update(torch.from_numpy(base).cuda(), torch.tensor([0, 0, 5], dtype=torch.int32, device="cuda"))
        l = l.cpu().numpy()
        assert np.all(np.isfinite(l[:2])) and np.isnan(l[2])
        th = _moved(base[[1, 1]], 2, rng)
        got = cache.loglike(torch.from_numpy(th).cuda(), torch.tensor([0, -1], dtype=torch.int32, device="cuda"), 2)
        got = got.cpu().numpy()
        ref = oracle_many(th, prob, 2)
        assert abs(got[0] - ref[0]) < 1e-6 and np.isnan(got[1])
        got1 = cache.loglike(torch.from_numpy(th).cuda(), torch.tensor([0, 2], dtype=torch.int32, device="cuda"), 1)
        got1 = got1.cpu().numpy()
        assert abs(got1[0] - ref[0]) < 1e-5 and np.isnan(got1[1])
        with pytest.raises(gw.GwError):
            cache.loglike(torch.from_numpy(th).cuda(), torch.tensor([0, 0], dtype=torch.int32, device="cuda"), 3)
        cache.close()


def test_wcache_large_update_matches_oracle():
    # an update of 600 slots builds them with one lane per slot (the kernel
    # for large lists), 24 slots with the kernel whose work follows the
    # count; moved rows on either agree with the oracle to the FP32 tolerance
    import paper_2607_28265_amd as gw
    from tests.gpu_common import oracle_many
    prob = problem("cfg1", loud=True)
    n_big, n_small = 600, 24
    base = _base_thetas(prob, n_big, 41)
    rng = np.random.default_rng(42)
    pick = np.arange(0, n_big, n_big // n_small)[:n_small]
    th = _moved(base[pick], 1, rng)
    ref = oracle_many(th, prob, 2)
    with gw.Context(prob) as ctx:
        for n_slots, rows in ((n_big, pick), (n_small, np.arange(n_small))):
            cache = gw.WaveformCache(ctx.handle, n_slots)
            src = base if n_slots == n_big else base[pick]
            cache.update(torch.from_numpy(src).cuda(), torch.arange(n_slots, dtype=torch.int32, device="cuda"))
            got = cache.loglike(torch.from_numpy(th).cuda(), torch.from_numpy(rows.astype(np.int32)).cuda(), 1)
            err = np.max(np.abs(got.cpu().numpy() - ref))
            print(f"{n_slots} slots: kind 1 on {len(rows)} rows, max |dlogL| vs oracle {err:.2e}")
            assert err < 1e-5
            cache.close()
