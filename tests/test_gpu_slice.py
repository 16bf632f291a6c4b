"""GPU slice_step against the oracle slice step, chain by chain.

Both sides consume the same random numbers (explicit uniforms, or Philox
counters), so the moves must agree exactly: number of likelihood calls and
status bit-exact, the new point to 1e-12 (the two sides round x + t d
differently by an ulp), log L to the FP64 parity tolerance.  A chain whose
oracle run came within 1e-6 of log L* at any comparison is a near tie (the GPU
and oracle likelihoods differ by ~1e-9) and is only checked for validity.
"""
import math

import numpy as np
import pytest

import gwsynth
from oracle import heterodyne as H
from oracle import likelihood as L
from oracle import sampler as S
from tests.gpu_common import problem

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def to_unit(th):
    lo = np.array([1.1, 0.5, -0.05, -0.05, 0.0, 0.0])
    hi = np.array([1.4, 1.0, 0.05, 0.05, 5000.0, 5000.0])
    u = np.empty(11)
    u[:6] = (th[:6] - lo) / (hi - lo)
    u[6] = (1 - math.cos(th[7])) / 2
    u[7] = th[8] / (2 * math.pi)
    u[8] = (math.sin(th[9]) + 1) / 2
    u[9] = th[10] / math.pi
    u[10] = (th[12] + 0.1) / 0.2
    return u


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_2607_28265_amd as gw
    prob = problem("cfg1", loud=True)
    het = H.setup(prob, prob.theta_inj, 200)
    ctx = gw.Context(prob)
    ctx.heterodyne_setup(prob.theta_inj, 200)
    dd = L.data_inner(prob)

    def loglike_u(u):
        return H.loglike(S.prior_transform(u), prob, het, L.PHASE_DIST, dd)

    k = 64
    u0 = to_unit(prob.theta_inj)
    rng = np.random.default_rng(5)
    x = np.clip(u0 + 0.01 * rng.standard_normal((k, 11)), 0.001, 0.999)
    logl = np.array([loglike_u(p) for p in x])
    yield gw, ctx, prob, het, loglike_u, x, logl
    ctx.close()


def _run_gpu(gw, ctx, x, logl, lstar, block, chol, uni=None, seed=0, counter=0, max_shrink=60, max_out=4,
             use_graph=True, prec=0, like=None):
    xt = torch.from_numpy(x.copy()).cuda()
    lt = torch.from_numpy(logl.copy()).cuda()
    ne = torch.zeros(len(x), dtype=torch.int32, device="cuda")
    stt = torch.zeros(len(x), dtype=torch.int32, device="cuda")
    ut = torch.from_numpy(uni).cuda() if uni is not None else None
    gw.slice_step(ctx.handle, xt, lt, lstar, block, chol, seed=seed, counter=counter, uniforms=ut, w=1.0,
                  max_out=max_out, max_shrink=max_shrink, like=gw.GW_HET if like is None else like,
                  marg=gw.GW_MARG_PHASE_DIST, prec=prec, n_evals=ne, status=stt, use_graph=use_graph)
    torch.cuda.synchronize()
    return xt.cpu().numpy(), lt.cpu().numpy(), ne.cpu().numpy(), stt.cpu().numpy()


# the Gibbs blocks, a 6-coordinate block and the unblocked sampler's single
# block of all 11 coordinates (6 Box-Muller pairs)
CASES = list(S.BLOCKS) + [(0, 1, 2, 3, 4, 5), tuple(range(11))]


@pytest.mark.parametrize("bi", range(len(CASES)))
@pytest.mark.parametrize("source", ["uniforms", "philox"])
def test_slice_step_matches_oracle(setup, bi, source):
    gw, ctx, prob, het, loglike_u, x, logl = setup
    block = CASES[bi]
    nfix = S.n_fixed_uniforms(len(block))
    assert nfix == gw.slice_uniforms_fixed(len(block))
    chol = S.block_cholesky(x, block)
    lstar = float(np.quantile(logl, 0.25))
    ok0 = logl > lstar
    x, logl = x[ok0], logl[ok0]
    k = len(x)
    max_shrink, max_out = 60, 4
    seed, counter = 1234 + bi, 77
    if source == "uniforms":
        uni = np.random.default_rng(100 + bi).uniform(size=(k, nfix + max_shrink))
        uni_c = lambda c: uni[c]
    else:
        uni = None
        uni_c = lambda c: S.philox_uniforms(seed, counter, c, nfix + max_shrink)
    gx, gl, gne, gst = _run_gpu(gw, ctx, x, logl, lstar, block, chol, uni, seed, counter, max_shrink, max_out)
    n_cmp = 0
    for c in range(k):
        ox, ol, one, ost, margin = S.slice_chain(x[c], logl[c], lstar, block, chol, uni_c(c), loglike_u, 1.0,
                                                 max_out, max_shrink)
        assert gl[c] > lstar or gst[c] == 1
        if margin < 1e-6:
            continue
        n_cmp += 1
        assert gne[c] == one and gst[c] == ost, (c, gne[c], one, gst[c], ost)
        assert np.max(np.abs(gx[c] - ox)) < 1e-12
        assert abs(gl[c] - ol) < 1e-6
    print(f"block {bi} ({source}): {n_cmp}/{k} chains compared, evals {gne.sum()}", flush=True)
    assert n_cmp >= k - 2


def test_slice_step_argument_errors(setup):
    gw, ctx, prob, het, loglike_u, x, logl = setup
    xt = torch.from_numpy(x.copy()).cuda()
    lt = torch.from_numpy(logl.copy()).cuda()
    with pytest.raises(gw.GwError):
        gw.slice_step(ctx.handle, xt, lt, 0.0, [0, 0], np.eye(2))  # repeated index
    with pytest.raises(gw.GwError):
        gw.slice_step(ctx.handle, xt, lt, 0.0, [11], np.eye(1))  # out of range
    with pytest.raises(gw.GwError):
        gw.slice_step(ctx.handle, xt, lt, 0.0, [0], np.eye(1), marg=gw.GW_MARG_NONE)


@pytest.mark.parametrize("like", [0, 1])
def test_graph_replay_equals_eager(setup, like):
    # the captured round group and the eager launches run the same kernels in
    # the same order: bit-identical moves; consecutive calls with different
    # blocks, constraints and chain counts reuse or re-capture the graph
    gw, ctx, prob, het, loglike_u, x, logl = setup
    for call, bi in enumerate([0, 4, 0, 6, 1]):
        block = S.BLOCKS[bi]
        chol = S.block_cholesky(x, block)
        lstar = float(np.quantile(logl, 0.2 + 0.05 * call))
        keep = logl > lstar
        if call == 3:
            keep[: len(keep) // 2] = False  # a smaller k forces a new capture
        xs, ls = x[keep], logl[keep]
        outs = [_run_gpu(gw, ctx, xs, ls, lstar, block, chol, None, 99, 1000 + call, 60, 4, use_graph=g, prec=1,
                         like=like) for g in (False, True)]
        for a, b in zip(*outs):
            assert np.array_equal(a, b), (call, bi)


@pytest.mark.parametrize("like,prec,unblocked", [(1, 0, 0), (1, 1, 0), (0, 1, 0), (1, 1, 1)])
def test_sweep_equals_sequential_steps(setup, like, prec, unblocked):
    # a chain's moves in one sweep are those of successive one-block steps
    # with counters counter, counter + 1, ...: bit-identical, although chains
    # start their next block at different rounds
    gw, ctx, prob, het, loglike_u, x, logl = setup
    lstar = float(np.quantile(logl, 0.25))
    keep = logl > lstar
    xs, ls = x[keep], logl[keep]
    # unblocked: the 11-coordinate block five times (one packed factor),
    # then two Gibbs blocks
    blocks = [tuple(range(11))] * 5 + list(S.BLOCKS[:2]) if unblocked else list(S.BLOCKS)
    chols = [S.block_cholesky(x, b) for b in blocks]
    seed, counter = 17, 500
    k = len(xs)
    xa = torch.from_numpy(xs.copy()).cuda()
    la = torch.from_numpy(ls.copy()).cuda()
    nea = torch.zeros(k, dtype=torch.int32, device="cuda")
    sta = torch.zeros(k, dtype=torch.int32, device="cuda")
    gw.slice_sweep(ctx.handle, xa, la, lstar, blocks, chols, seed=seed, counter=counter, w=1.0, max_out=4,
                   max_shrink=60, like=like, marg=gw.GW_MARG_PHASE_DIST, prec=prec, n_evals=nea, status=sta)
    xb = torch.from_numpy(xs.copy()).cuda()
    lb = torch.from_numpy(ls.copy()).cuda()
    ne_sum = np.zeros(k, np.int64)
    st_sum = np.zeros(k, np.int64)
    for b, (blk, ch) in enumerate(zip(blocks, chols)):
        ne = torch.zeros(k, dtype=torch.int32, device="cuda")
        st = torch.zeros(k, dtype=torch.int32, device="cuda")
        gw.slice_step(ctx.handle, xb, lb, lstar, blk, ch, seed=seed, counter=counter + b, w=1.0, max_out=4,
                      max_shrink=60, like=like, marg=gw.GW_MARG_PHASE_DIST, prec=prec, n_evals=ne, status=st)
        ne_sum += ne.cpu().numpy()
        st_sum += st.cpu().numpy()
    torch.cuda.synchronize()
    assert np.array_equal(xa.cpu().numpy(), xb.cpu().numpy())
    assert np.array_equal(la.cpu().numpy(), lb.cpu().numpy())
    assert np.array_equal(nea.cpu().numpy(), ne_sum)
    assert np.array_equal(sta.cpu().numpy(), st_sum)
    assert np.all(la.cpu().numpy() > lstar)
    print(f"like {like} prec {prec}: {k} chains, {int(ne_sum.sum())} evals, {int(st_sum.sum())} capped blocks")


def test_sweep_one_block_equals_step_and_errors(setup):
    gw, ctx, prob, het, loglike_u, x, logl = setup
    lstar = float(np.quantile(logl, 0.3))
    keep = logl > lstar
    xs, ls = x[keep], logl[keep]
    blk = S.BLOCKS[0]
    ch = S.block_cholesky(x, blk)
    a = _run_gpu(gw, ctx, xs, ls, lstar, blk, ch, None, 3, 77, 60, 4, prec=1)
    xt = torch.from_numpy(xs.copy()).cuda()
    lt = torch.from_numpy(ls.copy()).cuda()
    ne = torch.zeros(len(xs), dtype=torch.int32, device="cuda")
    st = torch.zeros(len(xs), dtype=torch.int32, device="cuda")
    gw.slice_sweep(ctx.handle, xt, lt, lstar, [blk], [ch], seed=3, counter=77, w=1.0, max_out=4, max_shrink=60,
                   like=gw.GW_HET, marg=gw.GW_MARG_PHASE_DIST, prec=1, n_evals=ne, status=st)
    torch.cuda.synchronize()
    for u, v in zip(a, (xt.cpu().numpy(), lt.cpu().numpy(), ne.cpu().numpy(), st.cpu().numpy())):
        assert np.array_equal(u, v)
    with pytest.raises(gw.GwError):
        gw.slice_sweep(ctx.handle, xt, lt, lstar, [[0, 0]], [np.eye(2)])  # repeated index
    with pytest.raises(gw.GwError):
        gw.slice_sweep(ctx.handle, xt, lt, lstar, [[0], [11]], [np.eye(1), np.eye(1)])  # out of range
    with pytest.raises(gw.GwError):
        gw.slice_sweep(ctx.handle, xt, lt, lstar, [[0]], [np.eye(1)], marg=gw.GW_MARG_PHASE)
    with pytest.raises(ValueError):
        gw.slice_sweep(ctx.handle, xt, lt, lstar, [[0]] * 17, [np.eye(1)] * 17)
    with pytest.raises(gw.GwError):  # two distinct 11-coordinate factors exceed the packed store
        gw.slice_sweep(ctx.handle, xt, lt, lstar, [list(range(11))] * 2, [np.eye(11), 0.5 * np.eye(11)])


def test_sweeps_between_other_heterodyned_calls(setup):
    # A heterodyned sweep writes the likelihood's argument block once and its
    # rounds (replayed from a graph) reuse it.  Batch calls on other rows
    # between sweeps rewrite the block; the next sweep must rewrite it again,
    # so graph-replayed sweeps interleaved with such calls equal eager sweeps,
    # and the batch calls equal the same call made alone.
    gw, ctx, prob, het, loglike_u, x, logl = setup
    blocks = list(S.BLOCKS)
    chols = [S.block_cholesky(x, b) for b in blocks]
    lstar = float(np.quantile(logl, 0.3))
    keep = logl > lstar
    xs, ls = x[keep], logl[keep]

    def sweep(use_graph, counter):
        xt = torch.from_numpy(xs.copy()).cuda()
        lt = torch.from_numpy(ls.copy()).cuda()
        ne = torch.zeros(len(xs), dtype=torch.int32, device="cuda")
        st = torch.zeros(len(xs), dtype=torch.int32, device="cuda")
        gw.slice_sweep(ctx.handle, xt, lt, lstar, blocks, chols, seed=11, counter=counter, w=1.0, max_out=4,
                       max_shrink=60, like=gw.GW_HET, marg=gw.GW_MARG_PHASE_DIST, prec=gw.GW_PREC_MIXED,
                       n_evals=ne, status=st, use_graph=use_graph)
        torch.cuda.synchronize()
        return [t.cpu().numpy() for t in (xt, lt, ne, st)]

    th = gw.gw_prior_transform(ctx.handle, torch.from_numpy(x[:37].copy()).cuda())
    alone = gw.loglike_batch(ctx.handle, th, gw.GW_HET, gw.GW_MARG_PHASE_DIST, gw.GW_PREC_MIXED).cpu().numpy()
    eager = [sweep(False, c) for c in (500, 600, 700)]
    replayed, between = [], []
    for c in (500, 600, 700):
        replayed.append(sweep(True, c))
        between.append(gw.loglike_batch(ctx.handle, th, gw.GW_HET, gw.GW_MARG_PHASE_DIST,
                                        gw.GW_PREC_MIXED).cpu().numpy())
    for call, (a, b) in enumerate(zip(eager, replayed)):
        for u, v in zip(a, b):
            assert np.array_equal(u, v), call
    assert eager[0][2].sum() > 0
    for v in between:
        assert np.array_equal(v, alone)
