"""GPU slice sweep with the learned prescreen against the oracle's slice chain
applying the same rule, chain by chain.

The network (random weights; input scaling from the chains, output scaled so
that the cut log L* - margin falls inside the spread of its predictions) runs
on the GPU in BF16 on the matrix cores with FP32 accumulation; the oracle
evaluates it with the same quantisation points in FP64 (oracle.mlp.
forward_bf16) and takes the same audit draws (Philox4x64-10, key (seed, 1)).
The two network forms differ by BF16 rounding flips (up to a few 1e-2 of log L
here); a chain with a candidate on which they fall on different sides of the
cut (the GPU network is re-run on every candidate the oracle saw), or whose
oracle run came within 1e-6 of log L* in an exact evaluation, is a near tie
and only checked for validity; every other chain
must make the same moves: exact evaluations and status bit-exact, the point to
1e-12, log L to the FP64 tolerance.
"""
import math

import numpy as np
import pytest

import gwsynth
from oracle import heterodyne as H
from oracle import likelihood as L
from oracle import mlp as M
from oracle import sampler as S
from tests.gpu_common import problem

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def to_unit(th):
    u = np.empty(11)
    u[:6] = (th[:6] - S.PRIOR_LO) / (S.PRIOR_HI - S.PRIOR_LO)
    u[6] = (1 - math.cos(th[7])) / 2
    u[7] = th[8] / (2 * math.pi)
    u[8] = (math.sin(th[9]) + 1) / 2
    u[9] = th[10] / math.pi
    u[10] = (th[12] + 0.1) / 0.2
    return u


def std_input(x, xm, xs):
    # the library standardises in FP32: (x - mean) * (1 / spread)
    inv = (1.0 / xs).astype(np.float32)
    return ((np.atleast_2d(x).astype(np.float32) - xm.astype(np.float32)) * inv).astype(np.float64)


def audit_uniform(seed, counter, c, kind, idx):
    w = S.philox4x64((counter, c, kind, idx), (seed, 1))[0]
    return ((w >> 11) + 0.5) * 2.0 ** -53


def network(seed):
    p = M.init(seed)
    rng = np.random.default_rng(seed + 100)
    p = [(w, rng.normal(0.0, 0.05, b.shape)) for w, b in p]
    vec = M.flatten(p).astype(np.float32)
    return vec, M.unflatten(vec.astype(np.float64))


@pytest.fixture(scope="module")
def gw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_2607_28265_amd as gw
    return gw


def chains(prob, loglike_u, k=96, seed=5):
    u0 = to_unit(prob.theta_inj)
    rng = np.random.default_rng(seed)
    x = np.clip(u0 + 0.01 * rng.standard_normal((k, 11)), 0.001, 0.999)
    logl = np.array([loglike_u(p) for p in x])
    lstar = float(np.quantile(logl, 0.25))
    keep = logl > lstar
    return x[keep], logl[keep], lstar


@pytest.mark.parametrize("like", ["full", "het"])
def test_prescreened_sweep_matches_oracle(gw, like):
    prob = problem("cfg1", loud=True)
    dd = L.data_inner(prob)
    if like == "het":
        het = H.setup(prob, prob.theta_inj, 200)
        loglike_u = lambda u: H.loglike(S.prior_transform(u), prob, het, L.PHASE_DIST, dd)
    else:
        loglike_u = lambda u: L.loglike(S.prior_transform(u), prob, L.PHASE_DIST, dd)
    x, logl, lstar = chains(prob, loglike_u)
    k = len(x)
    blocks = list(S.BLOCKS)
    chols = [S.block_cholesky(x, b) for b in blocks]
    vec, params = network(21)
    xm, xsd = x.mean(axis=0), x.std(axis=0) + 1e-3
    y_live = M.forward_bf16(params, std_input(x, xm, xsd))
    ys = 5.0
    margin, audit = 0.5, 0.15
    ym = lstar - margin - ys * float(np.quantile(y_live, 0.3))  # the cut at the 30th percentile at the chains
    seed, counter, max_shrink, max_out = 31, 4000, 60, 4
    with gw.Context(prob) as ctx:
        if like == "het":
            ctx.heterodyne_setup(prob.theta_inj, 200)
        net = gw.Mlp(ctx, seed=7)
        net.set_params(vec)
        net.set_scaling(xm, xsd, ym, ys)
        xt = torch.from_numpy(x.copy()).cuda()
        lt = torch.from_numpy(logl.copy()).cuda()
        ne = torch.zeros(k, dtype=torch.int32, device="cuda")
        st = torch.zeros(k, dtype=torch.int32, device="cuda")
        stats = {}
        gw.slice_sweep(ctx.handle, xt, lt, lstar, blocks, chols, seed=seed, counter=counter, w=1.0,
                       max_out=max_out, max_shrink=max_shrink, like=gw.GW_HET if like == "het" else gw.GW_FULL,
                       marg=gw.GW_MARG_PHASE_DIST, prec=gw.GW_PREC_FP64, n_evals=ne, status=st,
                       prescreen=(net, margin, audit), screen_stats=stats)
        torch.cuda.synchronize()
        gx, gl, gne, gst = xt.cpu().numpy(), lt.cpu().numpy(), ne.cpu().numpy(), st.cpu().numpy()
        n_cmp = 0
        tot = {"screened": 0, "audited": 0, "audited_inside": 0}
        seen = []  # every candidate the oracle screened, to measure the two network forms' difference
        ties = []
        for c in range(k):
            xc, lc = x[c].copy(), logl[c]
            ne_o = st_o = 0
            preds = []
            margin_l = math.inf
            for b, (blk, ch) in enumerate(zip(blocks, chols)):
                uni = S.philox_uniforms(seed, counter + b, c, S.n_fixed_uniforms(len(blk)) + max_shrink)

                def screen(xp, kind, idx, b=b):
                    pv = ym + ys * float(M.forward_bf16(params, std_input(xp, xm, xsd))[0])
                    preds.append(pv)
                    seen.append(np.array(xp))
                    return pv, audit_uniform(seed, counter + b, c, kind, idx)

                xc, lc, n1, s1, m1 = S.slice_chain(xc, lc, lstar, blk, ch, uni, loglike_u, 1.0, max_out,
                                                   max_shrink, screen=screen, screen_margin=margin,
                                                   audit_frac=audit, stats=tot)
                ne_o += n1
                st_o += s1
                margin_l = min(margin_l, m1)
            ties.append((len(seen) - len(preds), len(seen), margin_l, xc, lc, ne_o, st_o))
        # the GPU network's prediction for every candidate the oracle screened
        # (the same inference kernel, row by row): a chain with a candidate on
        # which the two network forms fall on different sides of the cut is a
        # near tie
        xs_seen = np.array(seen)
        gpu_pred = net.forward(torch.from_numpy(xs_seen).cuda()).cpu().numpy()
        ora_pred = ym + ys * M.forward_bf16(params, std_input(xs_seen, xm, xsd))
        d_pred = float(np.max(np.abs(gpu_pred - ora_pred)))
        cut = lstar - margin
        flip = (gpu_pred >= cut) != (ora_pred >= cut)
        net.close()
    for c in range(k):
        i0, i1, margin_l, xc, lc, ne_o, st_o = ties[c]
        assert gl[c] > lstar or gst[c] > 0
        if np.any(flip[i0:i1]) or margin_l < 1e-6:
            continue
        n_cmp += 1
        assert gne[c] == ne_o and gst[c] == st_o, (c, gne[c], ne_o, gst[c], st_o)
        assert np.max(np.abs(gx[c] - xc)) < 1e-12
        assert abs(gl[c] - lc) < 1e-6, (c, gl[c], lc)
    print(f"{like}: {n_cmp}/{k} chains compared (network GPU vs oracle max diff {d_pred:.2e} over {len(seen)} "
          f"candidates, {int(flip.sum())} decisions flipped); GPU screen counts {stats}, oracle {tot}", flush=True)
    assert n_cmp >= 0.8 * k
    assert stats["screened"] > 0 and stats["audited"] > 0
    if n_cmp == k:
        assert stats == tot


def test_prescreen_that_passes_everything_changes_nothing(gw):
    # margin so large that every prediction clears the cut: the sweep is the
    # unscreened sweep bit for bit (the audit draws use their own key)
    prob = problem("cfg1", loud=True)
    dd = L.data_inner(prob)
    loglike_u = lambda u: L.loglike(S.prior_transform(u), prob, L.PHASE_DIST, dd)
    x, logl, lstar = chains(prob, loglike_u, k=64, seed=9)
    blocks = list(S.BLOCKS)
    chols = [S.block_cholesky(x, b) for b in blocks]
    vec, _ = network(22)
    with gw.Context(prob) as ctx:
        net = gw.Mlp(ctx, seed=7)
        net.set_params(vec)
        net.set_scaling(x.mean(axis=0), x.std(axis=0) + 1e-3, lstar, 1.0)
        out = []
        for pre in (None, (net, 1e300, 0.5)):
            for use_graph in (True, False):
                xt = torch.from_numpy(x.copy()).cuda()
                lt = torch.from_numpy(logl.copy()).cuda()
                ne = torch.zeros(len(x), dtype=torch.int32, device="cuda")
                stats = {}
                gw.slice_sweep(ctx.handle, xt, lt, lstar, blocks, chols, seed=3, counter=70, w=1.0, max_out=4,
                               max_shrink=60, like=gw.GW_FULL, marg=gw.GW_MARG_PHASE_DIST, prec=gw.GW_PREC_MIXED,
                               n_evals=ne, use_graph=use_graph, prescreen=pre, screen_stats=stats)
                torch.cuda.synchronize()
                out.append((xt.cpu().numpy(), lt.cpu().numpy(), ne.cpu().numpy()))
                if pre is not None:
                    assert stats == {"screened": 0, "audited": 0, "audited_inside": 0}
        net.close()
    for o in out[1:]:
        assert all(np.array_equal(a, b) for a, b in zip(o, out[0]))


def test_prescreen_argument_errors(gw):
    prob = problem("cfg1")
    x = torch.full((4, 11), 0.5, dtype=torch.float64, device="cuda")
    lt = torch.zeros(4, dtype=torch.float64, device="cuda")
    with gw.Context(prob) as ctx, gw.Context(prob) as other:
        net = gw.Mlp(other, seed=7)
        for pre in ((net, 1.0, 0.01), ):
            with pytest.raises(gw.GwError):  # a network of another context
                gw.slice_sweep(ctx.handle, x, lt, -1.0, [S.BLOCKS[1]], [np.eye(1)], like=gw.GW_FULL, prescreen=pre)
        net.close()
        net = gw.Mlp(ctx, seed=7)
        for pre in ((net, math.inf, 0.01), (net, 1.0, 1.5), (net, 1.0, -0.1)):
            with pytest.raises(gw.GwError):
                gw.slice_sweep(ctx.handle, x, lt, -1.0, [S.BLOCKS[1]], [np.eye(1)], like=gw.GW_FULL, prescreen=pre)
        net.close()
