"""The detector sky frame of the sampler on the GPU, against the oracle.

The device prior transform in the detector frame (zenith and azimuth about
the baseline of detectors 0 and 1, optionally with the arrival time at
detector 0 as coordinate 10) against the oracle's transform; slice moves in
that frame chain by chain, as in the equatorial tests; argument errors.
"""
import math

import numpy as np
import pytest

import gwsynth
from oracle import detector as D
from oracle import heterodyne as H
from oracle import likelihood as L
from oracle import sampler as S
from tests.gpu_common import scale_to_snr, with_injection

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_2607_28265_amd as gw
    prob = gwsynth.make_problem(8.0, 20.0, 512.0, psd_scale=1e-49, gmst=0.7)
    th = gwsynth.prior_draws(gwsynth.SEEDS["injection"], 1)[0]
    prob = with_injection(prob, scale_to_snr(prob, th, 24.0))
    ctx = gw.Context(prob)
    ctx.heterodyne_setup(prob.theta_inj, 200)
    het = H.setup(prob, prob.theta_inj, 200)
    yield gw, ctx, prob, het
    gw.gw_set_sky_frame(ctx.handle, 0)
    ctx.close()


# the detector time replaces the sampled t_c, so it has no time-marginal form
@pytest.mark.parametrize("det_time,marg", [(False, 2), (True, 2), (False, 3)])
def test_transform_matches_oracle(setup, det_time, marg):
    gw, ctx, prob, het = setup
    gw.gw_set_sky_frame(ctx.handle, 1, 0, 1, det_time)
    u = np.random.default_rng(5).uniform(size=(512, 11))
    u[0, 8] = 0.0  # along the baseline
    u[1, 8] = 1.0  # opposite
    got = gw.gw_prior_transform(ctx.handle, torch.from_numpy(u).cuda(), marg=marg).cpu().numpy()
    dr = (prob.dist_grid[0], prob.dist_grid[-1]) if marg == 3 else None
    for r in range(len(u)):
        want = S.prior_transform_frame(u[r], prob.det_pos, prob.gmst, det_time=det_time, d_range=dr)
        d = np.abs(got[r] - want)
        d[8] = min(d[8], 2 * math.pi - d[8])  # ra modulo 2 pi
        assert np.all(d < 1e-12), (r, got[r], want)
    gw.gw_set_sky_frame(ctx.handle, 0)


@pytest.mark.parametrize("det_time", [False, True])
@pytest.mark.parametrize("block", [(7, 8), (10,), (0, 1, 4, 5)])
def test_slice_moves_in_the_detector_frame(setup, block, det_time):
    gw, ctx, prob, het = setup
    gw.gw_set_sky_frame(ctx.handle, 1, 0, 1, det_time)
    dd = L.data_inner(prob)
    to_theta = lambda u: S.prior_transform_frame(u, prob.det_pos, prob.gmst, det_time=det_time)
    loglike_u = lambda u: H.loglike(to_theta(u), prob, het, L.PHASE_DIST, dd)
    # start points: the injection's cube point in this frame plus noise
    n, e1, e2 = S.sky_frame_basis(prob.det_pos)
    sv, _, _ = D.source_frame(prob.theta_inj[8], prob.theta_inj[9], prob.gmst)
    u0 = np.empty(11)
    th0 = prob.theta_inj
    lo = np.array([1.1, 0.5, -0.05, -0.05, 0.0, 0.0])
    hi = np.array([1.4, 1.0, 0.05, 0.05, 5000.0, 5000.0])
    u0[:6] = (th0[:6] - lo) / (hi - lo)
    u0[6] = (1 - math.cos(th0[7])) / 2
    u0[7] = (math.atan2(sv @ e2, sv @ e1) % (2 * math.pi)) / (2 * math.pi)
    u0[8] = (1 - float(sv @ n)) / 2
    u0[9] = th0[10] / math.pi
    ta = th0[12] - float(sv @ prob.det_pos[0]) / S.C_SI if det_time else th0[12]
    u0[10] = (ta + 0.1) / 0.2
    assert np.allclose(to_theta(u0)[[8, 9, 12]], th0[[8, 9, 12]], atol=1e-12)
    rng = np.random.default_rng(6)
    x = np.clip(u0 + 0.003 * rng.standard_normal((48, 11)), 0.001, 0.999)
    logl = np.array([loglike_u(p) for p in x])
    lstar = float(np.quantile(logl, 0.25))
    keep = logl > lstar
    x, logl = x[keep], logl[keep]
    chol = S.block_cholesky(x, block)
    seed, counter, max_shrink, max_out = 21, 5, 60, 4
    xt = torch.from_numpy(x.copy()).cuda()
    lt = torch.from_numpy(logl.copy()).cuda()
    ne = torch.zeros(len(x), dtype=torch.int32, device="cuda")
    gw.slice_step(ctx.handle, xt, lt, lstar, block, chol, seed=seed, counter=counter, w=1.0, max_out=max_out,
                  max_shrink=max_shrink, like=gw.GW_HET, marg=gw.GW_MARG_PHASE_DIST, prec=0, n_evals=ne)
    torch.cuda.synchronize()
    gx, gl, gne = xt.cpu().numpy(), lt.cpu().numpy(), ne.cpu().numpy()
    n_cmp = 0
    for c in range(len(x)):
        uni = S.philox_uniforms(seed, counter, c, S.n_fixed_uniforms(len(block)) + max_shrink)
        ox, ol, one, ost, margin = S.slice_chain(x[c], logl[c], lstar, block, chol, uni, loglike_u, 1.0, max_out,
                                                 max_shrink)
        if margin < 1e-6:
            continue
        n_cmp += 1
        assert gne[c] == one and np.max(np.abs(gx[c] - ox)) < 1e-12 and abs(gl[c] - ol) < 1e-6, c
    gw.gw_set_sky_frame(ctx.handle, 0)
    print(f"block {block} det_time {det_time}: {n_cmp}/{len(x)} chains compared", flush=True)
    assert n_cmp >= len(x) - 2


def test_sky_frame_errors(setup):
    gw, ctx, prob, het = setup
    for args in [(2, 0, 1, 0), (1, 0, 0, 0), (1, 0, 3, 0), (1, -1, 1, 0), (0, 0, 1, 1)]:
        with pytest.raises(gw.GwError):
            gw.gw_set_sky_frame(ctx.handle, *args)
    gw.gw_set_sky_frame(ctx.handle, 0)
