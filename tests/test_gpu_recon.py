"""GPU post-hoc reconstruction of (d_L, phi_c) against the oracle, sample by sample.

Both sides draw with the same uniforms.  The grid indices are integers decided
by floating point: they must agree, except where u falls within the
likelihood tolerance of a boundary of the oracle's cumulative weights.  There
either neighbouring index is a correct draw, and the test checks that the
GPU's index is one of them.  The drawn values are then the grid nodes
themselves, compared exactly.
"""
import math

import numpy as np
import pytest

import gwsynth
from oracle import heterodyne as H
from oracle import likelihood as L
from oracle import reconstruct as R
from tests.gpu_common import N_PROC, problem

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _cdf(logw):
    w = np.exp(np.asarray(logw) - np.max(logw))
    return np.cumsum(w) / np.sum(w)


def _index_ok(gpu_j, ora_j, logw, u, tol):
    """Same index, or u within tol of the cumulative boundary between them."""
    if gpu_j == ora_j:
        return True, False
    if gpu_j < 0 or abs(gpu_j - ora_j) != 1:
        return False, True
    c = _cdf(logw)
    return abs(c[min(gpu_j, ora_j)] - u) < tol, True


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_2607_28265_amd as gw
    prob = problem("cfg1", loud=True)
    het = H.setup(prob, prob.theta_inj, 200)
    ctx = gw.Context(prob)
    ctx.heterodyne_setup(prob.theta_inj, 200)
    n = 96
    th = gwsynth.near_posterior(31, prob.theta_inj, n, scale=1.0)
    th[5, 1] = 1.5   # unphysical: q > 1
    th[17, 0] = -1.0  # unphysical: Mc < 0
    uni = np.random.default_rng(8).uniform(size=(n, 2))
    yield gw, ctx, prob, het, th, uni
    ctx.close()


@pytest.mark.parametrize("like", [0, 1])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("marg", [1, 2])
def test_reconstruct_matches_oracle(setup, like, prec, marg):
    gw, ctx, prob, het, th, uni = setup
    n_phase = 2048
    tt = torch.from_numpy(th).cuda()
    ut = torch.from_numpy(uni).cuda()
    out, idx, logl = gw.gw_reconstruct(ctx.handle, tt, ut, like=like, marg=marg, prec=prec, n_phase=n_phase)
    torch.cuda.synchronize()
    out, idx, logl = out.cpu().numpy(), idx.cpu().numpy(), logl.cpu().numpy()
    hh = het if like == 1 else None
    tol = 1e-9 if prec == 0 else 1e-4
    dd = L.data_inner(prob)
    n_edge = 0
    for r in range(len(th)):
        if not L.is_physical(th[r], marg):
            assert math.isnan(out[r, 0]) and math.isnan(out[r, 1]) and idx[r, 0] == -1 and idx[r, 1] == -1
            assert logl[r] == -math.inf
            continue
        d, phi, j, m = R.reconstruct(th[r], prob, uni[r], marg, n_phase, het=hh)
        z, h2 = R.sample_overlap(th[r], prob, marg, hh)
        if marg == 2:
            ok, edge = _index_ok(idx[r, 0], j, R.distance_logweights(z, h2, prob), uni[r, 0], tol)
            assert ok, (r, idx[r, 0], j)
            n_edge += edge
            jj = idx[r, 0]
            assert out[r, 0] == prob.dist_grid[jj]
            zc = z / prob.dist_grid[jj]
            if edge:  # the phase draw then follows the GPU's distance
                m = R.draw_index(R.phase_logweights(zc, n_phase), uni[r, 1])
        else:
            assert idx[r, 0] == -1 and out[r, 0] == th[r, 6]
            zc = z
        ok, edge = _index_ok(idx[r, 1], m, R.phase_logweights(zc, n_phase), uni[r, 1], tol)
        assert ok, (r, idx[r, 1], m)
        n_edge += edge
        assert out[r, 1] == 2 * math.pi * idx[r, 1] / n_phase
        want = H.loglike(th[r], prob, het, marg, dd) if like == 1 else L.loglike(th[r], prob, marg, dd)
        assert abs(logl[r] - want) < (1e-6 if prec == 0 else 1e-3), (r, logl[r], want)
    print(f"like {like} prec {prec} marg {marg}: {len(th)} samples, {n_edge} boundary draws", flush=True)
    assert n_edge <= 2


def test_reconstruct_edge_cases(setup):
    gw, ctx, prob, het, th, uni = setup
    tt = torch.from_numpy(th[:8].copy()).cuda()
    ut = torch.from_numpy(uni[:8].copy()).cuda()
    # one phase point: phi_c = 0 always
    out, idx, _ = gw.gw_reconstruct(ctx.handle, tt, ut, marg=2, prec=0, n_phase=1)
    o = out.cpu().numpy()
    ok = ~np.isnan(o[:, 0])
    assert np.all(o[ok, 1] == 0.0) and np.all(idx.cpu().numpy()[ok, 1] == 0)
    # empty batch
    e = torch.empty((0, 13), dtype=torch.float64, device="cuda")
    out, idx, logl = gw.gw_reconstruct(ctx.handle, e, torch.empty((0, 2), dtype=torch.float64, device="cuda"))
    assert out.shape == (0, 2)
    with pytest.raises(gw.GwError):
        gw.gw_reconstruct(ctx.handle, tt, ut, marg=0)
    with pytest.raises(gw.GwError):
        gw.gw_reconstruct(ctx.handle, tt, ut, marg=4)
    with pytest.raises(gw.GwError):
        gw.gw_reconstruct(ctx.handle, tt, ut, n_phase=0)
    with pytest.raises(ValueError):
        gw.gw_reconstruct(ctx.handle, tt, ut[:, :1].contiguous())


def test_reconstruct_full_size_sampled():
    """The 128 s, 20-2048 Hz band at 4096 samples (the size of the
    full-band benchmark); eight rows checked against the oracle."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_2607_28265_amd as gw
    prob = problem("cfg2", loud=True)
    n = 4096
    th = gwsynth.near_posterior(32, prob.theta_inj, n, scale=1.0)
    uni = np.random.default_rng(9).uniform(size=(n, 2))
    with gw.Context(prob) as ctx:
        out, idx, logl = gw.gw_reconstruct(ctx.handle, torch.from_numpy(th).cuda(), torch.from_numpy(uni).cuda(),
                                           like=0, marg=2, prec=1)
        torch.cuda.synchronize()
    out, idx = out.cpu().numpy(), idx.cpu().numpy()
    assert np.all(np.isin(out[:, 0], prob.dist_grid))
    rows = np.random.default_rng(10).choice(n, 8, replace=False)
    import multiprocessing as mp
    with mp.get_context("fork").Pool(min(8, N_PROC)) as pool:
        res = pool.starmap(R.reconstruct, [(th[r], prob, uni[r], 2, 2048) for r in rows])
    for r, (d, phi, j, m) in zip(rows, res):
        z, h2 = R.sample_overlap(th[r], prob, 2)
        ok, edge = _index_ok(idx[r, 0], j, R.distance_logweights(z, h2, prob), uni[r, 0], 1e-4)
        assert ok, (r, idx[r, 0], j)
        if not edge:
            ok, _ = _index_ok(idx[r, 1], m, R.phase_logweights(z / d, 2048), uni[r, 1], 1e-4)
            assert ok, (r, idx[r, 1], m)


@pytest.mark.parametrize("like", [0, 1])
@pytest.mark.parametrize("prec", [0, 1])
def test_time_reconstruction_matches_oracle(like, prec):
    # the phase+time marginal: (t_c, phi_c) drawn on the time grid and the
    # phase grid; indices as above, values the grid nodes
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_2607_28265_amd as gw
    prob = problem("cfg1", loud=True)
    th0 = prob.theta_inj.copy()
    th0[12] = 0.0
    het = H.setup(prob, th0, 200) if like == 1 else None
    n, n_phase = 40, 2048
    th = gwsynth.near_posterior(33, prob.theta_inj, n, scale=1.0)
    th[:, 12] = 0.0
    th[3, 1] = 1.5  # unphysical
    uni = np.random.default_rng(11).uniform(size=(n, 2))
    tgrid = L.time_grid(prob)
    with gw.Context(prob) as ctx:
        if like == 1:
            ctx.heterodyne_setup(th0, 200)
        out, idx, logl = gw.gw_reconstruct(ctx.handle, torch.from_numpy(th).cuda(), torch.from_numpy(uni).cuda(),
                                           like=like, marg=gw.GW_MARG_PHASE_TIME, prec=prec, n_phase=n_phase)
        torch.cuda.synchronize()
    out, idx, logl = out.cpu().numpy(), idx.cpu().numpy(), logl.cpu().numpy()
    tol = 1e-9 if prec == 0 else 1e-4
    n_edge = 0
    for r in range(n):
        if not L.is_physical(th[r], L.PHASE_TIME):
            assert math.isnan(out[r, 0]) and idx[r, 0] == -1 and logl[r] == -math.inf
            continue
        t, z, hh = R.time_conditional(th[r], prob, het)
        tc, phi, j, m = R.reconstruct_time(th[r], prob, uni[r], n_phase, het=het)
        ok, edge = _index_ok(idx[r, 0], j, R.time_logweights(z, hh), uni[r, 0], tol)
        assert ok, (r, idx[r, 0], j)
        n_edge += edge
        jj = idx[r, 0]
        assert out[r, 0] == tgrid[jj]
        if edge:
            m = R.draw_index(R.phase_logweights(z[jj], n_phase), uni[r, 1])
        ok, edge = _index_ok(idx[r, 1], m, R.phase_logweights(z[jj], n_phase), uni[r, 1], tol)
        assert ok, (r, idx[r, 1], m)
        n_edge += edge
        assert out[r, 1] == 2 * math.pi * idx[r, 1] / n_phase
    print(f"time: like {like} prec {prec}: {n} samples, {n_edge} boundary draws", flush=True)
    assert n_edge <= 2
