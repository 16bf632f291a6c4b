"""GPU prescreen network against the FP64 network oracle, and the prescreen's
gain on a nested-sampling state.

* gradients of the FP32 training path vs the oracle's backward pass (same
  FP32-rounded parameters, inputs and targets), with and without split-K;
* two Adam steps vs the oracle's Adam;
* FP32 forward vs the oracle forward; BF16 matrix-core forward vs the oracle
  forward with the BF16 path's quantisation points (tolerance from FP32
  accumulation and rare rounding flips), and its error vs the unquantised net;
* prescreened evaluation: flags, audit draws (Philox from the oracle's
  generator), exact confirmation; then the gain after training on pairs the
  sampler produced.
"""
import math

import numpy as np
import pytest

import gwsynth
from oracle import mlp as M
from oracle import sampler as S
from tests.gpu_common import problem

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2607_28265_amd as gw
    c = gw.Context(problem("cfg1", loud=True))
    yield c
    c.close()


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def random_params(seed, bias_sd=0.05):
    p = M.init(seed)
    rng = np.random.default_rng(seed + 100)
    p = [(w, rng.normal(0.0, bias_sd, b.shape)) for w, b in p]
    vec = M.flatten(p).astype(np.float32)
    return vec, M.unflatten(vec.astype(np.float64))


def make_mlp(ctx, vec, xm=None, xs=None, ym=0.0, ys=1.0):
    import paper_2607_28265_amd as gw
    m = gw.Mlp(ctx, seed=7)
    m.set_params(vec)
    m.set_scaling(np.zeros(11) if xm is None else xm, np.ones(11) if xs is None else xs, ym, ys)
    return m


@pytest.mark.parametrize("n", [300, 2500])
def test_gradients_match_oracle(ctx, n):
    vec, params = random_params(11)
    m = make_mlp(ctx, vec)
    rng = np.random.default_rng(n)
    x = rng.uniform(size=(n, 11))
    t = rng.normal(size=n)
    g, loss = m.grad(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda())
    y, cache = M.forward(params, f32(x))
    go = M.flatten(M.backward(params, cache, y, f32(t)))
    lo = float(np.mean((y - f32(t)) ** 2))
    assert abs(loss - lo) <= 1e-5 * lo, (loss, lo)
    off = 0
    for a, b in zip(M.SIZES[:-1], M.SIZES[1:]):
        for cnt, name in ((a * b, "W"), (b, "b")):
            gg, oo = g[off:off + cnt], go[off:off + cnt]
            err = np.max(np.abs(gg - oo))
            scale = np.max(np.abs(oo))
            print(f"n={n} layer {a}->{b} {name}: max err {err:.3e} / max {scale:.3e}")
            assert err <= 1e-4 * scale + 1e-9, (a, b, name, err, scale)
            off += cnt
    m.close()


def test_two_adam_steps_match_oracle(ctx):
    vec, params = random_params(12)
    m = make_mlp(ctx, vec)
    rng = np.random.default_rng(5)
    x = rng.uniform(size=(777, 11))
    t = rng.normal(size=777)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    lr = 1e-3
    st = M.adam_state(params)
    big = []
    for _ in range(2):
        m.train_step(xd, td, lr)
        y, cache = M.forward(params, f32(x))
        gr = M.backward(params, cache, y, f32(t))
        gflat = M.flatten(gr)
        big.append(np.abs(gflat) > 1e-3 * np.max(np.abs(gflat)))
        M.adam_step(params, gr, st, lr)
    torch.cuda.synchronize()
    p_gpu = m.get_params().astype(np.float64)
    p_or = M.flatten(params)
    mask = big[0] & big[1]
    err = np.abs(p_gpu - p_or)
    print(f"adam: {mask.mean():.3f} of coordinates checked, max err {err[mask].max():.3e}, "
          f"max move {np.max(np.abs(p_or - vec)):.3e}")
    assert mask.mean() > 0.3
    assert np.all(err[mask] <= 1e-2 * lr + 1e-6 * np.abs(p_or[mask]))
    assert np.all(np.abs(p_gpu - vec) <= 2.0 * lr * 1.001 + 1e-7)  # Adam moves at most lr per step (|m|<=sqrt v)
    m.close()


def _std_input(x, xm, xs):
    inv = (1.0 / xs).astype(np.float32)
    return ((x.astype(np.float32) - xm.astype(np.float32)) * inv).astype(np.float64)


@pytest.mark.parametrize("n", [1, 333, 4096])
def test_forward_fp32_and_bf16_match_oracle(ctx, n):
    vec, params = random_params(13)
    rng = np.random.default_rng(n + 1)
    xm = rng.uniform(0.3, 0.7, size=11)
    xs = rng.uniform(0.1, 0.4, size=11)
    ym, ys = -1234.5, 17.0
    m = make_mlp(ctx, vec, xm, xs, ym, ys)
    x = rng.uniform(size=(n, 11))
    xd = torch.from_numpy(x).cuda()
    a = _std_input(x, xm, xs)
    y32 = (m.forward(xd, bf16=False).cpu().numpy() - ym) / ys
    y16 = (m.forward(xd, bf16=True).cpu().numpy() - ym) / ys
    yo, _ = M.forward(params, a)
    yq = M.forward_bf16(params, a)
    scale = 1.0 + np.max(np.abs(yo))
    e32 = np.max(np.abs(y32 - yo))
    e16 = np.max(np.abs(y16 - yq))
    eq = np.max(np.abs(y16 - yo))
    print(f"n={n}: fp32 err {e32:.2e}, bf16 vs quantised oracle {e16:.2e}, bf16 vs exact net {eq:.2e}, "
          f"scale {scale:.2f}")
    assert e32 <= 1e-5 * scale
    assert e16 <= 1e-3 * scale
    assert eq <= 5e-2 * scale
    m.close()


def test_params_roundtrip_and_errors(ctx):
    import paper_2607_28265_amd as gw
    assert gw.Mlp.n_params() == 134913
    vec, _ = random_params(14)
    m = make_mlp(ctx, vec)
    assert np.array_equal(m.get_params(), vec)
    with pytest.raises(gw.GwError):
        m.set_scaling(np.zeros(11), np.zeros(11), 0.0, 1.0)
    with pytest.raises(gw.GwError):
        m.set_scaling(np.zeros(11), np.ones(11), 0.0, -1.0)
    with pytest.raises(gw.GwError):
        m.train_step(torch.zeros((4, 11), dtype=torch.float64, device="cuda"),
                     torch.zeros(4, dtype=torch.float64, device="cuda"), -1.0)
    out = m.forward(torch.zeros((0, 11), dtype=torch.float64, device="cuda"))
    assert out.numel() == 0
    m.close()


def _philox_audit(seed, i):
    w = S.philox4x64((i, 0, 0, 0), (seed, 1))[0]
    return ((w >> 11) + 0.5) * 2.0 ** -53


def test_prescreen_flags_audit_and_exact_confirmation(ctx):
    import paper_2607_28265_amd as gw
    vec, _ = random_params(15)
    m = make_mlp(ctx, vec, ym=-11700.0, ys=30.0)
    n = 3000
    x = np.random.default_rng(8).uniform(size=(n, 11))
    xd = torch.from_numpy(x).cuda()
    th = gw.gw_prior_transform(ctx.handle, xd)
    exact = ctx.loglike(th, marg=gw.GW_MARG_PHASE_DIST, prec=gw.GW_PREC_MIXED).cpu().numpy()
    # without the network every candidate is exact
    logl, flags, _, ne = m.prescreen(xd, -11700.0, 1.0, use_mlp=False)
    assert ne == n and np.all(flags.cpu().numpy() == 1)
    assert np.allclose(logl.cpu().numpy(), exact, rtol=0, atol=1e-7)
    # with it: bit1 iff pred >= cut; bit2 = audit draw among the rest
    pred = m.forward(xd).cpu().numpy()
    cut_star, margin, af, seed = float(np.median(pred)), 0.5, 0.05, 99
    logl, flags, pr, ne = m.prescreen(xd, cut_star, margin, audit_frac=af, seed=seed, use_mlp=True)
    flags, logl, pr = flags.cpu().numpy(), logl.cpu().numpy(), pr.cpu().numpy()
    assert np.array_equal(pr, pred)
    passed = pred >= cut_star - margin
    assert np.array_equal((flags & 2) != 0, passed)
    aud = np.array([(not passed[i]) and _philox_audit(seed, i) < af for i in range(n)])
    assert np.array_equal((flags & 4) != 0, aud)
    ev = (flags & 1) != 0
    assert np.array_equal(ev, passed | aud) and ne == int(ev.sum())
    assert np.all(np.isneginf(logl[~ev]))
    assert np.allclose(logl[ev], exact[ev], rtol=0, atol=1e-7)
    m.close()


@pytest.fixture(scope="module")
def trained(ctx):
    """A nested-sampling state, a network trained on the sampler's own pairs
    and one exactly evaluated candidate batch, and a fresh candidate batch."""
    import paper_2607_28265_amd as gw
    from paper_2607_28265_amd import prescreen as P
    from paper_2607_28265_amd.nested import NestedSampler
    ns = NestedSampler(ctx, n_live=500, n_delete=62, seed=6, like=gw.GW_FULL, prec=gw.GW_PREC_MIXED)
    for _ in range(180):
        ns.step()
    live_x = ns.x.cpu().numpy()
    live_l = ns.logl.cpu().numpy()
    lstar = float(np.sort(live_l)[ns.k - 1])
    xp, yp = P.sampler_pairs(ns, last_iters=30)

    def exact(xc):
        th = gw.gw_prior_transform(ctx.handle, torch.from_numpy(xc).cuda())
        return ctx.loglike(th, marg=gw.GW_MARG_PHASE_DIST, prec=gw.GW_PREC_MIXED).cpu().numpy()

    xa = P.slice_candidates(live_x, 16384, seed=1)
    ya = exact(xa)
    pre = P.Prescreen(ctx, seed=7)
    tr = pre.train(np.concatenate([xp, xa]), np.concatenate([yp, ya]), live_x, lstar)
    margin = pre.set_margin(lstar)
    xb = P.slice_candidates(live_x, 16384, seed=2)
    yb = exact(xb)
    print(f"train: {tr}; logL* {lstar:.3f}; margin {margin:.3f}")
    yield dict(pre=pre, lstar=lstar, xb=xb, yb=yb, tr=tr)
    pre.close()


def test_training_learns_the_likelihood_surface(trained):
    tr = trained["tr"]
    assert tr.loss_last < 0.05 * tr.loss_first
    pre, lstar, xb, yb = trained["pre"], trained["lstar"], trained["xb"], trained["yb"]
    p = pre.predict(torch.from_numpy(xb).cuda()).cpu().numpy()
    near = np.abs(yb - lstar) < 10.0
    rmse = float(np.sqrt(np.mean((p[near] - yb[near]) ** 2)))
    print(f"fresh candidates near logL*: {near.sum()}, rmse {rmse:.3f}, holdout rmse {tr.rmse_holdout:.3f}")
    assert near.sum() > 100
    assert rmse < 2.0


def test_prescreen_gain_with_exact_confirmation(trained):
    pre, lstar, xb, yb = trained["pre"], trained["lstar"], trained["xb"], trained["yb"]
    n = len(xb)
    logl, flags, pred, ne = pre.screen(torch.from_numpy(xb).cuda(), lstar, audit_frac=0.01, seed=3)
    logl, flags = logl.cpu().numpy(), flags.cpu().numpy()
    ev = (flags & 1) != 0
    truth_acc = yb > lstar
    got_acc = ev & (logl > lstar)
    # every accepted point is confirmed by the exact likelihood
    assert np.allclose(logl[ev], yb[ev], rtol=0, atol=1e-7)
    assert not np.any(got_acc & ~truth_acc)
    fn = truth_acc & ~ev
    aud = (flags & 4) != 0
    print(f"candidates {n}: exact without screen {n}, with {ne} ({ne / n:.3f}); accepted true "
          f"{truth_acc.sum()}, kept {got_acc.sum()}, false negatives {fn.sum()}; audited {aud.sum()} "
          f"of which accepted {int((aud & (logl > lstar)).sum())}")
    assert truth_acc.sum() > 50
    assert ne <= 0.8 * n  # at least 20 % of the exact evaluations saved
    assert fn.sum() <= 0.01 * truth_acc.sum()


def _to_cube(th):
    # inverse of the oracle's unit-cube prior transform (coordinates 0..10)
    u = np.empty(11)
    u[:6] = (th[:6] - S.PRIOR_LO) / (S.PRIOR_HI - S.PRIOR_LO)
    u[6] = (1.0 - math.cos(th[7])) / 2.0
    u[7] = th[8] / (2.0 * math.pi)
    u[8] = (math.sin(th[9]) + 1.0) / 2.0
    u[9] = th[10] / math.pi
    u[10] = (th[12] + 0.1) / 0.2
    return u


@pytest.mark.timeout(600)
def test_prescreen_confirmation_on_the_128s_grid_matches_oracle():
    # The prescreen's exact confirmation on the full-band 128 s grid (259,585
    # bins x 3 detectors, the grid the learned-prescreen workload confirms on):
    # every candidate the screen sends for evaluation gets the exact
    # phase+distance-marginal log L, compared here with the oracle's own
    # likelihood of the oracle's own prior transform of the same cube point.
    import paper_2607_28265_amd as gw
    from oracle import likelihood as L
    from tests.gpu_common import oracle_many
    prob = problem("cfg2", loud=True)
    rng = np.random.default_rng(17)
    n = 1024
    u0 = _to_cube(prob.theta_inj)
    x = np.concatenate([rng.uniform(size=(n // 2, 11)),
                        np.clip(u0 + 0.003 * rng.standard_normal((n // 2, 11)), 0.0, 1.0)])
    xd = torch.from_numpy(x).cuda()
    with gw.Context(prob) as c:
        vec, _ = random_params(16)
        m = make_mlp(c, vec, ym=-778000.0, ys=50.0)
        pred = m.forward(xd).cpu().numpy()
        cut = float(np.median(pred))
        ev_prev = None
        for prec, tol in ((gw.GW_PREC_FP64, 1e-6), (gw.GW_PREC_MIXED, 1e-3)):
            logl, flags, _, ne = m.prescreen(xd, cut, 0.0, audit_frac=0.02, seed=5, use_mlp=True, prec=prec)
            logl, flags = logl.cpu().numpy(), flags.cpu().numpy()
            ev = (flags & 1) != 0
            assert 0.3 * n < ne == ev.sum() < 0.8 * n
            if ev_prev is None:
                ref = oracle_many(np.array([S.prior_transform(u) for u in x[ev]]), prob, L.PHASE_DIST)
                ev_prev = ev
            assert np.array_equal(ev, ev_prev)  # the screen does not depend on the likelihood's precision
            err = np.abs(logl[ev] - ref)
            print(f"prescreen 128 s prec {prec}: {ne} confirmed of {n}, max |dlogL| vs oracle {err.max():.2e}, "
                  f"logL {ref.min():.1f} .. {ref.max():.1f}", flush=True)
            assert err.max() < tol
            assert np.all(np.isneginf(logl[~ev]))
        m.close()
