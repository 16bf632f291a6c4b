"""The allocation-free full-band entry point (loglike_batch_noalloc) against
loglike_batch, through the C ABI: two calls in a row on one context, the
second with a smaller batch (the shared device workspace keeps the first
call's contents), in every marginalisation mode and both precisions.  With the
same launch shape the two entry points run the same kernels on the same data
and must agree bit for bit; with each entry point's own shape the results may
differ only by summation order.  Batches beyond the workspace are refused."""
import numpy as np
import pytest

import gwsynth
from tests.gpu_common import problem

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

MARGS = (0, 1, 2)
TOL = {0: 1e-9, 1: 1e-6}


@pytest.fixture(scope="module")
def gw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_2607_28265_amd as gw
    return gw


@pytest.mark.parametrize("name,sizes", [("cfg1", (3000, 700)), ("cfg2", (4096, 1000))])
def test_noalloc_matches_loglike_batch(gw, name, sizes):
    prob = problem(name, loud=True)
    th_all = np.concatenate([gwsynth.near_posterior(61, prob.theta_inj, 64),
                             gwsynth.prior_draws(gwsynth.SEEDS["prior"], max(sizes) - 64)])
    with gw.Context(prob) as ctx:
        for n in sizes:  # a large call, then a smaller one on the same workspace
            th = torch.from_numpy(np.ascontiguousarray(th_all[:n])).cuda()
            for marg in MARGS:
                for prec in (gw.GW_PREC_FP64, gw.GW_PREC_MIXED):
                    # same launch shape (32 chunks fit the workspace at both sizes): bit for bit
                    ctx.set_full_shape(256 if n >= 2048 else 64, 32)
                    try:
                        ref = ctx.loglike(th, marg=marg, prec=prec).cpu().numpy()
                        out = torch.full((n,), 7.0, dtype=torch.float64, device="cuda")
                        gw.loglike_batch_noalloc(ctx.handle, th, marg=marg, prec=prec, out=out)
                        got = out.cpu().numpy()
                    finally:
                        ctx.set_full_shape(0, 0)
                    assert np.all(np.isfinite(got))
                    assert np.array_equal(got, ref), (name, n, marg, prec, np.max(np.abs(got - ref)))
                    # each entry point's own launch shape: summation order only
                    ref2 = ctx.loglike(th, marg=marg, prec=prec).cpu().numpy()
                    got2 = gw.loglike_batch_noalloc(ctx.handle, th, marg=marg, prec=prec).cpu().numpy()
                    err = np.max(np.abs(got2 - ref2))
                    print(f"{name} n={n} marg={marg} prec={prec}: default shapes max |d logL| {err:.2e}", flush=True)
                    assert err < TOL[prec]


def test_noalloc_limits_and_errors(gw):
    prob = problem("cfg1")
    with gw.Context(prob) as ctx:
        n_max = gw.noalloc_max_rows(3)
        assert n_max == (1 << 21) // (32 + 2 + 16 * 3) == 25575
        th = torch.from_numpy(gwsynth.prior_draws(gwsynth.SEEDS["prior"], n_max + 1)).cuda()
        out = torch.full((n_max + 1,), 3.0, dtype=torch.float64, device="cuda")
        with pytest.raises(gw.GwError) as e:
            gw.loglike_batch_noalloc(ctx.handle, th, out=out)
        assert e.value.status == gw._lib.GW_EINVAL and "maximum" in str(e.value)
        assert bool(torch.all(out == 3.0))
        # the largest batch runs, and matches loglike_batch at the same shape
        ctx.set_full_shape(256, 8)
        try:
            got = gw.loglike_batch_noalloc(ctx.handle, th[:n_max], marg=2, prec=1).cpu().numpy()
            ref = ctx.loglike(th[:n_max], marg=2, prec=1).cpu().numpy()
        finally:
            ctx.set_full_shape(0, 0)
        assert np.array_equal(got, ref)
        # a fixed shape that does not fit is refused, not lowered
        ctx.set_full_shape(256, 4096)
        try:
            with pytest.raises(gw.GwError):
                gw.loglike_batch_noalloc(ctx.handle, th[:4096])
        finally:
            ctx.set_full_shape(0, 0)
        with pytest.raises(gw.GwError):
            gw.loglike_batch_noalloc(ctx.handle, th[:10], marg=3)  # the time marginal is not offered
        assert gw.loglike_batch_noalloc(ctx.handle, th[:0]).numel() == 0
