"""Error paths of the C ABI on the GPU: an allocation that fails (forced from
the host with GW_FAULT=alloc, which makes every workspace allocation report
GW_ENOMEM) returns GW_ENOMEM and writes nothing, and the context keeps working
once allocation succeeds again."""
import numpy as np
import pytest

import gwsynth
from oracle import likelihood as L
from tests.gpu_common import problem

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def gw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_2607_28265_amd as gw
    return gw


@pytest.mark.parametrize("like", [0, 1])
def test_injected_allocation_failure_is_enomem_and_writes_nothing(gw, monkeypatch, like):
    prob = problem("cfg1")
    th = gwsynth.prior_draws(gwsynth.SEEDS["prior"], 3000)
    t = torch.from_numpy(th).cuda()
    with gw.Context(prob) as ctx:
        if like == 1:
            ctx.heterodyne_setup(prob.theta_inj, 100)
        out = torch.full((len(th),), 12345.0, dtype=torch.float64, device="cuda")
        monkeypatch.setenv("GW_FAULT", "alloc")
        with pytest.raises(gw.GwError) as e:
            ctx.loglike(t, like=like, marg=gw.GW_MARG_PHASE_DIST, prec=gw.GW_PREC_MIXED, out=out)
        torch.cuda.synchronize()
        assert e.value.status == gw._lib.GW_ENOMEM
        assert "injected" in str(e.value)
        assert bool(torch.all(out == 12345.0))
        monkeypatch.delenv("GW_FAULT")
        ctx.loglike(t, like=like, marg=gw.GW_MARG_PHASE_DIST, prec=gw.GW_PREC_FP64, out=out)
        got = out.cpu().numpy()
    assert np.all(np.isfinite(got))
    if like == 0:
        ref = np.array([L.loglike(x, prob, L.PHASE_DIST) for x in th[:8]])
        assert np.max(np.abs(got[:8] - ref)) < 1e-6
