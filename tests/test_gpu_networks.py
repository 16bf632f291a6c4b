"""Detector networks of 1, 2 and 4 detectors (the kernels are instantiated
per detector count; the benchmark uses 3).  Full band in every form and the
heterodyned path against the oracle on a 4 s, 20-256 Hz segment with an
SNR-24 injection (PSD scale 1e-49) and a mix of prior and near-posterior
proposals, GMST non-zero."""
import numpy as np
import pytest

import gwsynth
from oracle import heterodyne as H
from oracle import likelihood as L
from tests.gpu_common import oracle_many, scale_to_snr, with_injection

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = {0: 1e-6, 1: 1e-3}
MARGS = (L.PLAIN, L.PHASE, L.PHASE_DIST)


def network(n_det):
    prob = gwsynth.make_problem(4.0, 20.0, 256.0, psd_scale=1e-49, n_det=n_det, det_seed=11 + n_det, gmst=0.7)
    th = gwsynth.prior_draws(gwsynth.SEEDS["injection"], 1)[0]
    th = scale_to_snr(prob, th, 24.0)
    return with_injection(prob, th)


@pytest.mark.parametrize("n_det", [1, 2, 4])
def test_network_full_band_and_heterodyne(n_det):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2607_28265_amd as gw
    prob = network(n_det)
    th = np.concatenate([gwsynth.prior_draws(70 + n_det, 150),
                         gwsynth.near_posterior(80 + n_det, prob.theta_inj, 150, scale=0.5)])
    t = torch.from_numpy(th).cuda()
    het = H.setup(prob, prob.theta_inj, 64)
    with gw.Context(prob) as ctx:
        ctx.heterodyne_setup(prob.theta_inj, 64)
        for marg in MARGS:
            ref = oracle_many(th, prob, marg)
            for prec, kind in ((0, 1), (1, 1), (1, 2)):
                if kind == 2 and ctx.mom_blk == 0:
                    continue
                ctx.set_full_kernel(kind)
                got = ctx.loglike(t, marg=marg, prec=prec).cpu().numpy()
                ctx.set_full_kernel(0)
                err = np.max(np.abs(got - ref))
                print(f"{n_det} det full marg={marg} prec={prec} kind={kind}: max|dlogL|={err:.3e}", flush=True)
                assert np.all(np.isfinite(got)) and err < TOL[prec]
            href = H.loglike_many(th, prob, het, marg)
            for prec in (0, 1):
                got = ctx.loglike(t, like=gw.GW_HET, marg=marg, prec=prec).cpu().numpy()
                err = np.max(np.abs(got - href))
                print(f"{n_det} det het marg={marg} prec={prec}: max|dlogL|={err:.3e}", flush=True)
                assert np.all(np.isfinite(got)) and err < TOL[prec]
