"""The end-to-end event pipeline on a small synthetic event.

Fiducial search in the trigger's box, heterodyne on the found point, nested
sampling with the phase and coalescence time marginalised in the detector sky
frame, post-hoc (t_c, phi_c).  The checks are statistical, with wide margins:
the search lands near the injection, and the posterior means of the chirp
mass, coalescence time and distance lie within a few standard deviations of
the truth.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_event_pipeline_recovers_the_injection():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_2607_28265_amd import event
    prob, truth = event.make_event(seed=3, snr=30.0, duration=8.0, f_max=512.0)
    print("event: seed 3, 8 s, 512 Hz, SNR 30", flush=True)
    res = event.analyse(prob, float(truth[0]) + 2e-4, float(truth[12]) - 5e-4, truth, n_bins=200, pop=1024,
                        generations=60, n_live=128, n_delete=16, seed=5)
    fid = np.array(res["fiducial"])
    assert abs(fid[0] - truth[0]) < 2e-3 and abs(fid[12] - truth[12]) < 5e-3
    assert math.isfinite(res["log_z"]) and res["n_posterior_points"] > 100
    for name in ("mc", "tc", "dl"):
        row = res["posterior"][name]
        assert row["sd"] > 0.0 and abs(row["pull"]) < 5.0, (name, row)
    # reconstructed phases lie on the grid [0, 2 pi)
    assert 0.0 <= res["posterior"]["phic"]["mean"] < 2.0 * math.pi
    for k in ("search_s", "heterodyne_s", "sampling_s", "reconstruction_s"):
        assert res[k] > 0.0
