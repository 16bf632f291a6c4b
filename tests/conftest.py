import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def small_problem():
    """8 s, 20-512 Hz noise-only problem (3937 bins x 3 detectors)."""
    import gwsynth
    return gwsynth.make_problem(8.0, 20.0, 512.0, psd_scale=1e-46)


@pytest.fixture(scope="session")
def loud_problem():
    """8 s, 20-512 Hz, PSD scale 1e-49 with an oracle-made injection added."""
    import gwsynth
    from oracle import likelihood as L
    prob = gwsynth.make_problem(8.0, 20.0, 512.0, psd_scale=1e-49)
    theta = gwsynth.prior_draws(gwsynth.SEEDS["injection"], 1)[0]
    theta[6] = 60.0
    prob.data = prob.data + L.strain(theta, prob)
    prob.theta_inj = theta
    return prob


def rng(seed=0):
    return np.random.default_rng(seed)
