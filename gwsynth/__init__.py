"""Seeded synthetic workloads for the batched gravitational-wave likelihood.

This module only *draws inputs*: the frequency grid, the analytic noise PSD,
detector geometry, Gaussian noise, prior draws of the parameter vector, the
luminosity-distance quadrature grid and the uneven sub-batch layout.  It holds
none of the likelihood's arithmetic (no waveform, no projection, no inner
product), so both the FP64 oracle and the HIP path can take its outputs as
common inputs.  The injected signal that is added to the noise is made by the
caller (the oracle in tests, the library's template entry point elsewhere).
"""
from .workload import (  # noqa: F401
    SEEDS,
    PARAM_NAMES,
    N_PARAMS,
    FreqGrid,
    freq_grid,
    psd_fit,
    detectors,
    gaussian_noise,
    prior_draws,
    near_posterior,
    distance_grid,
    uneven_split,
    CONFIGS,
    Problem,
    make_problem,
)
