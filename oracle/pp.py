"""Calibration statistics of an injection campaign (P-P test), plain FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section on injection tests and P-P calibration:
  * for each injection and each sampled parameter, the credible level of the
    true value is the posterior mass below it,
        q = sum_s w_s 1(theta_s < theta_true) / sum_s w_s,
    taken with the nested-sampling weights w_s directly (no resampling);
  * a calibrated sampler gives credible levels uniform on [0, 1] across
    injections, which each parameter tests by the Kolmogorov-Smirnov p-value
    against U(0, 1);
  * all parameters together are summarised by Fisher's combination of their
    p-values, -2 sum ln p ~ chi^2 with 2 n_par degrees of freedom.
The KS test and Fisher's method are the library routines of scipy.stats.
"""
from __future__ import annotations

import numpy as np
from scipy import stats


def credible_level(samples, weights, truth: float) -> float:
    """Posterior mass of the samples strictly below the true value."""
    x = np.asarray(samples, dtype=np.float64)
    w = np.asarray(weights, dtype=np.float64)
    return float(np.sum(w[x < truth]) / np.sum(w))


def ks_pvalue(levels) -> float:
    """Kolmogorov-Smirnov p-value of credible levels against U(0, 1)."""
    return float(stats.kstest(np.asarray(levels, dtype=np.float64), "uniform").pvalue)


def fisher_combined(pvalues) -> float:
    """Fisher's combined p-value of independent p-values."""
    return float(stats.combine_pvalues(np.asarray(pvalues, dtype=np.float64), method="fisher").pvalue)


def pp_curve(levels, grid) -> np.ndarray:
    """Fraction of injections whose credible level is at most each grid value."""
    q = np.sort(np.asarray(levels, dtype=np.float64))
    return np.searchsorted(q, np.asarray(grid, dtype=np.float64), side="right") / q.size
