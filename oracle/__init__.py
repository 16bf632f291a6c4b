"""FP64 CPU oracle of the batched gravitational-wave likelihood.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow reference written
from the paper's definitions so that the HIP path can be checked against it.
Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import it; the product path never does.  It shares no code, constants or
tables with the HIP sources.

Modules
-------
waveform    TaylorF2 phase and Newtonian amplitude (stand-in waveform).
detector    antenna patterns and geocentre time delays.
likelihood  matched-filter log-likelihood (Sec. III.A, Eq. loglike) with the
            phase and distance marginalisations.
heterodyne  relative-binning bin edges, summary data and evaluation
            (Sec. III.D).
sampler     prior transform, hit-and-run slice step, nested-sampling loop
            (Sec. II.B, II.C, III.B).
mlp         FP64 forward / backward / Adam of the prescreen network.
reconstruct post-hoc draws of the marginalised d_L and phi_c on their grids
            (grid-marginalisation appendix).
pp          credible levels, KS and Fisher p-values of an injection campaign
            (P-P calibration section).
fiducial    differential-evolution search for the heterodyne fiducial and the
            conditional peak of (d_L, phi_c) (GW170817 section).

Parity unpinned: the TaylorF2 post-Newtonian and spin coefficients beyond the
Newtonian limit and the equal-mass tidal case (the paper prints no waveform
values); agreement there is GPU-vs-oracle only.
"""
