// Phase runs of the mixed-precision bin walks (gw_full.hip, gw_tmarg.hip).
#pragma once

#include <math.h>

#include "gw_device.h"

namespace gw {

// Mixed form: the phase along the descending bin walk by a cubic recurrence.
// The phase in cycles is lin(f) + nl(f), lin = a5 + a8 f the constant and
// linear terms and nl the rest of the TaylorF2 series.  A run of L bins
// evaluates nl directly on its first four bins, which fixes the backward
// differences n0..n3 of nl at the fourth; every later bin then costs three
// additions (p2 += p3, p1 += p2, p0 += p1) on the table of the full phase,
// whose first difference also carries the linear term's step -a8 df.  The
// cubic's extrapolation error over a run is at most |d^4 nl / df^4| / 4!
// (L df)^4, and rounding grows with the third difference's error times
// C(L, 3), so L is limited by both: the host picks, per frequency, the
// longest of 64, 32, 16 and 8 bins that keeps the extrapolation bound below
// 2e-8 cycles for chirp masses down to 0.8 Msun (the rounding bound,
// C(64, 3) 8 eps |nl|, stays below it too), and below that frequency every
// bin is evaluated directly.  Runs are aligned blocks: bin k lies in the run
// [s, s + len[j] - 1], s = k rounded down to a multiple of len[j], for the
// first level j (len descending, powers of two) with s >= k_min[j]; a run's
// directly evaluated bins are its top ones (the walk descends), and the
// band's top run may be cut at the last bin.  Bins in no run are evaluated
// directly.  A bin's phase thus depends on its run alone, not on how the
// walk is split into chunks.
struct PhaseRuns {
  int k_min[4];
  int len[4];
};

// nl(f): the phase without the constant (a5) and linear (a8) terms.
__device__ inline double phase_nonlinear(const PhaseCoef& c, double x, double x2, double xm5, double lnf) {
  double t = fma(x2, c.a12, c.a10);
  t = x2 * t;
  t = fma(x, t, c.a7);
  t = fma(x, t, c.a6);
  t = x * t;
  t = fma(x, t, c.a4);
  t = fma(x, t, c.a3);
  t = fma(x, t, c.a2);
  t = fma(x2, t, c.a0);
  const double lg = fma(c.b6, x, c.b5);
  return fma(lg, lnf, t * xm5);
}

// Run levels for a segment of bin spacing df starting at bin k0.  The bound
// on the fourth derivative uses the leading term of the phase,
// |nl| <= A (f / 20 Hz)^(-5/3) with A = 11,500 cycles (the Newtonian phase
// of a 0.8 Msun chirp mass at 20 Hz, about 3,800 cycles, times three for the
// post-Newtonian terms); its fourth derivative is
// (5/3)(8/3)(11/3)(14/3) |nl| / f^4.
inline PhaseRuns make_phase_runs(const Geom& g) {
  const double tol = 2e-8, amp = 11500.0;
  const double c4 = (5.0 / 3.0) * (8.0 / 3.0) * (11.0 / 3.0) * (14.0 / 3.0) / 24.0;
  PhaseRuns R;
  const int lens[4] = {64, 32, 16, 8};
  for (int j = 0; j < 4; ++j) {
    const double span = lens[j] * g.df;
    // c4 amp (f/20)^(-5/3) span^4 / f^4 <= tol  <=>  f^(17/3) >= c4 amp 20^(5/3) span^4 / tol
    const double fmin = pow(c4 * amp * pow(20.0, 5.0 / 3.0) * span * span * span * span / tol, 3.0 / 17.0);
    // the run's lowest bin must lie at or above fmin
    double kmin = ceil(fmin / g.df) - (double)g.k0;
    if (kmin < 0.0) kmin = 0.0;
    if (kmin > (double)g.n_freq) kmin = (double)g.n_freq;
    R.k_min[j] = (int)kmin;
    R.len[j] = lens[j];
  }
  return R;
}

}  // namespace gw
