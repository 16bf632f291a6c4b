"""Pins of the oracle's coalescence-time (and phase) marginal, PHASE_TIME.

The marginal is a grid sum over time shifts t_j = j delta (the sampling
interval of the segment) of I0(|Z(t_j)|), Z(t) the overlap of the template
shifted by t.  It is pinned against:
* a library routine: on the grid t_j = j delta the shifted overlaps are a
  discrete Fourier transform of the per-bin overlap weights placed at their
  frequency indices, which numpy's FFT computes independently;
* the special case of a one-point grid, which is the phase marginal at t_c = 0;
* the time-shift property: an injection at t_c = s delta moves the overlap
  sequence by s grid points, with its peak at j = s (a wrong sign of the
  shift exponent would put it at -s);
* the zero-signal limit, where the grid average of I0(0) = 1 leaves -<d|d>/2.
"""
import math

import numpy as np
import pytest

import gwsynth
from oracle import likelihood as L


@pytest.fixture(scope="module")
def prob():
    cfg = gwsynth.CONFIGS["cfg1"]
    p = gwsynth.make_problem(cfg["duration"], cfg["f_min"], cfg["f_max"], psd_scale=1e-49)
    th = gwsynth.prior_draws(gwsynth.SEEDS["injection"], 1)[0]
    p.theta_inj = th
    return p


def test_grid(prob):
    t = L.time_grid(prob, oversample=1)
    delta = t[1] - t[0]
    # 8 s at 20-512 Hz: the segment's sampling interval is 1/1024 s
    assert delta == pytest.approx(1.0 / 1024.0, rel=1e-15)
    assert t[0] == -t[-1] and abs(t[-1]) <= L.TIME_WINDOW < abs(t[-1]) + delta
    assert t.size == 2 * 102 + 1
    # the default grid has four points per sampling interval over the same span
    t4 = L.time_grid(prob)
    assert L.TIME_OVERSAMPLE == 4 and t4.size == 2 * 102 * 4 + 1
    assert t4[1] - t4[0] == pytest.approx(delta / 4, rel=1e-15) and t4[-1] == pytest.approx(t[-1], rel=1e-15)


def test_oversampled_grid_converges_to_the_integral(monkeypatch):
    # The grid mean of I0(|Z(t)|) approximates (1 / 2W) times its integral.
    # For a loud template half a sampling interval off the grid, the plain
    # interval is far off and the error falls quickly with the oversampling;
    # the limit agrees with adaptive quadrature of the same integrand up to the
    # grid's O(1 / N_t) end correction.
    from scipy import integrate
    from scipy.special import i0e
    p = gwsynth.make_problem(4.0, 20.0, 128.0, psd_scale=1e-49)
    th = gwsynth.prior_draws(gwsynth.SEEDS["injection"], 1)[0]
    _, hh = L.overlap(th, p)
    th[6] *= math.sqrt(hh) / 40.0  # network SNR 40
    th[11] = th[12] = 0.0
    monkeypatch.setattr(L, "TIME_WINDOW", 0.004)
    native = L.time_grid(p, oversample=1)
    delta = native[1] - native[0]
    inj = th.copy()
    inj[12] = 0.5 * delta
    p.data = L.strain(inj, p)
    a, _ = L.overlap_weights(th, p)
    vals = {}
    ladder = (1, 2, 4, 8, 16, 32, 64)
    for r in ladder:
        tg = L.time_grid(p, oversample=r)
        z = np.abs(L.time_shifted_overlaps(a, p, tg))
        vals[r] = float(np.max(z) + np.log(np.mean(i0e(z) * np.exp(z - np.max(z)))))
    errs = [abs(vals[r] - vals[64]) for r in ladder[:-1]]
    assert errs[0] > 10.0 and all(x > y for x, y in zip(errs, errs[1:])) and errs[-1] < 1e-2
    zmax = np.max(np.abs(L.time_shifted_overlaps(a, p, L.time_grid(p, oversample=64))))
    f = lambda t: float(i0e(abs(L.time_shifted_overlaps(a, p, np.array([t]))[0]))
                        * np.exp(abs(L.time_shifted_overlaps(a, p, np.array([t]))[0]) - zmax))
    span = native[-1]
    integ, _ = integrate.quad(f, -span, span, points=[0.5 * delta], limit=400, epsabs=0, epsrel=1e-10)
    want = zmax + math.log(integ / (2 * span))
    n64 = L.time_grid(p, oversample=64).size
    assert abs(vals[64] - want) < 2.0 / n64


def test_shifted_overlaps_are_an_fft(prob):
    th = prob.theta_inj.copy()
    a, _ = L.overlap_weights(th, prob)
    t = L.time_grid(prob)
    z = L.time_shifted_overlaps(a, prob, t)
    n = int(round(1.0 / ((t[1] - t[0]) * prob.df)))
    x = np.zeros(n, dtype=np.complex128)
    x[prob.k0:prob.k0 + prob.n_freq] = a
    fx = np.fft.fft(x)
    j = np.rint(t / (t[1] - t[0])).astype(int)
    assert np.max(np.abs(z - fx[j % n])) < 1e-9 * np.max(np.abs(z))


def test_one_point_grid_is_phase_marginal(prob, monkeypatch):
    dd = 3.0
    th = prob.theta_inj.copy()
    th[12] = 0.0
    monkeypatch.setattr(L, "TIME_WINDOW", 0.0)
    assert L.time_grid(prob).size == 1
    v = L.loglike(th, prob, L.PHASE_TIME, dd)
    assert v == pytest.approx(L.loglike(th, prob, L.PHASE, dd), abs=1e-9)


def test_time_shift_moves_the_overlap_peak(prob):
    # noise-free data: the injection itself, at t_c = 0 and at t_c = 7 delta
    t = L.time_grid(prob)
    delta = t[1] - t[0]
    th = prob.theta_inj.copy()
    th[6] = 40.0
    th[11] = 0.0
    th[12] = 0.0
    base = gwsynth.make_problem(8.0, 20.0, 512.0, psd_scale=1e-49)
    seqs = []
    for s in (0, 7):
        p = base
        inj = th.copy()
        inj[12] = s * delta
        p.data = L.strain(inj, p)
        a, _ = L.overlap_weights(th, p)
        seqs.append(np.abs(L.time_shifted_overlaps(a, p, t)))
    mid = t.size // 2
    assert int(np.argmax(seqs[0])) == mid
    assert int(np.argmax(seqs[1])) == mid + 7
    assert np.max(np.abs(seqs[1][7:] - seqs[0][:-7])) < 1e-9 * np.max(seqs[0])


def test_zero_signal_limit(prob):
    dd = L.data_inner(prob)
    th = prob.theta_inj.copy()
    th[6] = 1e30  # amplitude ~ 1e-30 of the injection's: Z and <h|h> vanish
    assert L.loglike(th, prob, L.PHASE_TIME, dd) == pytest.approx(-0.5 * dd, abs=1e-9)


def test_heterodyned_one_point_grid_is_phase_marginal(prob, monkeypatch):
    from oracle import heterodyne as H
    het = H.setup(prob, prob.theta_inj, 100)
    dd = 3.0
    th = prob.theta_inj.copy()
    th[12] = 0.0
    monkeypatch.setattr(L, "TIME_WINDOW", 0.0)
    assert H.loglike(th, prob, het, L.PHASE_TIME, dd) == pytest.approx(H.loglike(th, prob, het, L.PHASE, dd),
                                                                       abs=1e-9)


def test_heterodyned_time_marginal_approaches_full_band(prob, monkeypatch):
    # the binned likelihood converges to the full band as the bins shrink, at
    # every shift of the grid and hence for the marginal; slowly, because a
    # time shift winds the phase across each bin (the weakness of relative
    # binning for t_c that the paper reports): 385, 1.7 and 0.075 in log L at
    # 50, 400 and 2000 bins on this problem
    from oracle import heterodyne as H
    monkeypatch.setattr(L, "TIME_WINDOW", 0.01)
    th = prob.theta_inj.copy()
    th[0] *= 1 + 2e-5
    th[6] = 100.0
    dd = L.data_inner(prob)
    full = L.loglike(th, prob, L.PHASE_TIME, dd)
    errs = []
    for nb in (50, 400, 2000):
        het = H.setup(prob, prob.theta_inj, nb)
        errs.append(abs(H.loglike(th, prob, het, L.PHASE_TIME, dd) - full))
    assert errs[0] > errs[1] > errs[2] and errs[2] < 0.1
