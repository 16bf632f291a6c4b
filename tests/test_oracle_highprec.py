"""High-precision brute force of the oracle's reduction and marginal stages.

On a 13-bin, 3-detector grid, every sum of the likelihood is redone in
mpmath at 50 significant digits from the same FP64 inputs (data, PSD and the
oracle's FP64 template values, each exactly representable): the plain
log-likelihood as -1/2 sum <d - h|d - h>, the phase marginal as
-1/2 dd - 1/2 hh + ln I0(|Z|) with mpmath's own Bessel function, and the
distance marginal as the log of the weighted grid sum of exp terms.  This
bounds the oracle's FP64 rounding in these stages and pins its ln I0,
log-sum-exp and marginal arithmetic to an independent implementation.  (The
waveform itself is pinned by the closed forms of test_oracle_waveform.)
"""
import mpmath
import numpy as np

import gwsynth
from oracle import likelihood as L

mpmath.mp.dps = 50


def tiny_problem():
    prob = gwsynth.make_problem(8.0, 20.0, 21.5, psd_scale=1e-49, n_dist=200)
    assert prob.n_freq == 13
    th = gwsynth.prior_draws(gwsynth.SEEDS["injection"], 1)[0]
    th[6] = 60.0
    prob.data = prob.data + L.strain(th, prob)
    return prob, th


def mp_inner(a, b, psd, df):
    s = mpmath.mpf(0)
    for x, y, p in zip(a, b, psd):
        s += (mpmath.mpc(complex(x)).conjugate() * mpmath.mpc(complex(y)) / mpmath.mpf(float(p))).real
    return 4 * mpmath.mpf(df) * s


def test_plain_loglike_high_precision():
    prob, th0 = tiny_problem()
    for s in range(4):
        th = gwsynth.near_posterior(50 + s, th0, 1, scale=0.5)[0]
        h = L.strain(th, prob)
        r = prob.data - h
        ref = -sum(mp_inner(r[i], r[i], prob.psd[i], prob.df) for i in range(3)) / 2
        got = L.loglike(th, prob, L.PLAIN)
        assert abs(mpmath.mpf(got) - ref) < 1e-12 * max(1.0, abs(float(ref)))


def test_phase_and_distance_marginals_high_precision():
    prob, th0 = tiny_problem()
    dd = sum(mp_inner(prob.data[i], prob.data[i], prob.psd[i], prob.df) for i in range(3))
    for s in range(4):
        th = gwsynth.near_posterior(60 + s, th0, 1, scale=0.5)[0]
        # phase marginal at the given distance
        t = th.copy()
        t[11] = 0.0
        h = L.strain(t, prob)
        z = mpmath.mpc(0)
        hh = mpmath.mpf(0)
        for i in range(3):
            for k in range(prob.n_freq):
                z += 4 * mpmath.mpf(prob.df) * mpmath.mpc(complex(prob.data[i][k])).conjugate() * \
                    mpmath.mpc(complex(h[i][k])) / mpmath.mpf(float(prob.psd[i][k]))
            hh += mp_inner(h[i], h[i], prob.psd[i], prob.df)
        ref = -dd / 2 - hh / 2 + mpmath.log(mpmath.besseli(0, abs(z)))
        got = L.loglike(th, prob, L.PHASE)
        assert abs(mpmath.mpf(got) - ref) < 1e-12 * max(1.0, abs(float(ref)))
        # distance marginal: Z1, hh1 at d_L = 1 Mpc, grid sum of w_j exp(-hh1/(2 d^2)) I0(|Z1| / d)
        t[6] = 1.0
        h1 = L.strain(t, prob)
        z1 = mpmath.mpc(0)
        hh1 = mpmath.mpf(0)
        for i in range(3):
            for k in range(prob.n_freq):
                z1 += 4 * mpmath.mpf(prob.df) * mpmath.mpc(complex(prob.data[i][k])).conjugate() * \
                    mpmath.mpc(complex(h1[i][k])) / mpmath.mpf(float(prob.psd[i][k]))
            hh1 += mp_inner(h1[i], h1[i], prob.psd[i], prob.df)
        acc = mpmath.mpf(0)
        for d, lw in zip(prob.dist_grid, prob.dist_logw):
            d = mpmath.mpf(float(d))
            acc += mpmath.exp(mpmath.mpf(float(lw)) - hh1 / (2 * d * d)) * mpmath.besseli(0, abs(z1) / d)
        ref = -dd / 2 + mpmath.log(acc)
        got = L.loglike(th, prob, L.PHASE_DIST)
        assert abs(mpmath.mpf(got) - ref) < 1e-12 * max(1.0, abs(float(ref))), (float(ref), got)
