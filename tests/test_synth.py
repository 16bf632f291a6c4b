"""Checks of the seeded workload generator (no likelihood arithmetic)."""
import numpy as np

import gwsynth


def test_grid_counts_match_paper():
    # Sec. III.D: ~2.6e5 bins per detector for 128 s over 20-2048 Hz, and
    # ~7.8e5 operations for the three-detector full-resolution sum.
    g2 = gwsynth.freq_grid(128.0, 20.0, 2048.0)
    assert (g2.k0, g2.n_freq) == (2560, 259585)
    assert abs(g2.n_freq - 2.6e5) / 2.6e5 < 0.01
    assert abs(3 * g2.n_freq - 7.8e5) / 7.8e5 < 0.01
    g1 = gwsynth.freq_grid(8.0, 20.0, 512.0)
    assert (g1.k0, g1.n_freq) == (160, 3937)
    f = g1.freqs
    assert f[0] == 20.0 and f[-1] == 512.0


def test_psd_fit_values():
    # At x = 1: 1 - 5 + 111 * 0.5 / 1.5 = 33.
    assert np.isclose(gwsynth.psd_fit(np.array([215.0]), 1.0)[0], 33.0, rtol=1e-14)
    f = gwsynth.freq_grid(128.0, 20.0, 2048.0).freqs
    s = gwsynth.psd_fit(f, 1e-46)
    assert np.all(s > 0) and np.all(np.isfinite(s))


def test_detectors_geometry():
    pos, tens = gwsynth.detectors(1, 3)
    assert np.allclose(np.linalg.norm(pos, axis=1), gwsynth.workload.EARTH_RADIUS_M)
    for i in range(3):
        d = tens[i]
        assert np.allclose(d, d.T)
        assert abs(np.trace(d)) < 1e-15
        ev = np.sort(np.linalg.eigvalsh(d))
        assert np.allclose(ev, [-0.5, 0.0, 0.5])
        # arms in the local tangent plane: the radial direction is a null vector
        n = pos[i] / np.linalg.norm(pos[i])
        assert np.linalg.norm(d @ n) < 1e-14


def test_noise_variance():
    g = gwsynth.freq_grid(8.0, 20.0, 512.0)
    s = gwsynth.psd_fit(g.freqs)
    n = gwsynth.gaussian_noise(3, np.tile(s, (3, 1)), g.df)
    r = (np.abs(n) ** 2) * 4 * g.df / s
    # E|n|^2 4 df / S = 2 per bin
    assert abs(r.mean() - 2.0) < 0.05


def test_prior_draws_ranges():
    th = gwsynth.prior_draws(4, 4096)
    assert th.shape == (4096, 13)
    assert np.all((th[:, 0] >= 1.1) & (th[:, 0] <= 1.4))
    assert np.all((th[:, 1] >= 0.5) & (th[:, 1] <= 1.0))
    assert np.all(np.abs(th[:, 2:4]) <= 0.05)
    assert np.all((th[:, 7] >= 0) & (th[:, 7] <= np.pi))
    assert np.all(np.abs(th[:, 9]) <= np.pi / 2)
    assert np.all(np.abs(th[:, 12]) <= 0.1)
    # isotropic inclination: cos(iota) uniform
    assert abs(np.mean(np.cos(th[:, 7]))) < 0.05


def test_uneven_split():
    off = gwsynth.uneven_split(5, 65536)
    sizes = np.diff(off)
    assert off[0] == 0 and off[-1] == 65536
    assert np.all(sizes >= 100)
    assert np.all(sizes[:-1] <= 8000)
    assert len(sizes) > 5


def test_distance_grid_normalised():
    d, lw = gwsynth.distance_grid(1000)
    assert d[0] == 10.0 and d[-1] == 200.0
    assert abs(np.exp(lw).sum() - 1.0) < 1e-12
