"""Pins of the bilateral-filter oracle against what the definition fixes in
its limits: a constant image and a linear ramp pass unchanged (symmetric
weights, interior pixels), an infinite range sigma is a normalised Gaussian
blur (scipy), a vanishing range sigma is the identity, a depth step is kept
on both sides, invalid pixels neither contribute nor are filled."""
import numpy as np
from scipy import ndimage

from oracle.bilateral import bilateral


def test_constant_and_linear_ramp_pass_unchanged():
    yy, xx = np.mgrid[0:40, 0:50].astype(np.float64)
    const = np.full((40, 50), 2.5)
    assert np.allclose(bilateral(const, 3, 2.0, 0.02), const, rtol=0, atol=1e-12)
    ramp = 1.0 + 0.01 * xx - 0.004 * yy
    out = bilateral(ramp, 3, 2.0, 0.02)
    np.testing.assert_allclose(out[3:-3, 3:-3], ramp[3:-3, 3:-3], rtol=0, atol=1e-12)
    # at the border the window is one-sided: the ramp is not preserved there
    assert abs(out[0, 25] - ramp[0, 25]) > 1e-4


def test_infinite_range_sigma_is_a_gaussian_blur():
    rng = np.random.default_rng(0)
    d = rng.uniform(1.0, 3.0, (30, 33))
    r, ss = 2, 1.5
    k = np.exp(-(np.arange(-r, r + 1)[:, None] ** 2 + np.arange(-r, r + 1)[None, :] ** 2) / (2 * ss * ss))
    want = ndimage.correlate(d, k, mode="constant") / ndimage.correlate(np.ones_like(d), k, mode="constant")
    np.testing.assert_allclose(bilateral(d, r, ss, 1e9), want, rtol=1e-12)


def test_vanishing_range_sigma_is_the_identity():
    rng = np.random.default_rng(1)
    d = rng.uniform(1.0, 3.0, (20, 20))
    np.testing.assert_allclose(bilateral(d, 2, 2.0, 1e-6), d, rtol=0, atol=1e-15)


def test_step_edge_is_kept_and_holes_stay():
    d = np.full((24, 30), 1.0)
    d[:, 15:] = 2.0
    d[5:8, 5:8] = 0.0
    out = bilateral(d, 3, 3.0, 0.02)
    assert np.all(out[:, :15][d[:, :15] > 0] == 1.0) and np.all(out[:, 15:] == 2.0)
    assert np.all(out[5:8, 5:8] == 0.0)
    # holes neither contribute nor get filled: a constant surface with holes stays constant
    rng = np.random.default_rng(2)
    d2 = np.full((25, 31), 1.5)
    d2[rng.random(d2.shape) < 0.3] = 0.0
    out2 = bilateral(d2, 2, 1.5, 0.05)
    assert np.abs(out2[d2 > 0] - 1.5).max() < 1e-14 and np.all(out2[d2 == 0] == 0.0)
