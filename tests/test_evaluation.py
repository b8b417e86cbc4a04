"""Pins of the evaluation of the fused models (the surface RMS of the analytic
signed distance at raycast hits, and the equal-error comparison of a
prefiltered path with the plain one) on the CPU: the RMS of points at known
distances from the scene's surfaces, and the equal-error selection on
hand-made curves (first N reaching e*, the coverage gate, ties, never)."""
import numpy as np
import pytest

from paper_1708_00783_amd.prefilter import equal_error, rms_of
from synth import analytic_sdf, configs


def test_rms_of_points_at_known_distances():
    sc = configs.c2_scene(0)
    rng = np.random.default_rng(0)
    # points off the floor (z = 0) and the x = 0 wall of the room, away from every primitive
    d = rng.uniform(-0.004, 0.004, 200)
    floor = np.stack([rng.uniform(1.0, 1.02, 100), rng.uniform(3.3, 3.31, 100), np.zeros(100)], 1)
    wall = np.stack([np.zeros(100), rng.uniform(0.2, 0.21, 100), rng.uniform(2.5, 2.51, 100)], 1)
    pts = np.concatenate([floor + np.stack([0 * d[:100], 0 * d[:100], d[:100]], 1),
                          wall + np.stack([d[100:], 0 * d[100:], 0 * d[100:]], 1)])
    e = analytic_sdf(sc, pts)
    np.testing.assert_allclose(np.abs(e), np.abs(d), atol=1e-12)
    assert rms_of(e) == pytest.approx(np.sqrt(np.mean(d * d)), rel=1e-12)
    # the RMS over the union of two poses' hits, not the mean of their RMS
    a, b = np.full(10, 0.001), np.full(30, 0.003)
    assert rms_of(np.concatenate([a, b])) == pytest.approx(np.sqrt((10 * 1e-6 + 30 * 9e-6) / 40), rel=1e-12)
    assert np.isnan(rms_of([]))


def test_equal_error_selection():
    ns = [5, 10, 20, 300]
    raw = [4.0, 3.0, 2.0, 1.5]
    hraw = [900, 950, 990, 1000]
    traw = [0.001, 0.002, 0.004, 0.06]
    # reaches e* = 1.5 first at N = 10
    e, nd, r = equal_error(ns, raw, [1.6, 1.4, 1.2, 1.1], hraw, [900, 960, 990, 1000], traw,
                           [0.0015, 0.003, 0.006, 0.09])
    assert (e, nd) == (1.5, 10) and r == pytest.approx(0.06 / 0.003)
    # below e* at N = 5 but covering only 90% of the raw path's hits: N = 10
    e, nd, r = equal_error(ns, raw, [1.0, 1.4, 1.2, 1.1], hraw, [900, 960, 990, 1000], traw,
                           [0.0015, 0.003, 0.006, 0.09])
    assert nd == 10
    # a tie counts as reaching
    _, nd, _ = equal_error(ns, raw, [1.5, 1.4, 1.2, 1.1], hraw, [960, 960, 990, 1000], traw, traw)
    assert nd == 5
    # never reached
    e, nd, r = equal_error(ns, raw, [2.0, 1.9, 1.8, 1.6], hraw, hraw, traw, traw)
    assert e == 1.5 and nd is None and r is None
    # the plain path against itself reaches e* at the last N, ratio 1
    _, nd, r = equal_error(ns, raw, raw, hraw, hraw, traw, traw)
    assert nd == 300 and r == pytest.approx(1.0)
