"""Pins of the surfel-fusion oracle (Sec. 7.3) against closed forms: a static
camera over a plane makes one surfel per input pixel and then only raises
confidences (N alpha); a plane that moves by less than the depth gate is
averaged to the midpoint, by more it makes a second layer; an occluder in
front of known surfels makes new surfels that later frames find first; the
batch update equals the paper's update applied point by point in either
order; alpha and the normals of a tilted plane match their formulas; the
capacity is respected with a flag."""
import numpy as np

from oracle import surfel as S
from synth.scenes import look_at

K = np.array([30.0, 30.0, 19.5, 14.5], np.float32)
W, H = 40, 30
POSE = look_at((0.0, 0.0, 0.0), (0.0, 1.0, 0.0)).astype(np.float32)   # camera z = world +y


def _plane(D):
    return np.full((H, W), D, np.float32)


def test_static_plane_makes_one_surfel_per_pixel_and_raises_confidence():
    m = S.SurfelMap(10 ** 6)
    valid, P, N, alpha, _ = S.input_points(_plane(1.5), K, POSE)
    assert valid.sum() == (W - 1) * (H - 1)
    for k in range(4):
        corr = S.fuse(m, _plane(1.5), K, POSE)
        assert len(m.pos) == (W - 1) * (H - 1)
        if k == 0:
            assert np.all(corr[valid] == -1)
        else:
            # every input pixel finds the surfel made from it (raster order)
            assert np.array_equal(corr[valid], np.arange(valid.sum()))
    np.testing.assert_allclose(m.pos[:, :3], P[valid], atol=1e-6)
    np.testing.assert_allclose(m.nrm[:, 3], 4 * alpha[valid], rtol=1e-6)
    # the normal faces the camera: world -y
    np.testing.assert_allclose(m.nrm[:, :3], np.tile([0.0, -1.0, 0.0], (len(m.pos), 1)), atol=1e-6)
    assert np.all(m.time == 3)
    # radius: the circle around the pixel footprint
    np.testing.assert_allclose(m.pos[:, 3], 1.5 * np.sqrt(2) / 2 / 30.0, rtol=1e-6)


def test_moving_plane_is_averaged_within_the_gate_and_layered_beyond_it():
    m = S.SurfelMap(10 ** 6, delta_z=0.05)
    S.fuse(m, _plane(1.5), K, POSE)
    n0 = len(m.pos)
    _, P1, _, alpha, _ = S.input_points(_plane(1.5), K, POSE)
    valid, P2, _, _, _ = S.input_points(_plane(1.53), K, POSE)
    S.fuse(m, _plane(1.53), K, POSE)
    assert len(m.pos) == n0
    np.testing.assert_allclose(m.pos[:, :3], 0.5 * (P1[valid] + P2[valid]), atol=2e-6)
    np.testing.assert_allclose(m.nrm[:, 3], 2 * alpha[valid], rtol=1e-6)
    # a jump beyond the gate: a second layer, the first untouched
    before = m.pos.copy()
    S.fuse(m, _plane(1.65), K, POSE)
    assert len(m.pos) == 2 * n0
    assert np.array_equal(m.pos[:n0], before)


def test_occluder_makes_new_surfels_that_later_frames_find_first():
    m = S.SurfelMap(10 ** 6)
    S.fuse(m, _plane(2.0), K, POSE)
    n0 = len(m.pos)
    d = _plane(2.0)
    d[10:20, 12:25] = 1.0                     # a box face 1 m in front
    valid, _, _, _, _ = S.input_points(d, K, POSE)
    near = np.zeros((H, W), bool)
    near[10:20, 12:25] = True
    # far pixels whose forward differences reach the box have tilted normals:
    # they fail the normal gate against the far surfels
    rim = np.zeros((H, W), bool)
    rim[10:20, 11] = True
    rim[9, 12:25] = True
    corr = S.fuse(m, d, K, POSE)
    assert np.array_equal(corr == -1, valid & (near | rim))
    n1 = len(m.pos)
    assert n1 - n0 == int((valid & (near | rim)).sum())
    corr = S.fuse(m, d, K, POSE)              # the near surfels now win the index map there
    assert np.all(corr[valid & near] >= n0)
    assert np.all(corr[valid & ~near & ~rim] < n0) and np.all(corr[valid & ~near & ~rim] >= 0)
    # a rim pixel's new surfel ties in depth with the older far surfel, which
    # keeps the pixel (smaller index) and fails the gate again
    assert np.all(corr[rim] == -1) and len(m.pos) == n1 + int(rim.sum())


def test_batch_update_equals_the_sequential_update():
    """a surfel whose circle covers several pixels takes all their points: the
    result equals the paper's update applied one point after another"""
    m = S.SurfelMap(10 ** 6, delta_z=0.5, tau_n=-1.0)
    S.fuse(m, _plane(1.5), K, POSE)
    s = int(np.flatnonzero((m.pos[:, 0] > -0.01) & (m.pos[:, 0] < 0.03))[0])
    m.pos[:, 3] = 1e-6
    m.pos[s, 3] = 0.12                        # about 2.4 pixels at 1.5 m
    before = (m.pos[s].astype(np.float64).copy(), m.nrm[s].astype(np.float64).copy())
    rng = np.random.default_rng(0)
    d = (_plane(1.5) + rng.uniform(-0.01, 0.01, (H, W))).astype(np.float32)
    corr = S.fuse(m, d, K, POSE)
    pix = np.argwhere(corr == s)
    assert len(pix) >= 9
    _, P, N, alpha, _ = S.input_points(d, K, POSE)
    for order in (pix, pix[::-1]):
        v, n, c = before[0][:3].copy(), before[1][:3].copy(), before[1][3]
        for y, x in order:
            a = float(alpha[y, x])
            v = (c * v + a * P[y, x]) / (c + a)
            n = (c * n + a * N[y, x]) / (c + a)
            c = c + a
        np.testing.assert_allclose(m.pos[s, :3], v, rtol=1e-6)
        np.testing.assert_allclose(m.nrm[s, :3], n, rtol=1e-6, atol=1e-7)
        np.testing.assert_allclose(m.nrm[s, 3], c, rtol=1e-6)


def test_alpha_and_tilted_plane_normals():
    valid, P, N, alpha, _ = S.input_points(_plane(1.0), K, POSE)
    cx, cy = K[2], K[3]
    ys, xs = np.mgrid[0:H, 0:W]
    gam = np.hypot(xs - cx, ys - cy) / np.hypot(cx, cy)
    np.testing.assert_allclose(alpha, np.exp(-gam ** 2 / (2 * 0.36)), rtol=1e-6)
    # a plane tilted about the camera x axis: camera z = 1 + 0.4 y_cam
    d = np.zeros((H, W), np.float32)
    for y in range(H):
        t = (y - cy) / K[1]
        d[y, :] = 1.0 / (1.0 - 0.4 * t)
    valid, P, N, _, _ = S.input_points(d, K, POSE)
    n_cam = np.array([0.0, 0.4, -1.0]) / np.linalg.norm([0.0, 0.4, -1.0])    # towards the camera
    n_world = POSE[:3, :3].T.astype(np.float64) @ n_cam
    assert np.abs(N[valid] - n_world).max() < 1e-4


def test_capacity_is_respected():
    m = S.SurfelMap(500)
    S.fuse(m, _plane(1.5), K, POSE)
    assert len(m.pos) == 500 and m.overflow
