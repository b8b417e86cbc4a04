"""Pins of the depth-tracker oracle (Sec. 4.1.1, ITMDepthTracker) against
what the geometry fixes: brute-force pyramid levels, the pixel-centre
mapping of the level intrinsics, the Jacobian against finite differences of
the point-to-plane residual, the normal-equation step against a generic
least-squares solve, a closed-form translation recovered on three planes,
and a known synthetic trajectory recovered frame by frame."""
import numpy as np

from oracle import track as TR
from pose_helpers import pose_error
from synth import configs, scenes
from synth.scenes import Intrinsics, Scene, look_at, render_depth

K_HALF = Intrinsics(262.5, 262.5, 159.75, 119.75, 320, 240)


def test_pyramid_levels_by_brute_force():
    rng = np.random.default_rng(3)
    d = rng.uniform(0.5, 3.0, (19, 27)).astype(np.float32)
    d[rng.random(d.shape) < 0.35] = 0.0
    d[0:4, 0:4] = 0.0                                   # a block with no valid depth
    p = TR.pyramid(d, 4)
    assert [x.shape for x in p] == [(19, 27), (9, 13), (4, 6), (2, 3)]
    for l in range(1, 4):
        src, dst = p[l - 1], p[l]
        for y in range(dst.shape[0]):
            for x in range(dst.shape[1]):
                vals = [float(src[2 * y + j, 2 * x + i]) for j in (0, 1) for i in (0, 1)
                        if src[2 * y + j, 2 * x + i] > 0]
                want = sum(vals) / len(vals) if vals else 0.0
                assert abs(float(dst[y, x]) - want) <= 4e-7 * want, (l, y, x)
    assert p[1][0, 0] == 0.0 and p[1][1, 1] == 0.0


def test_level_intrinsics_map_pixel_centres():
    """a coarse pixel coordinate is the mean of the fine pixel centres it
    covers: u_l = (u_0 + 0.5) / 2^l - 0.5 for every projected point"""
    K = configs.KINECT_INTR.as_array()
    rng = np.random.default_rng(4)
    X = rng.uniform([-1, -1, 0.5], [1, 1, 4], (100, 3))
    u0 = K[0] * X[:, 0] / X[:, 2] + K[2]
    v0 = K[1] * X[:, 1] / X[:, 2] + K[3]
    for l in (1, 2, 3):
        Kl = TR.level_intrinsics(K, l).astype(np.float64)
        ul = Kl[0] * X[:, 0] / X[:, 2] + Kl[2]
        vl = Kl[1] * X[:, 1] / X[:, 2] + Kl[3]
        np.testing.assert_allclose(ul, (u0 + 0.5) / 2 ** l - 0.5, atol=1e-4)
        np.testing.assert_allclose(vl, (v0 + 0.5) / 2 ** l - 0.5, atol=1e-4)


def _live_and_reference(shift=(0.012, -0.008, 0.01), yaw_deg=1.0):
    sc = configs.c2_scene(0)
    P0 = configs.c2_poses(300)[0]
    R0, t0 = TR.invert_pose(P0)
    c, s = np.cos(np.radians(yaw_deg)), np.sin(np.radians(yaw_deg))
    Rz = np.array([[c, -s, 0], [s, c, 0], [0, 0, 1.0]])
    R1, t1 = Rz @ R0, t0 + np.array(shift)
    P1 = np.eye(4)
    P1[:3, :3] = R1.T
    P1[:3, 3] = -(R1.T @ t1)
    V, N = scenes.render_points_normals(sc, P0, K_HALF)
    d = render_depth(sc, P1, K_HALF).astype(np.float32)
    return sc, P0.astype(np.float32), P1, V, N, d


def test_jacobian_matches_finite_differences():
    """each Jacobian column is the derivative of the residual of the fixed
    pairs under the world-frame increment Exp(omega) q + delta_t"""
    _, P0, _, V, N, d = _live_and_reference()
    R, t = TR.invert_pose(P0)
    K = K_HALF.as_array()
    mask, J, r, q, v, n = TR.pair_terms(d, K, V, N, K, P0, R.astype(np.float32), t.astype(np.float32), 0.2)
    assert mask.sum() == len(r) > 10000
    q64, v64, n64 = q.astype(np.float64), v.astype(np.float64), n.astype(np.float64)

    def resid(xi):
        qq = q64 @ TR.exp_rotation(xi[:3]).T + xi[3:]
        return np.einsum("ij,ij->i", qq - v64, n64)

    np.testing.assert_allclose(resid(np.zeros(6)), r, atol=2e-6)
    eps = 1e-6
    for k in range(6):
        e = np.zeros(6)
        e[k] = eps
        fd = (resid(e) - resid(-e)) / (2 * eps)
        np.testing.assert_allclose(J[:, k], fd, atol=1e-5 * max(1.0, np.abs(fd).max()))


def test_step_is_the_least_squares_solution_of_the_linearised_pairs():
    _, P0, _, V, N, d = _live_and_reference()
    R, t = TR.invert_pose(P0)
    K = K_HALF.as_array()
    _, J, r, _, _, _ = TR.pair_terms(d, K, V, N, K, P0, R.astype(np.float32), t.astype(np.float32), 0.2)
    A, g, rr, n = TR.normal_equations(J, r)
    xi = TR.solve_step(A, g)
    xi_ls = np.linalg.lstsq(J.astype(np.float64), -r.astype(np.float64), rcond=None)[0]
    np.testing.assert_allclose(xi, xi_ls, rtol=1e-7, atol=1e-12)
    assert n == len(r) and abs(rr - float(np.sum(r.astype(np.float64) ** 2))) <= 1e-9 * rr
    # a lone plane leaves the system singular: no step
    J1 = np.tile(np.array([[0, 0, 0, 0, 0, 1]], np.float32), (50, 1))
    assert TR.solve_step(*TR.normal_equations(J1, np.ones(50, np.float32))[:2]) is None


def test_pure_translation_on_three_planes():
    """two walls and the floor of an empty room: a translated camera is
    recovered (the residual is exactly linear in a translation, so the fixed
    point is the true pose)"""
    sc = Scene(rooms=[((0.0, 0.0, 0.0), (4.0, 4.0, 3.0))])
    eye0, target0 = np.array([2.5, 2.5, 1.6]), np.array([4.0, 4.0, 0.3])
    P0 = look_at(eye0, target0)
    delta = np.array([0.012, -0.008, 0.010])
    P1 = look_at(eye0 + delta, target0 + delta)
    K = configs.KINECT_INTR
    V, N = scenes.render_points_normals(sc, P0, K)
    d = render_depth(sc, P1, K).astype(np.float32)
    M, info = TR.track(d, K.as_array(), V, N, K.as_array(), P0.astype(np.float32), P0.astype(np.float32),
                       [6], [0.1])
    et, er = pose_error(M, P1)
    assert et < 2e-5 and er < 0.02, (et, er)
    assert info[0]["iterations"] == 6 and info[0]["pairs"] > 0.95 * d.size
    # and with the hierarchy
    M, info = TR.track(d, K.as_array(), V, N, K.as_array(), P0.astype(np.float32), P0.astype(np.float32),
                       [3, 3, 5], [0.1, 0.2, 0.3])
    et, er = pose_error(M, P1)
    assert et < 2e-5 and er < 0.02, (et, er)


def test_known_trajectory_is_recovered():
    """frame-to-model tracking along the full-frame room trajectory against
    an exact model of the room (analytic point and normal maps rendered at
    the previous estimate): every frame within 0.05 mm and 0.005 degrees,
    while frames move ~16 mm and ~1.4 degrees apart"""
    sc = configs.c2_scene(0)
    poses = configs.c2_poses(300)
    K = K_HALF
    est = poses[0].astype(np.float32)
    for k in range(1, 5):
        V, N = scenes.render_points_normals(sc, est, K)
        d = render_depth(sc, poses[k], K).astype(np.float32)
        M, info = TR.track(d, K.as_array(), V, N, K.as_array(), est, est, [4, 5, 10], [0.1, 0.2, 0.3])
        et, er = pose_error(M, poses[k])
        mt, mr = pose_error(poses[k - 1], poses[k])
        assert mt > 0.01 and mr > 1.0
        assert et < 5e-5 and er < 5e-3, (k, et, er)
        assert all(i["iterations"] > 0 for i in info)
        est = M


def test_noisy_depth_stays_close():
    """Kinect-like noise and millimetre quantisation on the live frame"""
    from synth.scenes import kinect_noise, to_mm_u16
    sc, P0, P1, V, N, d = _live_and_reference()
    z = render_depth(sc, P1, K_HALF)
    dn = (to_mm_u16(kinect_noise(z, np.random.default_rng(7))).astype(np.float32) / np.float32(1000.0))
    M, _ = TR.track(dn.astype(np.float32), K_HALF.as_array(), V, N, K_HALF.as_array(), P0, P0,
                    [4, 5, 10], [0.1, 0.2, 0.3])
    et, er = pose_error(M, P1)
    assert et < 2e-3 and er < 0.1, (et, er)
