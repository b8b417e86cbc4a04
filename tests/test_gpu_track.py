"""GPU parity of the depth tracker (Sec. 4.1.1) against the oracle, through
the C ABI.  Per level and pose, the pair count is exact (both sides take the
pixel, bounds and distance decisions in the same float32 arithmetic) and the
float64 sums agree to 1e-9 relative (only their summation order differs).  A
whole tracking call matches the oracle's pose within 1e-5 m and 1e-4 degrees
with the same iteration counts; u16 and f32 inputs give identical results; a
call is bit-reproducible; empty and degenerate inputs stop without an update.
The loop closes on the GPU: frames fused at tracked poses, each tracked
against the raycast of the model fused so far."""
import numpy as np
import pytest

from gpu_helpers import to_device
from pose_helpers import pose_error
from synth import Intrinsics, configs, render_depth, scenes

pytestmark = pytest.mark.gpu

K2 = configs.KINECT_INTR


def _log(*a):
    print(*a, flush=True)


def _ref_maps(seed, pose, K):
    V, N = scenes.render_points_normals(configs.c2_scene(seed), pose, K)
    return V, N


def _oracle_depth(mm):
    return (mm.astype(np.float32) / np.float32(1000.0)).astype(np.float32)


def _perturbed(P, shift=(0.01, -0.006, 0.008), yaw_deg=0.8):
    """world->camera P with the camera moved by `shift` and turned about world z"""
    P = np.asarray(P, np.float64)
    R, t = P[:3, :3].T, -(P[:3, :3].T @ P[:3, 3])
    c, s = np.cos(np.radians(yaw_deg)), np.sin(np.radians(yaw_deg))
    Rz = np.array([[c, -s, 0], [s, c, 0], [0, 0, 1.0]])
    R1, t1 = Rz @ R, t + np.asarray(shift)
    Q = np.eye(4)
    Q[:3, :3] = R1.T
    Q[:3, 3] = -(R1.T @ t1)
    return Q.astype(np.float32)


def _compare_sums(res, info, level, tag):
    assert res["pairs"][level] == info[level]["pairs"], (tag, res["pairs"][level], info[level]["pairs"])
    o = np.concatenate([info[level]["A"][np.triu_indices(6)], info[level]["g"], [info[level]["rr"]]])
    g = res["sums"][level]
    scale = np.abs(o[:21]).max()
    np.testing.assert_allclose(g[:21], o[:21], rtol=1e-9, atol=1e-12 * scale, err_msg=tag)
    np.testing.assert_allclose(g[21:27], o[21:27], rtol=1e-9, atol=1e-9 * np.abs(o[21:27]).max(), err_msg=tag)
    np.testing.assert_allclose(g[27], o[27], rtol=1e-9, err_msg=tag)


def test_level_sums_match_oracle():
    """one system per level at the initial pose: pairs exact, sums 1e-9"""
    import paper_1708_00783_amd as T
    from oracle import track as TR
    P = configs.c2_poses(300)
    V, N = _ref_maps(0, P[0], K2)
    mm = configs.c2_frame(1)
    dV, dN, dd = to_device(V), to_device(N), to_device(mm)
    trk = T.Tracker(K2.width, K2.height, 3)
    for init in (P[0], _perturbed(P[0])):
        for level in range(3):
            iters = [0, 0, 0]
            iters[level] = 1
            taus = [0.1, 0.2, 0.3]
            res = trk.track(dd, K2, dV, dN, K2, P[0], init, T.make_track_params(iters, taus))
            _, info = TR.track(_oracle_depth(mm), K2.as_array(), V, N, K2.as_array(), P[0], init, iters, taus)
            _compare_sums(res, info, level, f"level {level}")
            assert res["iterations"][:len(info)] == [i["iterations"] for i in info]
            _log(f"level {level}: {res['pairs'][level]} pairs")


def test_tracking_matches_oracle():
    import paper_1708_00783_amd as T
    from oracle import track as TR
    P = configs.c2_poses(300)
    V, N = _ref_maps(0, P[0], K2)
    mm = configs.c2_frame(1)
    trk = T.Tracker(K2.width, K2.height, 3)
    iters, taus = [4, 5, 10], [0.1, 0.2, 0.3]
    res = trk.track(to_device(mm), K2, to_device(V), to_device(N), K2, P[0], P[0], T.make_track_params(iters, taus))
    M, info = TR.track(_oracle_depth(mm), K2.as_array(), V, N, K2.as_array(), P[0], P[0], iters, taus)
    et, er = pose_error(res["pose_w2c"], M)
    assert et < 1e-5 and er < 1e-4, (et, er)
    assert res["iterations"][:len(info)] == [i["iterations"] for i in info] == iters
    for l in range(3):
        assert abs(res["pairs"][l] - info[l]["pairs"]) <= 1e-3 * info[l]["pairs"]
    gt_t, gt_r = pose_error(res["pose_w2c"], P[1])
    _log(f"tracked frame 1: gpu vs oracle {et:.2e} m {er:.2e} deg; vs truth {gt_t * 1e3:.3f} mm {gt_r:.4f} deg")
    assert gt_t < 3e-3 and gt_r < 0.1


def test_ragged_sizes_and_other_reference_resolution():
    """a 333x251 f32 live image against 200x150 reference maps of another
    view (odd pyramid sizes 166x125, 83x62), four levels"""
    import paper_1708_00783_amd as T
    from oracle import track as TR
    P = configs.c2_poses(300)
    Kl = Intrinsics(270.0, 268.0, 166.3, 124.8, 333, 251)
    Kr = Intrinsics(160.0, 160.0, 99.5, 74.5, 200, 150)
    V, N = _ref_maps(0, P[3], Kr)
    d = render_depth(configs.c2_scene(0), P[5], Kl).astype(np.float32)
    d[100:140, 50:90] = 0.0
    trk = T.Tracker(Kl.width, Kl.height, 4)
    iters, taus = [3, 3, 4, 6], [0.08, 0.15, 0.25, 0.4]
    dd, dV, dN = to_device(d), to_device(V), to_device(N)
    for level in range(4):
        it = [0, 0, 0, 0]
        it[level] = 1
        res = trk.track(dd, Kl, dV, dN, Kr, P[3], P[3], T.make_track_params(it, taus))
        _, info = TR.track(d, Kl.as_array(), V, N, Kr.as_array(), P[3], P[3], it, taus)
        _compare_sums(res, info, level, f"ragged level {level}")
    res = trk.track(dd, Kl, dV, dN, Kr, P[3], P[3], T.make_track_params(iters, taus))
    M, info = TR.track(d, Kl.as_array(), V, N, Kr.as_array(), P[3], P[3], iters, taus)
    et, er = pose_error(res["pose_w2c"], M)
    assert et < 1e-5 and er < 1e-4, (et, er)
    assert res["iterations"][:len(info)] == [i["iterations"] for i in info]


def test_u16_and_f32_inputs_agree_and_calls_repeat():
    import torch
    import paper_1708_00783_amd as T
    P = configs.c2_poses(300)
    V, N = _ref_maps(0, P[0], K2)
    mm = configs.c2_frame(1)
    trk = T.Tracker(K2.width, K2.height, 3)
    dV, dN = to_device(V), to_device(N)
    prm = T.make_track_params()
    trk.track_async(to_device(mm), K2, dV, dN, K2, P[0], P[0], prm)
    a = trk.result.clone()
    trk.track_async(to_device(_oracle_depth(mm)), K2, dV, dN, K2, P[0], P[0], prm)
    b = trk.result.clone()
    trk.track_async(to_device(mm), K2, dV, dN, K2, P[0], P[0], prm)
    c = trk.result.clone()
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(a, c)


def test_empty_and_degenerate_inputs():
    import paper_1708_00783_amd as T
    P = configs.c2_poses(300)
    V, N = _ref_maps(0, P[0], K2)
    trk = T.Tracker(K2.width, K2.height, 3)
    zero = np.zeros((K2.height, K2.width), np.uint16)
    res = trk.track(to_device(zero), K2, to_device(V), to_device(N), K2, P[0], P[0], T.make_track_params())
    assert res["pairs"] == [0, 0, 0, 0] and res["iterations"] == [0, 0, 0, 0] and res["status"] == 0b111
    np.testing.assert_allclose(res["pose_w2c"], P[0], atol=1e-6)
    # one plane: the system is singular at every level
    from synth.scenes import Scene, look_at
    sc = Scene(floors=[0.0])
    Pp = look_at((0.0, 0.0, 1.5), (0.0, 0.01, 0.0)).astype(np.float32)
    Vp, Np_ = scenes.render_points_normals(sc, Pp, K2)
    dp = render_depth(sc, Pp, K2).astype(np.float32)
    res = trk.track(to_device(dp), K2, to_device(Vp), to_device(Np_), K2, Pp, Pp, T.make_track_params())
    assert res["status"] == 0b111 and res["iterations"] == [0, 0, 0, 0] and res["pairs"][0] > 100000
    # argument errors are returned before anything is launched
    with pytest.raises(T.TsdfError):
        trk.track(to_device(dp), K2, to_device(Vp), to_device(Np_), K2, Pp, Pp,
                  T.make_track_params((4, 5, 10), (0.1, -0.2, 0.3)))


def test_early_stop_matches_oracle():
    import paper_1708_00783_amd as T
    from oracle import track as TR
    P = configs.c2_poses(300)
    V, N = _ref_maps(0, P[0], K2)
    d = render_depth(configs.c2_scene(0), P[1], K2).astype(np.float32)
    trk = T.Tracker(K2.width, K2.height, 3)
    iters, taus = [20, 20, 20], [0.1, 0.2, 0.3]
    res = trk.track(to_device(d), K2, to_device(V), to_device(N), K2, P[0], P[0],
                    T.make_track_params(iters, taus, min_update=1e-5))
    M, info = TR.track(d, K2.as_array(), V, N, K2.as_array(), P[0], P[0], iters, taus, min_update=1e-5)
    assert res["iterations"][:len(info)] == [i["iterations"] for i in info]
    assert max(res["iterations"][:3]) < 20
    et, er = pose_error(res["pose_w2c"], M)
    assert et < 1e-5 and er < 1e-4
    _log(f"early stop: iterations {res['iterations'][:3]}")


def test_frame_to_model_loop():
    """fuse at tracked poses, track each new frame against the model's
    raycast at the previous estimate; every call against the oracle run on
    the same maps; the trajectory stays near the truth"""
    import torch
    import paper_1708_00783_amd as T
    from oracle import track as TR
    n = 16
    P = configs.c2_poses(300)
    frames = np.stack([configs.c2_frame(k) for k in range(n)])
    d = to_device(frames)
    vol = T.Volume(configs.C2_VOLUME, K2.width, K2.height)
    trk = T.Tracker(K2.width, K2.height, 3)
    pts = torch.empty((K2.height, K2.width, 4), dtype=torch.float32, device="cuda")
    nrm = torch.empty_like(pts)
    iters, taus = [4, 5, 10], [0.1, 0.2, 0.3]
    prm = T.make_track_params(iters, taus)
    est = P[0].astype(np.float32)
    vol.frame(d[0], K2, est, pts, nrm)
    worst = (0.0, 0.0)
    for k in range(1, n):
        res = trk.track(d[k], K2, pts, nrm, K2, est, est, prm)
        V, N = pts.cpu().numpy(), nrm.cpu().numpy()
        M, _ = TR.track(_oracle_depth(frames[k]), K2.as_array(), V, N, K2.as_array(), est, est, iters, taus)
        et, er = pose_error(res["pose_w2c"], M)
        assert et < 1e-5 and er < 1e-4, (k, et, er)
        est = res["pose_w2c"]
        vol.frame(d[k], K2, est, pts, nrm)
        gt = pose_error(est, P[k])
        worst = max(worst, gt)
    _log(f"loop of {n} frames: worst error vs truth {worst[0] * 1e3:.2f} mm, {worst[1]:.3f} deg")
    assert worst[0] < 0.01 and worst[1] < 0.5
