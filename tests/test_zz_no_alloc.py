"""The tracker entry point that allocates nothing (tf_track_noalloc) gives
the result of tf_track bit for bit, on two calls in a row with the second on
a smaller input, and refuses an image whose workspace exceeds its fixed
array."""
import ctypes

import numpy as np
import pytest

from gpu_helpers import to_device
from synth import Intrinsics, configs, render_depth, scenes

pytestmark = pytest.mark.gpu


def _case_full():
    P = configs.c2_poses(300)
    K = configs.KINECT_INTR
    V, N = scenes.render_points_normals(configs.c2_scene(0), P[0], K)
    return K, to_device(configs.c2_frame(1)), to_device(V), to_device(N), K, P[0], P[0], ((4, 5, 10), (0.1, 0.2, 0.3))


def _case_small():
    P = configs.c2_poses(300)
    Kl = Intrinsics(270.0, 268.0, 166.3, 124.8, 333, 251)
    Kr = Intrinsics(160.0, 160.0, 99.5, 74.5, 200, 150)
    V, N = scenes.render_points_normals(configs.c2_scene(0), P[3], Kr)
    d = render_depth(configs.c2_scene(0), P[5], Kl).astype(np.float32)
    return Kl, to_device(d), to_device(V), to_device(N), Kr, P[3], P[3], ((3, 3, 4, 6), (0.08, 0.15, 0.25, 0.4))


def test_noalloc_matches_tf_track_on_two_calls():
    import torch
    import paper_1708_00783_amd as T
    out = torch.empty(ctypes.sizeof(T.tf_track_result), dtype=torch.uint8, device="cuda")
    for case in (_case_full(), _case_small()):
        K, d, V, N, Kr, Pr, Pi, (it, tau) = case
        prm = T.make_track_params(it, tau)
        trk = T.Tracker(K.width, K.height, len(it))
        ref = trk.track(d, K, V, N, Kr, Pr, Pi, prm)
        out.fill_(0xAB)
        T.tf_track_noalloc(d, K, V, N, Kr, Pr, Pi, prm, out)
        got = T.parse_track_result(out.cpu().numpy())
        assert np.array_equal(got["pose_w2c"], ref["pose_w2c"])
        assert got["iterations"] == ref["iterations"] and got["pairs"] == ref["pairs"]
        assert got["status"] == ref["status"] and np.array_equal(got["sums"], ref["sums"])
        assert torch.equal(out, trk.result)
        print(f"noalloc {K.width}x{K.height}: pairs {got['pairs']}", flush=True)


def test_noalloc_refuses_images_beyond_its_array():
    import torch
    import paper_1708_00783_amd as T
    K = Intrinsics(1000.0, 1000.0, 959.5, 539.5, 1920, 1080)
    assert T.lib().tf_track_workspace_bytes(1920, 1080, 4) > T.TF_TRACK_NOALLOC_MAX_BYTES
    d = torch.zeros((1080, 1920), dtype=torch.float32, device="cuda")
    V = torch.zeros((1080, 1920, 4), dtype=torch.float32, device="cuda")
    out = torch.empty(ctypes.sizeof(T.tf_track_result), dtype=torch.uint8, device="cuda")
    P = np.eye(4, dtype=np.float32)
    with pytest.raises(T.TsdfError, match="workspace too small"):
        T.tf_track_noalloc(d, K, V, V, K, P, P, T.make_track_params((1, 1, 1, 1), (0.1, 0.1, 0.1, 0.1)), out)
