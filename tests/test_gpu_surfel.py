"""GPU parity of surfel fusion (Sec. 7.3) against the oracle, through the C
ABI.  Each frame starts from the GPU map's own state, which the oracle also
takes; the bar: index map, per-pixel correspondences and surfel count equal
(integer decisions, float32 on both sides in the same order); new surfels'
positions, normals and radii equal to float32 rounding, their confidences
(alpha, an exp) within 1e-6 relative; updated surfels within 2e-5 m and
2e-5 of the float64 oracle (float32 sums over a surfel's circle); time
stamps equal.  A map fused from noiseless frames lies on the analytic
scene; runs are bit-reproducible; the capacity is kept with a flag."""
import numpy as np
import pytest

from gpu_helpers import to_device
from synth import analytic_sdf, configs, render_depth

pytestmark = pytest.mark.gpu

K2 = configs.KINECT_INTR


def _log(*a):
    print(*a, flush=True)


def _oracle_depth(mm):
    return (mm.astype(np.float32) / np.float32(1000.0)).astype(np.float32)


def test_frames_match_oracle_step_by_step():
    import paper_1708_00783_amd as T
    from oracle import surfel as S
    poses = np.stack(configs.c2_poses(300)[:8]).astype(np.float32)
    g = T.SurfelMap(1 << 21, K2.width, K2.height)
    for k in range(0, 8, 2):
        mm = configs.c2_frame(k)
        pos, nrm, tm = g.export()
        o = S.SurfelMap.from_state(pos, nrm, tm, g.stats()["frames"], 1 << 21)
        n0 = len(pos)
        ocorr = S.fuse(o, _oracle_depth(mm), K2.as_array(), poses[k])
        g.fuse(to_device(mm), K2, poses[k])
        gim, gcorr = g.export_frame()
        assert np.array_equal(gim, o.index_map), f"frame {k}: index maps differ"
        assert np.array_equal(gcorr, ocorr), f"frame {k}: correspondences differ"
        gp, gn, gt = g.export()
        assert len(gp) == len(o.pos), (k, len(gp), len(o.pos))
        assert np.array_equal(gt, o.time)
        # new surfels: the same float32 arithmetic
        np.testing.assert_allclose(gp[n0:], o.pos[n0:], rtol=0, atol=1e-6)
        np.testing.assert_allclose(gn[n0:, :3], o.nrm[n0:, :3], rtol=0, atol=1e-6)
        np.testing.assert_allclose(gn[n0:, 3], o.nrm[n0:, 3], rtol=1e-6)
        # updated surfels: float32 sums against float64
        np.testing.assert_allclose(gp[:n0], o.pos[:n0], rtol=0, atol=2e-5)
        np.testing.assert_allclose(gn[:n0, :3], o.nrm[:n0, :3], rtol=0, atol=2e-5)
        np.testing.assert_allclose(gn[:n0, 3], o.nrm[:n0, 3], rtol=2e-5)
        upd = int((gcorr >= 0).sum())
        _log(f"frame {k}: {len(gp)} surfels ({len(gp) - n0} new), {upd} pixels fused into existing ones")


def test_ragged_image_f32_and_reproducible():
    import paper_1708_00783_amd as T
    from oracle import surfel as S
    from synth import Intrinsics
    K = Intrinsics(270.0, 268.0, 166.3, 124.8, 333, 251)
    sc = configs.c2_scene(2)
    P = np.stack(configs.c2_poses(300, 2)[:3]).astype(np.float32)
    frames = [render_depth(sc, P[k], K).astype(np.float32) for k in range(3)]
    runs = []
    for _ in range(2):
        g = T.SurfelMap(1 << 20, 400, 300, max_depth_diff=0.03, min_normal_dot=0.7)
        for k in range(3):
            g.fuse(to_device(frames[k]), K, P[k])
        runs.append(g.export())
    for a, b in zip(*runs):
        assert np.array_equal(a, b)
    o = S.SurfelMap(1 << 20, delta_z=0.03, tau_n=0.7)
    g = T.SurfelMap(1 << 20, 400, 300, max_depth_diff=0.03, min_normal_dot=0.7)
    for k in range(2):
        g.fuse(to_device(frames[k]), K, P[k])
    pos, nrm, tm = g.export()
    o = S.SurfelMap.from_state(pos, nrm, tm, 2, 1 << 20, delta_z=0.03, tau_n=0.7)
    corr = S.fuse(o, frames[2], K.as_array(), P[2])
    g.fuse(to_device(frames[2]), K, P[2])
    gim, gcorr = g.export_frame()
    assert np.array_equal(gim, o.index_map) and np.array_equal(gcorr, corr)
    assert g.stats()["count"] == len(o.pos)


def test_noiseless_map_lies_on_the_scene():
    import paper_1708_00783_amd as T
    sc = configs.c2_scene(0)
    P = np.stack(configs.c2_poses(300)[:20]).astype(np.float32)
    g = T.SurfelMap(1 << 22, K2.width, K2.height)
    for k in range(0, 20, 4):
        g.fuse(to_device(render_depth(sc, P[k], K2).astype(np.float32)), K2, P[k])
    pos, nrm, tm = g.export()
    seen = nrm[:, 3] > 1.2            # fused more than once
    e = analytic_sdf(sc, pos[seen, :3].astype(np.float64))
    rms = float(np.sqrt(np.mean(e * e)))
    _log(f"{len(pos)} surfels, {int(seen.sum())} fused more than once, surface RMS {rms * 1e3:.3f} mm")
    assert seen.sum() > 100000 and rms < 2e-3


def test_capacity_and_empty_frames():
    import torch
    import paper_1708_00783_amd as T
    g = T.SurfelMap(1000, K2.width, K2.height)
    g.fuse(to_device(configs.c2_frame(0)), K2, configs.c2_poses(300)[0])
    st = g.stats()
    assert st["count"] == 1000 and st["flags"] & T.TF_FLAG_SURFEL_OVERFLOW
    g.reset()
    g.fuse(torch.zeros((K2.height, K2.width), dtype=torch.int16, device="cuda"), K2, configs.c2_poses(300)[0])
    st = g.stats()
    assert st["count"] == 0 and st["flags"] == 0 and st["frames"] == 1
