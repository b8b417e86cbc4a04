"""Pins for the integration step (Sec. 4.3, computeUpdatedVoxelDepthInfo).

Closed forms: a fronto-parallel plane seen from the identity pose gives, for
every voxel of a visible block, weight 1 exactly where the voxel projects
inside the 1-pixel image border and lies no more than mu behind the plane,
and SDF = trunc(min(1, (Z0 - z) / mu) * 32767).  Repeated identical frames
give weight min(k, maxW) with the SDF held within 1 LSB.
"""
import numpy as np
import pytest

from synth import Intrinsics, configs, look_at, render_depth
from synth.scenes import Scene

K = configs.C1_INTR
VP = configs.C1_VOLUME
Z0 = 1.0


def plane_volume(oracle_mod, frames=1, z0=Z0, vp=VP):
    depth = np.full((K.height, K.width), z0, np.float32)
    pose = np.eye(4, dtype=np.float32)
    vol = oracle_mod.Volume.from_params(vp)
    for _ in range(frames):
        vol.alloc_and_visible(depth, K.as_array(), pose)
        vol.integrate(depth, K.as_array(), pose)
    return vol


def voxel_coords(pos):
    """(N, 512, 3) integer voxel coordinates, in-block order l = lx + 8 ly + 64 lz"""
    l = np.arange(512)
    off = np.stack([l & 7, (l >> 3) & 7, l >> 6], axis=1)
    return 8 * pos[:, None, :].astype(np.int64) + off[None, :, :]


def closed_form_plane(p, vs, mu, z0):
    """float64 closed form: (weight, sdf_float, ambiguous) for voxels p"""
    X = p * vs
    z = X[..., 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        u = K.fx * X[..., 0] / z + K.cx
        v = K.fy * X[..., 1] / z + K.cy
    inside = (z > 0) & (u >= 1) & (u <= K.width - 2) & (v >= 1) & (v <= K.height - 2)
    eta = z0 - z
    upd = inside & (eta >= -mu)
    amb = (np.abs(u - 1) < 1e-4) | (np.abs(u - (K.width - 2)) < 1e-4) | \
          (np.abs(v - 1) < 1e-4) | (np.abs(v - (K.height - 2)) < 1e-4) | (np.abs(eta + mu) < 1e-6)
    F = np.minimum(1.0, eta / mu)
    return upd, F, amb


def test_plane_single_frame_closed_form(oracle_mod):
    vol = plane_volume(oracle_mod, 1)
    pos, sdf, w = vol.voxels_by_position()
    assert len(pos) > 100
    p = voxel_coords(pos)
    upd, F, amb = closed_form_plane(p, VP.voxel_size, VP.mu, Z0)
    ok = ~amb
    assert np.array_equal(w[ok] == 1, upd[ok])
    assert np.all(w[~upd & ok] == 0) and np.all(sdf[~upd & ok] == 32767)
    want = np.trunc(F * 32767.0)
    diff = np.abs(sdf.astype(np.float64) - want)[upd & ok]
    assert diff.max() <= 1.0
    # the update covers the band on both sides of the surface
    assert (sdf[upd & ok] < 0).any() and (sdf[upd & ok] == 32767).any()


@pytest.mark.parametrize("frames", [3, 105])
def test_plane_repeated_frames(oracle_mod, frames):
    v1 = plane_volume(oracle_mod, 1)
    vk = plane_volume(oracle_mod, frames)
    p1, s1, w1 = v1.voxels_by_position()
    pk, sk, wk = vk.voxels_by_position()
    assert np.array_equal(p1, pk)
    assert np.array_equal(wk, np.where(w1 == 1, min(frames, VP.max_w), 0))
    assert np.abs(sk.astype(np.int32) - s1.astype(np.int32)).max() <= 1


def test_tilted_plane_closed_form_at_rounded_pixel(oracle_mod):
    """A floor seen obliquely: float64 closed form evaluated at the rounded pixel."""
    scene = Scene(floors=[0.0])
    pose = look_at([0.3, -1.0, 1.0], [0.0, 0.5, 0.0]).astype(np.float32)
    depth = render_depth(scene, pose, K).astype(np.float32)
    vol = oracle_mod.Volume.from_params(VP)
    vol.alloc_and_visible(depth, K.as_array(), pose)
    vol.integrate(depth, K.as_array(), pose)
    pos, sdf, w = vol.voxels_by_position()
    p = voxel_coords(pos).reshape(-1, 3)
    M = pose.astype(np.float64)
    c = (p * VP.voxel_size) @ M[:3, :3].T + M[:3, 3]
    z = c[:, 2]
    u = K.fx * c[:, 0] / z + K.cx
    v = K.fy * c[:, 1] / z + K.cy
    inside = (z > 0) & (u >= 1) & (u <= K.width - 2) & (v >= 1) & (v <= K.height - 2)
    ix = np.floor(np.where(inside, u, 1) + 0.5).astype(int)
    iy = np.floor(np.where(inside, v, 1) + 0.5).astype(int)
    d = depth[iy, ix].astype(np.float64)
    eta = d - z
    upd = inside & (d > 0) & (eta >= -VP.mu)
    frac_u = np.abs((u + 0.5) - np.round(u + 0.5))
    frac_v = np.abs((v + 0.5) - np.round(v + 0.5))
    amb = (frac_u < 1e-4) | (frac_v < 1e-4) | (np.abs(eta + VP.mu) < 1e-6) | \
          (np.abs(u - 1) < 1e-4) | (np.abs(u - (K.width - 2)) < 1e-4) | \
          (np.abs(v - 1) < 1e-4) | (np.abs(v - (K.height - 2)) < 1e-4)
    ok = ~amb
    wf = w.reshape(-1)
    sf = sdf.reshape(-1).astype(np.float64)
    assert ok.mean() > 0.99
    assert np.array_equal(wf[ok] == 1, upd[ok])
    want = np.trunc(np.minimum(1.0, eta / VP.mu) * 32767.0)
    assert np.abs(sf - want)[upd & ok].max() <= 1.0
    assert upd.sum() > 10000


def test_reciprocal_form_matches_division_form(oracle_mod):
    """The evaluation order used (one reciprocal of z, multiplications by
    1/mu and 1/(w+1)) against the same update with every quotient as a
    division, over the ten C1 frames: weights differ only where a pixel
    choice flips (rare), SDFs by <= 1 LSB elsewhere."""
    d, p, intr, _ = configs.c1_frames()
    a = oracle_mod.Volume.from_params(VP)
    b = oracle_mod.Volume.from_params(VP)
    for k in range(len(d)):
        for vol, div in ((a, False), (b, True)):
            vol.alloc_and_visible(d[k], intr.as_array(), p[k])
            vol.integrate(d[k], intr.as_array(), p[k], divide=div)
    pa, sa, wa = a.voxels_by_position()
    pb, sb, wb = b.voxels_by_position()
    assert np.array_equal(pa, pb)
    same_w = wa == wb
    assert same_w.mean() > 1 - 1e-4
    ds = np.abs(sa.astype(np.int32) - sb.astype(np.int32))[same_w]
    assert np.mean(ds <= 1) > 1 - 1e-4


def test_integration_independent_of_thread_count(oracle_mod, monkeypatch):
    import subprocess
    import sys
    code = ("import numpy as np, sys; sys.path.insert(0, '.');"
            "from oracle import oracle as O; from synth import configs;"
            "d,p,K,_=configs.c1_frames(4); v=O.Volume.from_params(configs.C1_VOLUME)\n"
            "for k in range(4): v.frame(d[k], K.as_array(), p[k])\n"
            "pos,s,w=v.voxels_by_position(); pts,n=v.raycast(160,120,K.as_array(),p[3]);"
            "import hashlib; print(hashlib.sha1(s.tobytes()+w.tobytes()+pts.tobytes()+n.tobytes()).hexdigest())")
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    outs = []
    for t in ("1", "4"):
        env = dict(os.environ, OMP_NUM_THREADS=t)
        outs.append(subprocess.check_output([sys.executable, "-c", code], cwd=root, env=env).strip())
    assert outs[0] == outs[1]
