"""Pins for the search range and the raycast (Sec. 4.4).

* plane closed form: the refined hit lies on the plane up to the SDF
  quantisation plus the analytic residual of the two refinement steps,
  v (1 - dir_z)^2 for a ray with camera-frame direction z component dir_z;
  the normal is exactly (0, 0, -1) in the camera frame;
* analytic scene (C1 sphere on a floor, noiseless): surface RMS of the
  analytic signed distance at the hit points <= 0.5 voxel, <= 1 voxel at
  non-grazing, non-silhouette pixels;
* brute-force march: a dense 0.05-voxel march for the first + to - crossing
  of the trilinear field agrees with the state machine;
* the search range contains every point of every listed block (float64
  projection of random points inside the blocks).
"""
import numpy as np
import pytest

from synth import Intrinsics, analytic_sdf, configs, render_depth
from synth.scenes import Scene

K = configs.C1_INTR
VP = configs.C1_VOLUME


def _plane(oracle_mod, z0=1.0, frames=2):
    depth = np.full((K.height, K.width), z0, np.float32)
    pose = np.eye(4, dtype=np.float32)
    vol = oracle_mod.Volume.from_params(VP)
    for _ in range(frames):
        vol.alloc_and_visible(depth, K.as_array(), pose)
        vol.integrate(depth, K.as_array(), pose)
    return vol, pose


def test_plane_raycast_closed_form(oracle_mod):
    z0 = 1.0
    vol, pose = _plane(oracle_mod, z0)
    pts, nrm = vol.raycast(K.width, K.height, K.as_array(), pose)
    ys, xs = np.mgrid[0:K.height, 0:K.width]
    a = (xs - K.cx) / K.fx
    b = (ys - K.cy) / K.fy
    dir_z = 1.0 / np.sqrt(a * a + b * b + 1.0)
    interior = (xs >= 6) & (xs < K.width - 6) & (ys >= 6) & (ys < K.height - 6)
    hit = pts[..., 3] == 1
    assert hit[interior].all()
    quant = VP.mu / 32767.0 + 1e-6
    bound = VP.voxel_size * (1 - dir_z) ** 2 + quant
    err = np.abs(pts[..., 2] - z0)
    assert np.all(err[interior] <= bound[interior])
    centre = interior & ((xs - K.cx) ** 2 + (ys - K.cy) ** 2 <= 20 ** 2)
    assert err[centre].max() <= 2e-6
    # the hit lies on its own pixel ray
    zs = pts[..., 2]
    assert np.abs(pts[..., 0] - zs * a)[interior].max() <= 1e-5
    assert np.abs(pts[..., 1] - zs * b)[interior].max() <= 1e-5
    # gradient normal of a grid-aligned plane is exact
    assert np.all(nrm[interior] == np.array([0, 0, -1, 1], np.float32))
    # no hit outside the range image
    zmin, zmax = vol.range_image(K.width, K.height, K.as_array(), pose)
    assert not hit[~(zmin <= zmax)].any()


def _c1_volume(oracle_mod):
    d, p, intr, scene = configs.c1_frames()
    vol = oracle_mod.Volume.from_params(VP)
    for k in range(len(d)):
        vol.alloc_and_visible(d[k], intr.as_array(), p[k])
        vol.integrate(d[k], intr.as_array(), p[k])
    return vol, d, p, intr, scene


def test_c1_surface_error_against_analytic_sdf(oracle_mod):
    vol, d, p, intr, scene = _c1_volume(oracle_mod)
    pts, nrm = vol.raycast(K.width, K.height, intr.as_array(), p[-1])
    hit = pts[..., 3] == 1
    assert hit.mean() > 0.5
    e = np.zeros(hit.shape)
    e[hit] = analytic_sdf(scene, pts[hit][:, :3])
    rms = float(np.sqrt(np.mean(e[hit] ** 2)))
    assert rms <= 0.5 * VP.voxel_size
    # non-grazing, non-silhouette pixels: analytic normal vs ray below 60 deg,
    # no depth jump to a 4-neighbour, closer than 3 m
    depth = d[-1].astype(np.float64)
    jump = np.zeros_like(hit)
    dz = np.abs(np.diff(depth, axis=1)) > 0.05
    jump[:, :-1] |= dz
    jump[:, 1:] |= dz
    dzy = np.abs(np.diff(depth, axis=0)) > 0.05
    jump[:-1] |= dzy
    jump[1:] |= dzy
    q = pts[..., :3].reshape(-1, 3).astype(np.float64)
    h = 1e-4
    g = np.stack([(analytic_sdf(scene, q + h * np.eye(3)[i]) - analytic_sdf(scene, q - h * np.eye(3)[i]))
                  for i in range(3)], axis=1)
    g /= np.maximum(np.linalg.norm(g, axis=1, keepdims=True), 1e-12)
    M = p[-1].astype(np.float64)
    eye = -M[:3, :3].T @ M[:3, 3]
    ray = q - eye
    ray /= np.maximum(np.linalg.norm(ray, axis=1, keepdims=True), 1e-12)
    cosang = np.abs(np.sum(g * ray, axis=1)).reshape(hit.shape)
    # the integration leaves a 1-pixel image rim unobserved (u, v outside
    # [1, W-2] x [1, H-2]), so rays near the rim read unobserved neighbours
    ys, xs = np.mgrid[0:K.height, 0:K.width]
    rim = (xs < 4) | (xs >= K.width - 4) | (ys < 4) | (ys >= K.height - 4)
    good = hit & ~jump & ~rim & (depth > 0) & (depth < 3.0) & (cosang > 0.5)
    assert good.sum() > 3000
    assert np.abs(e[good]).max() <= VP.voxel_size
    # normals point against the ray and agree with the analytic normal
    n = nrm.reshape(-1, 3 + 1)[:, :3].astype(np.float64)
    cos_n = np.sum(n * g, axis=1).reshape(hit.shape)
    assert np.median(cos_n[good]) > 0.99


def test_brute_force_march_agrees(oracle_mod):
    """Dense march (0.05 voxel) on a small image: the first sample pair going
    from F >= 0 in a block with device data to F < 0, refined by bisection.
    The state machine steps at least one voxel, so it may step over a dip of
    the field thinner than that; the pin therefore asks that (i) hit/miss
    agrees on >= 99% of the pixels with a search range, (ii) at non-grazing
    pixels away from the unobserved image rim the two points agree within
    0.05 voxel for >= 90% of the pixels (otherwise the dense march found an
    earlier crossing), and (iii) every such hit lies within
    half a voxel (along the ray) of a + to - crossing of the field."""
    vol, d, p, intr, scene = _c1_volume(oracle_mod)
    small = Intrinsics(30.0, 30.0, 20.0, 15.0, 40, 30)
    pose = p[-1]
    pts, nrm = vol.raycast(small.width, small.height, small.as_array(), pose)
    zmin, zmax = vol.range_image(small.width, small.height, small.as_array(), pose)
    M = pose.astype(np.float64)
    Rinv = M[:3, :3].T
    tinv = -Rinv @ M[:3, 3]
    vs = VP.voxel_size
    o = tinv / vs
    _, _, ptr = vol.entries()

    def alloc(P):
        b = np.floor(np.floor(P) / 8.0).astype(int)
        i = vol.lookup(*b)
        return i >= 0 and ptr[i] >= 0

    def F(t, dr):
        return vol.trilinear(*(o + t * dr).astype(np.float32))

    agree = disagree = 0
    close = far = 0
    for y in range(small.height):
        for x in range(small.width):
            if not zmin[y, x] <= zmax[y, x]:
                continue
            r = np.array([(x - small.cx) / small.fx, (y - small.cy) / small.fy, 1.0])
            nr = np.linalg.norm(r)
            dr = Rinv @ (r / nr)
            t0, t1 = zmin[y, x] * nr / vs, zmax[y, x] * nr / vs
            prev_t, prev_F, found = None, None, None
            for t in np.arange(t0 - 8.0, t1 + 0.05, 0.05):
                if not alloc(o + t * dr):
                    prev_t = None
                    continue
                f = F(t, dr)
                if prev_t is not None and prev_F >= 0 and f < 0:
                    lo, hi = prev_t, t
                    for _ in range(30):
                        mid = 0.5 * (lo + hi)
                        lo, hi = (mid, hi) if F(mid, dr) >= 0 else (lo, mid)
                    found = 0.5 * (lo + hi)
                    break
                prev_t, prev_F = t, f
            hit = pts[y, x, 3] == 1
            if (found is not None) != hit:
                disagree += 1
                continue
            agree += 1
            if not hit:
                continue
            c = abs(float(np.dot(nrm[y, x, :3], dr)))
            if c < 0.5 or not (2 <= x < small.width - 2 and 2 <= y < small.height - 2):
                continue
            t_hit = float(np.dot(pts[y, x, :3] / vs - o, dr))
            if abs(found - t_hit) <= 0.05:
                close += 1
            else:
                # only a crossing the state machine stepped over may come first
                assert found < t_hit, (y, x, found, t_hit)
                far += 1
            ts = np.arange(t_hit - 0.5, t_hit + 0.5001, 0.05)
            fs = np.array([F(t, dr) for t in ts])
            assert np.any((fs[:-1] >= 0) & (fs[1:] < 0)), (y, x)
    assert agree + disagree > 500
    assert disagree <= 0.01 * (agree + disagree)
    assert close + far > 150
    assert far <= 0.10 * (close + far)


def test_range_contains_every_visible_block(oracle_mod):
    vol, d, p, intr, scene = _c1_volume(oracle_mod)
    pose = p[-1]
    zmin, zmax = vol.range_image(K.width, K.height, intr.as_array(), pose)
    pos, _, _ = vol.entries()
    vis = vol.visible()
    rng = np.random.default_rng(3)
    M = pose.astype(np.float64)
    n_checked = 0
    for i in vis:
        pts = (8.0 * pos[i].astype(np.float64) + rng.uniform(0, 8, size=(16, 3))) * VP.voxel_size
        c = pts @ M[:3, :3].T + M[:3, 3]
        z = c[:, 2]
        front = z > 0.06
        u = K.fx * c[front, 0] / z[front] + K.cx
        v = K.fy * c[front, 1] / z[front] + K.cy
        ins = (u >= 0) & (u <= K.width - 1) & (v >= 0) & (v <= K.height - 1)
        for uu, vv, zz in zip(u[ins], v[ins], z[front][ins]):
            for px in (int(np.floor(uu)), int(np.ceil(uu))):
                for py in (int(np.floor(vv)), int(np.ceil(vv))):
                    assert zmin[py, px] <= zz + 1e-5 and zz - 1e-5 <= zmax[py, px]
                    n_checked += 1
    assert n_checked > 1000


def test_range_for_foreign_pose_uses_all_blocks(oracle_mod):
    vol, d, p, intr, scene = _c1_volume(oracle_mod)
    zmin_all, zmax_all = vol.range_image(K.width, K.height, intr.as_array(), p[0], blocks="all")
    zmin_vis, zmax_vis = vol.range_image(K.width, K.height, intr.as_array(), p[0])
    cov_all = zmin_all <= zmax_all
    cov_vis = zmin_vis <= zmax_vis
    assert np.all(cov_all[cov_vis])
    assert np.all(zmin_all[cov_vis] <= zmin_vis[cov_vis])
    assert np.all(zmax_all[cov_vis] >= zmax_vis[cov_vis])


def test_range_clips_blocks_at_the_near_plane(oracle_mod):
    """A block straddling the near plane covers only the pixels of its part
    beyond the plane: one far to the side of the view covers none, and for
    cameras close to the surface every point of every block beyond the plane
    still falls inside its pixel's search interval."""
    vol, d, p, intr, scene = _c1_volume(oracle_mod)
    pos, _, ptr = vol.entries()
    blocks = pos[ptr >= 0].astype(np.float64)
    # pick a block; put the camera so the block spans camera z 0.05 at x = +0.5 m
    b = blocks[len(blocks) // 2]
    centre = (8.0 * b + 4.0) * VP.voxel_size
    M = np.eye(4)
    M[:3, 3] = -centre + np.array([0.5, 0.0, 0.05])        # world -> camera: pure translation
    one = np.array([np.flatnonzero(ptr >= 0)[len(blocks) // 2]], np.int32)
    zmin, zmax = vol.range_image(K.width, K.height, intr.as_array(), M.astype(np.float32), blocks=list(one))
    assert not np.any(zmin <= zmax)      # the old whole-image rule would cover every pixel
    # containment with cameras right at the surface
    rng = np.random.default_rng(11)
    for P in (p[-1], p[0]):
        Mc = P.astype(np.float64).copy()
        # slide the camera 1.15 m forward along its axis: about 5 cm from the sphere
        Mc[2, 3] -= 1.15
        zmin, zmax = vol.range_image(K.width, K.height, intr.as_array(), Mc.astype(np.float32), blocks="all")
        n = 0
        for i in np.flatnonzero(ptr >= 0):
            pts = (8.0 * pos[i].astype(np.float64) + rng.uniform(0, 8, size=(8, 3))) * VP.voxel_size
            c = pts @ Mc[:3, :3].T + Mc[:3, 3]
            z = c[:, 2]
            f = z > 0.06
            u = K.fx * c[f, 0] / z[f] + K.cx
            v = K.fy * c[f, 1] / z[f] + K.cy
            ins = (u >= 0) & (u <= K.width - 1) & (v >= 0) & (v <= K.height - 1)
            for uu, vv, zz in zip(u[ins], v[ins], z[f][ins]):
                px, py = int(round(uu)), int(round(vv))
                assert zmin[py, px] <= zz + 1e-5 and zz - 1e-5 <= zmax[py, px]
                n += 1
        assert n > 200
