"""Pins for allocation and the visible list (Sec. 4.2).

The segment sampling is checked against exact float64 geometry (a slab test
of every block against the pixel's segment), the allocated set against a
plain set union of the per-pixel block keys (no hash table), and the visible
list against a float64 frustum test of its corners.
"""
import numpy as np
import pytest

from synth import Intrinsics, configs, render_depth

TINY_INTR = Intrinsics(30.0, 30.0, 20.0, 15.0, 40, 30)


def tiny_frames(n=2):
    scene = configs.c1_scene()
    poses = configs.c1_poses(10)
    idx = [0, 9][:n]
    depths = [render_depth(scene, poses[i], TINY_INTR).astype(np.float32) for i in idx]
    return depths, [poses[i].astype(np.float32) for i in idx]


def exact_segment(d, x, y, intr, pose, vs, mu):
    """float64 end points of the pixel's [d-mu, d+mu] segment in block units."""
    M = pose.astype(np.float64)
    R, t = M[:3, :3], M[:3, 3]
    r = np.array([(x - intr.cx) / intr.fx, (y - intr.cy) / intr.fy, 1.0])
    ends = []
    for z in (float(d) - mu, float(d) + mu):
        Xc = z * r
        Xw = R.T @ (Xc - t)
        ends.append(Xw / (8.0 * vs))
    return ends[0], ends[1]


def chord(a, b, lo, hi):
    """length of the part of segment a->b inside the box [lo, hi] (float64)"""
    d = b - a
    t0, t1 = 0.0, 1.0
    for k in range(3):
        if abs(d[k]) < 1e-15:
            if a[k] < lo[k] or a[k] > hi[k]:
                return -1.0
            continue
        u0 = (lo[k] - a[k]) / d[k]
        u1 = (hi[k] - a[k]) / d[k]
        if u0 > u1:
            u0, u1 = u1, u0
        t0, t1 = max(t0, u0), min(t1, u1)
        if t0 > t1:
            return -1.0
    return (t1 - t0) * float(np.linalg.norm(d))


def test_segment_blocks_match_exact_geometry(oracle_mod):
    vp = configs.C1_VOLUME
    depths, poses = tiny_frames(1)
    d, pose = depths[0], poses[0]
    K = TINY_INTR
    eps = 1e-4
    checked = 0
    for y in range(K.height):
        for x in range(K.width):
            if d[y, x] <= 0:
                continue
            keys = oracle_mod.segment_blocks(d[y, x], x, y, K.as_array(), K.width, K.height, pose,
                                             vp.voxel_size, vp.mu)
            a, b = exact_segment(d[y, x], x, y, K, pose, vp.voxel_size, vp.mu)
            L = float(np.linalg.norm(b - a))
            n = max(1, int(np.ceil(2 * L - 1e-6)))
            step = L / n
            assert n <= len(keys) <= n + 2          # n + 1 samples, n from float32 ceil(2L)
            ks = {tuple(k) for k in keys}
            # soundness: each key block touches the exact segment
            for k in ks:
                lo = np.array(k, np.float64) - eps
                assert chord(a, b, lo, lo + 1.0 + 2 * eps) >= 0.0, (x, y, k)
            # completeness: each block crossed over more than one sample spacing is present
            lo_b = np.floor(np.minimum(a, b)).astype(int) - 1
            hi_b = np.floor(np.maximum(a, b)).astype(int) + 1
            for bx in range(lo_b[0], hi_b[0] + 1):
                for by in range(lo_b[1], hi_b[1] + 1):
                    for bz in range(lo_b[2], hi_b[2] + 1):
                        lo = np.array([bx, by, bz], np.float64)
                        if chord(a, b, lo, lo + 1.0) >= step + eps:
                            assert (bx, by, bz) in ks, (x, y, (bx, by, bz))
            checked += 1
    assert checked > 300


def test_allocated_set_equals_union_of_segments(oracle_mod):
    vp = configs.C1_VOLUME
    depths, poses = tiny_frames(2)
    K = TINY_INTR
    vol = oracle_mod.Volume.from_params(vp)
    union = set()
    for d, pose in zip(depths, poses):
        touched = set()
        for y in range(K.height):
            for x in range(K.width):
                if d[y, x] > 0:
                    ks = oracle_mod.segment_blocks(d[y, x], x, y, K.as_array(), K.width, K.height,
                                                   pose, vp.voxel_size, vp.mu)
                    touched |= {tuple(k) for k in ks}
        union |= touched
        vol.alloc_and_visible(d, K.as_array(), pose)
        alloc = {tuple(p) for p in vol.allocated_positions()}
        assert alloc == union
        pos, _, _ = vol.entries()
        vis = {tuple(p) for p in pos[vol.visible()]}
        assert touched <= vis
    assert vol.flags == 0


def corner_visibility(block, vs, pose, K, margin=1e-3):
    """(+1 clearly inside, -1 clearly outside, 0 ambiguous) float64 test of
    whether some corner of the block projects into the image in front of the camera"""
    M = pose.astype(np.float64)
    best = -1
    for c in range(8):
        p = 8.0 * (np.array(block, np.float64) + [(c & 1), (c >> 1) & 1, (c >> 2) & 1])
        X = p * vs
        cc = M[:3, :3] @ X + M[:3, 3]
        if cc[2] <= 1e-9:
            continue
        u = K.fx * cc[0] / cc[2] + K.cx
        v = K.fy * cc[1] / cc[2] + K.cy
        if margin <= u <= K.width - 1 - margin and margin <= v <= K.height - 1 - margin:
            return 1
        if -margin <= u <= K.width - 1 + margin and -margin <= v <= K.height - 1 + margin:
            best = 0
    return best


def test_visible_list_carries_blocks_in_frustum(oracle_mod):
    vp = configs.C1_VOLUME
    depths, poses = tiny_frames(2)
    K = TINY_INTR
    vol = oracle_mod.Volume.from_params(vp)
    vol.alloc_and_visible(depths[0], K.as_array(), poses[0])
    pos, _, _ = vol.entries()
    vis1 = {tuple(p) for p in pos[vol.visible()]}
    assert vis1 == {tuple(p) for p in vol.allocated_positions()}
    before = {tuple(p) for p in vol.allocated_positions()}
    vol.alloc_and_visible(depths[1], K.as_array(), poses[1])
    pos, _, _ = vol.entries()
    vis2 = {tuple(p) for p in pos[vol.visible()]}
    after = {tuple(p) for p in vol.allocated_positions()}
    new = after - before
    assert new <= vis2
    # touched blocks of frame 2
    touched = set()
    d = depths[1]
    for y in range(K.height):
        for x in range(K.width):
            if d[y, x] > 0:
                touched |= {tuple(k) for k in oracle_mod.segment_blocks(
                    d[y, x], x, y, K.as_array(), K.width, K.height, poses[1], vp.voxel_size, vp.mu)}
    assert touched <= vis2
    assert vis2 <= touched | vis1
    n_in = n_out = 0
    for b in vis1 - touched:
        s = corner_visibility(b, vp.voxel_size, poses[1], K)
        if s == 1:
            assert b in vis2
            n_in += 1
        elif s == -1:
            assert b not in vis2
            n_out += 1
    assert n_in > 0


def test_depth_ingest_is_correctly_rounded(oracle_mod):
    mm = np.arange(0, 65536, dtype=np.uint16)
    got = oracle_mod.depth_from_mm(mm)
    want = (mm.astype(np.float64) / 1000.0).astype(np.float32)   # exact quotient, rounded once
    assert np.array_equal(got, want)
