"""GPU parity of the batched rigid submaps (Sec. 7.2) through the C ABI
against the oracle's submaps and combined field.

Per submap: allocated and visible sets equal, voxel weights bit-exact, SDF
within 1 LSB (frames are fused with the camera composed with the submap
pose).  Combined-field raycast of several views of different sizes: points
within 1e-4 m, normals within 1e-3, at most 0.1% hit/miss disagreement; the
search range of a view is exact.  Every launch shape gives the same outputs,
and a HIP graph replay gives what the direct launches give."""
import numpy as np
import pytest

from gpu_helpers import compare_raycast, compare_tables, compare_visible, oracle_depth, to_device
from synth import Intrinsics, configs, look_at

pytestmark = pytest.mark.gpu

VP = configs.C1_VOLUME
K = configs.C1_INTR


def _log(*a):
    print(*a, flush=True)


def _rot(axis, ang, t):
    c, s = np.cos(ang), np.sin(ang)
    R = {"z": [[c, -s, 0], [s, c, 0], [0, 0, 1]], "x": [[1, 0, 0], [0, c, -s], [0, s, c]],
         "y": [[c, 0, s], [0, 1, 0], [-s, 0, c]]}[axis]
    P = np.eye(4)
    P[:3, :3] = R
    P[:3, 3] = t
    return P.astype(np.float32)


POSES = np.stack([np.eye(4, dtype=np.float32), _rot("z", 0.5236, [0.137, -0.081, 0.029]),
                  _rot("x", -0.31, [-0.05, 0.21, 0.013])])
# which frames go to which submaps (every submap misses some frames)
SCHEDULE = [[0, 2], [0, 1], [1, 2], [0, 1, 2], [1], [0, 2], [2], [0, 1], [1, 2], [0, 1, 2]]
VIEW2 = Intrinsics(150.0, 150.0, 99.5, 74.5, 200, 150)


def _views_poses(p):
    return [(K, p[-1]), (VIEW2, look_at([0.9, -0.8, 0.7], [0.0, 0.0, 0.2]).astype(np.float32)),
            (K, p[4])]


class MultiPair:
    def __init__(self, n_frames=10):
        from oracle import oracle as O
        import paper_1708_00783_amd as T
        self.d, self.p, _, _ = configs.c1_frames(n_frames)
        self.ovols = [O.Volume.from_params(VP) for _ in POSES]
        self.o = O.Multi(self.ovols, POSES)
        self.g = T.MultiMap(VP, POSES, K.width, K.height, 200, 150, 1 << 20)

    def integrate(self, k):
        sel = SCHEDULE[k]
        for i in sel:
            self.o.integrate_frame(i, oracle_depth(self.d[k]), K.as_array(), self.p[k])
        self.g.integrate(to_device(self.d[k]), K, self.p[k], sel)
        return sel

    def views(self):
        import torch
        out = []
        for intr, pose in _views_poses(self.p):
            pts = torch.full((intr.height, intr.width, 4), -7.0, dtype=torch.float32, device="cuda")
            nrm = torch.full_like(pts, -7.0)
            out.append((intr, pose, pts, nrm))
        return out


def test_submaps_integrate_and_combined_raycast():
    mp = MultiPair()
    _log("case submaps: 3 submaps (identity, rotated z, rotated x), c1 frames, 3 views")
    for k in range(len(mp.d)):
        sel = mp.integrate(k)
        for i in sel:
            gv = mp.g.submap(i)
            compare_visible(gv, mp.ovols[i], f"frame {k} submap {i}")
            nblk, nsd = compare_tables(gv, mp.ovols[i], f"frame {k} submap {i}")
        _log(f"frame {k} into {sel}: last submap blocks {nblk} sdf-lsb-diffs {nsd}")
    views = mp.views()
    mp.g.raycast(views)
    for vi, (intr, pose, pts, nrm) in enumerate(views):
        op, on = mp.o.raycast(intr.width, intr.height, intr.as_array(), pose)
        nhit, flips = compare_raycast(pts.cpu().numpy(), nrm.cpu().numpy(), op, on, f"view {vi}")
        _log(f"view {vi} {intr.width}x{intr.height}: hits {nhit} flips {flips}")
        assert nhit > 0.2 * intr.width * intr.height
    st = mp.g.stats()
    assert st["flags"] == 0
    assert st["allocated_blocks"] == sum(len(v.allocated_positions()) for v in mp.ovols)


def test_submaps_range_image_exact():
    mp = MultiPair(6)
    for k in range(6):
        mp.integrate(k)
    for intr, pose in _views_poses(mp.p):
        gz0, gz1 = mp.g.range_image(intr, pose)
        oz0, oz1 = mp.o.range_image(intr.width, intr.height, intr.as_array(), pose)
        assert np.array_equal(gz0.cpu().numpy(), oz0)
        assert np.array_equal(gz1.cpu().numpy(), oz1)


def test_every_launch_shape_gives_the_same_outputs():
    mp = MultiPair(6)
    for k in range(6):
        mp.integrate(k)
    ref = None
    for tw, th in ((16, 16), (32, 8), (16, 8), (8, 8)):
        for bg in (1, 64, 300):
            mp.g.set_config(tile_w=tw, tile_h=th, bin_groups=bg)
            views = mp.views()
            mp.g.raycast(views)
            out = [(p.cpu().numpy(), n.cpu().numpy()) for _, _, p, n in views]
            if ref is None:
                ref = out
            for (a, b), (c, d) in zip(ref, out):
                assert np.array_equal(a, c) and np.array_equal(b, d), (tw, th, bg)
    # integration shapes: identical maps
    a, b = MultiPair(4), MultiPair(4)
    b.g.set_config(integrate_threads=64, integrate_groups=7)
    for k in range(4):
        a.integrate(k)
        b.integrate(k)
    for i in range(len(POSES)):
        pa, sa, wa = a.g.submap(i).voxels_by_position()
        pb, sb, wb = b.g.submap(i).voxels_by_position()
        assert np.array_equal(pa, pb) and np.array_equal(sa, sb) and np.array_equal(wa, wb)


def test_graph_replay_matches_direct_launches():
    import torch
    direct, graph = MultiPair(8), MultiPair(8)
    for k in range(8):
        for mp, use_graph in ((direct, False), (graph, True)):
            views = mp.views()
            mp.g.frame(to_device(mp.d[k]), K, mp.p[k], SCHEDULE[k], views, use_graph=use_graph)
            mp._last = views
        torch.cuda.synchronize()
        for (_, _, p0, n0), (_, _, p1, n1) in zip(direct._last, graph._last):
            assert torch.equal(p0, p1) and torch.equal(n0, n1), f"frame {k}"
    for i in range(len(POSES)):
        pa, sa, wa = direct.g.submap(i).voxels_by_position()
        pb, sb, wb = graph.g.submap(i).voxels_by_position()
        assert np.array_equal(pa, pb) and np.array_equal(sa, sb) and np.array_equal(wa, wb)


def test_autotune_picks_a_supported_shape_and_keeps_results():
    mp = MultiPair(5)
    for k in range(4):
        mp.integrate(k)
    views = mp.views()
    best, ms = mp.g.autotune(to_device(mp.d[4]), K, mp.p[4], SCHEDULE[4], views, reps=2)
    _log(f"autotune: {best} {ms:.3f} ms")
    assert (best["tile_w"], best["tile_h"]) in ((16, 16), (32, 8), (16, 8), (8, 8))
    assert ms > 0
    # the autotune allocated frame 4's blocks but integrated nothing
    for i in SCHEDULE[4]:
        w = mp.g.submap(i).voxels_by_position()[2]
        ow = mp.ovols[i].voxels_by_position()[2]
        assert int(w.astype(np.int64).sum()) == int(ow.astype(np.int64).sum())
    mp.integrate(4)
    for i in SCHEDULE[4]:
        compare_tables(mp.g.submap(i), mp.ovols[i], f"after autotune, submap {i}")


def test_tiny_views_whose_bins_overflow_the_tile_table():
    """One-tile views (16x16 pixels for 16x16 tiles, 8x8 for 8x8) that see the
    whole scene: every block of the three submaps lands in the view's one
    tile, so its bin holds more records than the tile's LDS table (2048 at
    16x16, 1024 at 8x8) and the table keeps the records nearest the camera;
    the outputs still match the oracle."""
    mp = MultiPair()
    for k in range(len(mp.d)):
        mp.integrate(k)
    import torch
    eye = look_at([1.1, -0.9, 0.8], [0.0, 0.0, 0.2]).astype(np.float32)
    for tw, th, intr, cap in ((16, 16, Intrinsics(9.0, 9.0, 7.5, 7.5, 16, 16), 2048),
                              (8, 8, Intrinsics(4.5, 4.5, 3.5, 3.5, 8, 8), 1024)):
        mp.g.set_config(tile_w=tw, tile_h=th)
        pts = torch.full((intr.height, intr.width, 4), -7.0, dtype=torch.float32, device="cuda")
        nrm = torch.full_like(pts, -7.0)
        b0 = mp.g.stats()["total_bin_entries"]
        mp.g.raycast([(intr, eye, pts, nrm)])
        entries = mp.g.stats()["total_bin_entries"] - b0
        _log(f"one {tw}x{th} tile: {entries} bin entries, table {cap}")
        assert entries > cap
        op, on = mp.o.raycast(intr.width, intr.height, intr.as_array(), eye)
        nhit, flips = compare_raycast(pts.cpu().numpy(), nrm.cpu().numpy(), op, on, f"one-tile view {tw}x{th}")
        _log(f"one-tile view {intr.width}x{intr.height}: hits {nhit} flips {flips}")
        assert nhit > 0.2 * intr.width * intr.height


def test_close_view_blocks_over_many_tiles():
    """A 200x150 view 7 cm from the sphere's surface: a block's grown cube
    covers dozens of 16x16 tiles, so the binning takes its global path for
    those blocks (no per-chunk aggregation); the outputs match the oracle."""
    mp = MultiPair()
    for k in range(len(mp.d)):
        mp.integrate(k)
    import torch
    eye = look_at([0.26, -0.15, 0.35], [0.0, 0.0, 0.25]).astype(np.float32)
    mp.g.set_config(tile_w=16, tile_h=16)
    pts = torch.full((VIEW2.height, VIEW2.width, 4), -7.0, dtype=torch.float32, device="cuda")
    nrm = torch.full_like(pts, -7.0)
    b0 = mp.g.stats()
    mp.g.raycast([(VIEW2, eye, pts, nrm)])
    b1 = mp.g.stats()
    entries = b1["total_bin_entries"] - b0["total_bin_entries"]
    pairs = b1["total_block_views"] - b0["total_block_views"]
    # tiles of the grown cubes (3 voxels) of submap 0's blocks (its pose is the identity)
    pos = mp.ovols[0].allocated_positions().astype(np.float64)
    c = np.array([[(k & 1), (k >> 1) & 1, k >> 2] for k in range(8)], np.float64)
    X = ((pos[:, None, :] * 8 - 3) + c[None] * 14) * VP.voxel_size
    Pc = X @ eye[:3, :3].T.astype(np.float64) + eye[:3, 3]
    front = (Pc[..., 2] > 0.05).all(1)
    u = VIEW2.fx * Pc[front][..., 0] / Pc[front][..., 2] + VIEW2.cx
    v = VIEW2.fy * Pc[front][..., 1] / Pc[front][..., 2] + VIEW2.cy
    u0, u1 = np.clip(u.min(1), 0, VIEW2.width - 1), np.clip(u.max(1), 0, VIEW2.width - 1)
    v0, v1 = np.clip(v.min(1), 0, VIEW2.height - 1), np.clip(v.max(1), 0, VIEW2.height - 1)
    ntiles = (u1 // 16 - u0 // 16 + 1) * (v1 // 16 - v0 // 16 + 1)
    _log(f"close view: {pairs} blocks in view, {entries} bin entries; submap 0: {int((ntiles > 16).sum())} "
         f"blocks over 16 tiles, at most {int(ntiles.max())}")
    assert (ntiles > 16).sum() > 10
    op, on = mp.o.raycast(VIEW2.width, VIEW2.height, VIEW2.as_array(), eye)
    nhit, flips = compare_raycast(pts.cpu().numpy(), nrm.cpu().numpy(), op, on, "close view")
    _log(f"close view: hits {nhit} flips {flips}")
    assert nhit > 0.2 * VIEW2.width * VIEW2.height


def _pool_map(fn, items):
    import multiprocessing as mp
    import os
    n = max(1, min(16, len(os.sched_getaffinity(0))))
    with mp.get_context("fork").Pool(n) as pool:
        return pool.map(fn, items, chunksize=max(1, len(items) // (4 * n)))


def _prefill_depth(a):
    return configs.c4_prefill_frame(*a)


def _walk_depth(k):
    return configs.c4_frame(k)


def test_benchmark_shape_sampled_parity():
    """The benchmark's shape: 64 submaps with its volume parameters and poses
    (5 mm voxels), each fused from 3 noiseless 320x240 viewpoints of its region
    (a fixed schedule), then walk frames 0 and 1 at 640x480 fused into the
    submaps they overlap; its 8 views, 320x240 to 1280x720, raycast on the
    combined field.  The oracle fuses the same frames into its own submaps.
    Compared: the tables of the submaps the last walk frame reaches (first 3),
    every view's range image exactly, and the raycast at 1024 seeded pixels of
    every view (the oracle marches only those, each from the whole view's range
    image), at most one hit/miss disagreement per view."""
    import torch
    import paper_1708_00783_amd as T
    from oracle import oracle as O
    KW = configs.KINECT_INTR
    KP = configs.C4_PREFILL_INTR
    subs = configs.c4_submaps()
    P = np.stack([s.pose for s in subs])
    items = [(i, j) for i in range(len(subs)) for j in range(3)]
    walk = configs.c4_poses()
    prefill = _pool_map(_prefill_depth, items)
    walk_d = _pool_map(_walk_depth, [0, 1])
    _log(f"case benchmark shape: {len(subs)} submaps, {len(items)} prefill frames, 2 walk frames, 8 views")
    ovols = [O.Volume.from_params(configs.C4_VOLUME) for _ in subs]
    o = O.Multi(ovols, P)
    g = T.MultiMap(configs.C4_VOLUME, P, KW.width, KW.height, 1280, 720, 1 << 25)
    for (i, j), dep in zip(items, prefill):
        pose = configs.c4_prefill_pose(i, j)
        g.integrate(torch.from_numpy(dep).cuda(), KP, pose, [i])
        o.integrate_frame(i, dep, KP.as_array(), pose)
    sel = []
    for k in range(2):
        sel = configs.c4_select(walk[k])
        g.integrate(to_device(walk_d[k]), KW, walk[k], sel)
        for i in sel:
            o.integrate_frame(i, oracle_depth(walk_d[k]), KW.as_array(), walk[k])
    for i in sel[:3]:
        compare_visible(g.submap(i), ovols[i], f"submap {i}")
        nblk, nsd = compare_tables(g.submap(i), ovols[i], f"submap {i}")
        _log(f"submap {i}: blocks {nblk} sdf-lsb-diffs {nsd}")
    views = []
    for intr, pose in configs.c4_views(1):
        pts = torch.full((intr.height, intr.width, 4), -7.0, dtype=torch.float32, device="cuda")
        views.append((intr, pose, pts, torch.full_like(pts, -7.0)))
    g.raycast(views)
    st = g.stats()
    assert st["flags"] == 0, st   # no capacity or bin overflow
    assert st["allocated_blocks"] == sum(len(v.allocated_positions()) for v in ovols)
    rng = np.random.default_rng(11)
    for vi, (intr, pose, pts, nrm) in enumerate(views):
        W, H = intr.width, intr.height
        gz0, gz1 = g.range_image(intr, pose)
        oz0, oz1 = o.range_image(W, H, intr.as_array(), pose)
        assert np.array_equal(gz0.cpu().numpy(), oz0) and np.array_equal(gz1.cpu().numpy(), oz1), f"view {vi} range"
        m = np.zeros((H, W), bool)
        m.flat[rng.choice(W * H, 1024, replace=False)] = True
        op, on = o.raycast(W, H, intr.as_array(), pose, mask=m)
        gp, gn = pts.cpu().numpy(), nrm.cpu().numpy()
        nhit, flips = compare_raycast(gp[m], gn[m], op[m], on[m], f"view {vi} {W}x{H}")
        _log(f"view {vi} {W}x{H}: sampled hits {nhit} of 1024, flips {flips}")
        assert nhit > 500
