"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded frames.  Bars: allocated and visible block sets equal; voxel
weights bit-exact; stored SDF within 1 LSB; raycast points within 1e-4 m,
normals within 1e-3, at most 0.1% hit/miss disagreement."""
import numpy as np
import pytest

from gpu_helpers import (Pair, compare_raycast, compare_tables, compare_visible, oracle_depth,
                         to_device)
from synth import Intrinsics, configs, look_at, render_depth
from synth.scenes import Scene

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, flush=True)


def test_c1_all_frames_parity():
    d, p, K, _ = configs.c1_frames()
    _log("case c1 tiny 160x120, 10 frames")
    pair = Pair(configs.C1_VOLUME, K.width, K.height)
    for k in range(len(d)):
        pair.frame(d[k], K, p[k])
        nvis = compare_visible(pair.g, pair.o, f"c1 frame {k}")
        nblk, nsd = compare_tables(pair.g, pair.o, f"c1 frame {k}")
        gp, gn, op, on = pair.raycast(K, p[k])
        nhit, flips = compare_raycast(gp, gn, op, on, f"c1 frame {k}")
        _log(f"c1 frame {k}: blocks {nblk} visible {nvis} sdf-lsb-diffs {nsd} hits {nhit} flips {flips}")
    st = pair.g.stats()
    assert st["flags"] == 0 and st["frames"] == len(d)
    assert st["n_allocated"] == len(pair.o.allocated_positions())


def test_c1_range_image_exact():
    d, p, K, _ = configs.c1_frames(4)
    pair = Pair(configs.C1_VOLUME, K.width, K.height)
    for k in range(4):
        pair.frame(d[k], K, p[k])
    gz0, gz1 = pair.g.range_image(p[3], K)
    oz0, oz1 = pair.o.range_image(K.width, K.height, K.as_array(), p[3])
    assert np.array_equal(gz0.cpu().numpy(), oz0)
    assert np.array_equal(gz1.cpu().numpy(), oz1)
    # a pose that is not the allocation pose projects every block
    gz0, gz1 = pair.g.range_image(p[0], K)
    oz0, oz1 = pair.o.range_image(K.width, K.height, K.as_array(), p[0], blocks="all")
    assert np.array_equal(gz0.cpu().numpy(), oz0)
    assert np.array_equal(gz1.cpu().numpy(), oz1)


def test_c2_full_frame_parity():
    """the first 32 frames of the full-frame trajectory, fused in order from
    frame 0 (fusion is sequential): visible sets and raycasts every frame,
    the whole map (allocated set, weights, SDF) every 8th frame and the last"""
    n_frames = 32
    d, p, K, _ = configs.c2_frames(n_frames)
    _log(f"case c2 full 640x480 u16, {n_frames} frames")
    pair = Pair(configs.C2_VOLUME, K.width, K.height)
    for k in range(n_frames):
        pair.frame(d[k], K, p[k])
        nvis = compare_visible(pair.g, pair.o, f"c2 frame {k}")
        gp, gn, op, on = pair.raycast(K, p[k])
        nhit, flips = compare_raycast(gp, gn, op, on, f"c2 frame {k}")
        msg = f"c2 frame {k}: visible {nvis} hits {nhit} flips {flips}"
        if k % 8 == 0 or k == n_frames - 1:
            nblk, nsd = compare_tables(pair.g, pair.o, f"c2 frame {k}")
            msg += f" blocks {nblk} sdf-lsb-diffs {nsd}"
        _log(msg)
    assert pair.g.stats()["flags"] == 0


def test_ragged_image_and_foreign_view():
    """image sizes that are not multiples of the 16x16 tile; raycast from a
    pose other than the allocation pose (all blocks feed the search range)"""
    K = Intrinsics(50.0, 50.0, 18.5, 11.0, 37, 23)
    scene = configs.c1_scene()
    poses = [P.astype(np.float32) for P in configs.c1_poses(6)]
    pair = Pair(configs.C1_VOLUME, 64, 64)
    for k in range(5):
        depth = render_depth(scene, poses[k], K).astype(np.float32)
        pair.frame(depth, K, poses[k])
    compare_tables(pair.g, pair.o, "ragged")
    compare_visible(pair.g, pair.o, "ragged")
    gp, gn, op, on = pair.raycast(K, poses[5])            # foreign pose
    compare_raycast(gp, gn, op, on, "ragged foreign pose")
    K2 = Intrinsics(40.0, 40.0, 30.0, 30.0, 61, 59)       # foreign intrinsics
    gp, gn, op, on = pair.raycast(K2, poses[4])
    compare_raycast(gp, gn, op, on, "ragged foreign intrinsics")


def test_search_range_reuse_and_rebuild():
    """The allocation view's search range is binned by the integration launch
    and consumed by the next raycast of that view; a repeated raycast, a
    raycast of another view in between, a range image, and an integration at
    a pose other than the allocation's (no binning) all match the oracle."""
    d, p, K, _ = configs.c1_frames(5)
    pair = Pair(configs.C1_VOLUME, K.width, K.height)
    for k in range(4):
        pair.frame(d[k], K, p[k])
    for tag, pose in (("allocation view", p[3]), ("allocation view again", p[3]), ("other view", p[0]),
                      ("allocation view after another", p[3])):
        gp, gn, op, on = pair.raycast(K, pose)
        nhit, flips = compare_raycast(gp, gn, op, on, tag)
        _log(f"{tag}: hits {nhit} flips {flips}")
    # bins pending from the integration, then a range image of the allocation view
    pair.frame(d[4], K, p[4])
    gz0, gz1 = pair.g.range_image(p[4], K)
    oz0, oz1 = pair.o.range_image(K.width, K.height, K.as_array(), p[4])
    assert np.array_equal(gz0.cpu().numpy(), oz0) and np.array_equal(gz1.cpu().numpy(), oz1)
    # allocation at one pose, integration at another: the raycast bins for itself
    pair.alloc(d[3], K, p[3])
    pair.integrate(d[3], K, p[2])
    gp, gn, op, on = pair.raycast(K, p[3])
    compare_raycast(gp, gn, op, on, "integration at another pose")
    compare_tables(pair.g, pair.o, "integration at another pose")


def test_empty_and_invalid_depth():
    K = configs.C1_INTR
    pair = Pair(configs.C1_VOLUME, K.width, K.height)
    zero = np.zeros((K.height, K.width), np.float32)
    pose = np.eye(4, dtype=np.float32)
    pair.frame(zero, K, pose)
    assert len(pair.g.allocated_positions()) == 0
    assert len(pair.g.visible()) == 0
    gp, gn, op, on = pair.raycast(K, pose)
    assert not (gp[..., 3] != 0).any()
    # then a real frame, then an empty one: the visible list carries over
    d, p, _, _ = configs.c1_frames(2)
    pair.frame(d[0], K, p[0])
    pair.frame(zero, K, p[0])
    compare_visible(pair.g, pair.o, "carry over")
    compare_tables(pair.g, pair.o, "carry over")
    assert len(pair.g.visible()) > 0


def test_plane_parity_and_weight_cap():
    """105 identical frames of a plane: the weight saturates at maxW"""
    K = configs.C1_INTR
    pair = Pair(configs.C1_VOLUME, K.width, K.height)
    depth = np.full((K.height, K.width), 1.0, np.float32)
    pose = np.eye(4, dtype=np.float32)
    for _ in range(105):
        pair.frame(depth, K, pose)
    compare_tables(pair.g, pair.o, "plane x105")
    _, _, w = pair.g.voxels_by_position()
    assert w.max() == configs.C1_VOLUME.max_w
    gp, gn, op, on = pair.raycast(K, pose)
    compare_raycast(gp, gn, op, on, "plane")


def test_collisions_in_tiny_table():
    """2^4 buckets force long excess chains built concurrently"""
    from synth.configs import VolumeParams
    vp = VolumeParams(0.01, 0.04, 100, 1 << 4, 1 << 13, 1 << 14)
    d, p, K, _ = configs.c1_frames(3)
    pair = Pair(vp, K.width, K.height)
    for k in range(3):
        pair.frame(d[k], K, p[k])
    nblk, _ = compare_tables(pair.g, pair.o, "tiny table")
    compare_visible(pair.g, pair.o, "tiny table")
    gp, gn, op, on = pair.raycast(K, p[2])
    compare_raycast(gp, gn, op, on, "tiny table")
    pos, off, ptr = pair.g.entries()
    assert int((ptr[16:] >= 0).sum()) == nblk - int((ptr[:16] >= 0).sum())


def test_block_exhaustion_sets_flag_and_keeps_invariants():
    from synth.configs import VolumeParams
    vp = VolumeParams(0.01, 0.04, 100, 1 << 16, 1 << 12, 500)
    d, p, K, _ = configs.c1_frames(2)
    pair = Pair(vp, K.width, K.height)
    pair.frame(d[0], K, p[0])
    st = pair.g.stats()
    assert st["flags"] & 1
    assert st["n_allocated"] == 500
    gset = {tuple(x) for x in pair.g.allocated_positions()}
    full = Pair(configs.C1_VOLUME, K.width, K.height)
    full.o.alloc_and_visible(d[0], K.as_array(), p[0])
    assert gset <= {tuple(x) for x in full.o.allocated_positions()}
    pos, off, ptr = pair.g.entries()
    alloc = ptr >= 0
    assert len(set(ptr[alloc].tolist())) == int(alloc.sum())
    # the volume keeps working after exhaustion
    pair.g.integrate(to_device(d[0]), p[0])
    pts, _ = pair.g.raycast(p[0], K)
    assert (pts.cpu().numpy()[..., 3] == 1).any()


def test_exhaustion_in_consecutive_frames_keeps_the_stacks_consistent():
    """Pops past an empty stack in several frames in a row (the stack height
    goes below zero inside the insertion and is clamped before the next push).
    Blocks exhausted: the allocated count stays at capacity and every allocated
    entry holds a distinct block.  Excess slots exhausted (16 buckets, 32
    slots): every slot holds a block, the free-slot count reads zero, and the
    blocks popped for links that found no slot went back to the stack."""
    import paper_1708_00783_amd as T
    from synth.configs import VolumeParams
    d, p, K, _ = configs.c1_frames(3)
    g = T.Volume(VolumeParams(0.01, 0.04, 100, 1 << 16, 1 << 12, 500), K.width, K.height)
    for k in range(3):
        g.frame(to_device(d[k]), K, p[k])
        st = g.stats()
        assert st["flags"] & 1 and st["n_allocated"] == 500, (k, st)
        _, _, ptr = g.entries()
        alloc = ptr >= 0
        assert int(alloc.sum()) == 500 and len(set(ptr[alloc].tolist())) == 500, k
    g = T.Volume(VolumeParams(0.01, 0.04, 100, 1 << 4, 32, 1 << 14), K.width, K.height)
    for k in range(2):
        g.frame(to_device(d[k]), K, p[k])
        st = g.stats()
        assert st["flags"] & 2 and st["n_free_excess"] == 0, (k, st)
        _, _, ptr = g.entries()
        alloc = ptr >= 0
        assert int(alloc[16:].sum()) == 32, k
        assert st["n_allocated"] == int(alloc.sum()), (k, st)
        assert len(set(ptr[alloc].tolist())) == int(alloc.sum()), k


def test_repeatable():
    d, p, K, _ = configs.c1_frames(4)
    import paper_1708_00783_amd as T
    outs = []
    for _ in range(2):
        g = T.Volume(configs.C1_VOLUME, K.width, K.height)
        for k in range(4):
            pts, nrm = g.frame(to_device(d[k]), K, p[k])
        pos, sdf, w = g.voxels_by_position()
        outs.append((pos, sdf, w, pts.cpu().numpy(), nrm.cpu().numpy()))
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)


def test_tile_bins_overflow_fall_back_to_all_records():
    """More than 512 search-range records in a 16x16 tile: the raycast takes
    the per-pixel range over the full record list, with block lookups in the
    global table.  A 24x20 image with a 6-pixel focal length (four tiles, the
    whole C1 map in view): from another view every allocated block is binned,
    and from the view of an allocation at that size the ~3300 visible blocks."""
    d, p, K, _ = configs.c1_frames(5)
    Kt = Intrinsics(6.0, 6.0, 11.5, 9.5, 24, 20)
    pair = Pair(configs.C1_VOLUME, K.width, K.height)
    for k in range(4):
        pair.frame(d[k], K, p[k])
    n_alloc = pair.g.stats()["n_allocated"]
    assert n_alloc > 4 * 512
    gp, gn, op, on = pair.raycast(Kt, p[3])          # another view: all blocks
    nhit, flips = compare_raycast(gp, gn, op, on, "overflowing bins, all blocks")
    assert nhit > 20          # the fused patch covers a small part of the wide view
    gz0, gz1 = pair.g.range_image(p[2], Kt)
    oz0, oz1 = pair.o.range_image(Kt.width, Kt.height, Kt.as_array(), p[2], blocks="all")
    assert np.array_equal(gz0.cpu().numpy(), oz0) and np.array_equal(gz1.cpu().numpy(), oz1)
    dt = render_depth(configs.c1_scene(), p[4], Kt).astype(np.float32)
    pair.frame(dt, Kt, p[4])                         # allocation view at 24x20
    nvis = compare_visible(pair.g, pair.o, "tiny frame")
    assert nvis > 4 * 512
    gp, gn, op, on = pair.raycast(Kt, p[4])
    nhit2, flips2 = compare_raycast(gp, gn, op, on, "overflowing bins, visible list")
    compare_tables(pair.g, pair.o, "tiny frame")
    _log(f"bin overflow: allocated {n_alloc}, visible {nvis}, hits {nhit}/{nhit2}, flips {flips}/{flips2}")


def test_voxel_array_beyond_4_gib():
    """2^22 blocks (6 GiB of voxels): block indices are taken from the top of
    the free stack, so every voxel address lies past 4 GiB and the raycast
    runs its 64-bit-offset variant; results against the oracle (which holds
    the plain 2^14-block volume: block indices differ, values by position
    must not)."""
    from synth.configs import VolumeParams
    import paper_1708_00783_amd as T
    from oracle import oracle as O
    vp = configs.C1_VOLUME
    big = VolumeParams(vp.voxel_size, vp.mu, vp.max_w, vp.n_buckets, vp.n_excess, 1 << 22)
    d, p, K, _ = configs.c1_frames(4)
    _log("case c1 with a 6 GiB voxel array")
    g = T.Volume(big, K.width, K.height)
    o = O.Volume.from_params(vp)
    for k in range(4):
        g.frame(to_device(d[k]), K, p[k])
        o.alloc_and_visible(d[k], K.as_array(), p[k])
        o.integrate(d[k], K.as_array(), p[k])
        compare_visible(g, o, f"big frame {k}")
        compare_tables(g, o, f"big frame {k}")
        gp, gn = g.raycast(p[k], K)
        op, on = o.raycast(K.width, K.height, K.as_array(), p[k])
        nhit, flips = compare_raycast(gp.cpu().numpy(), gn.cpu().numpy(), op, on, f"big frame {k}")
        _log(f"big frame {k}: hits {nhit} flips {flips}")
    _, _, ptr = g.entries()
    assert int(ptr[ptr >= 0].min()) * 1536 > (1 << 32)
    gp, gn = g.raycast(p[0], K)                    # another view
    op, on = o.raycast(K.width, K.height, K.as_array(), p[0], blocks="all")
    compare_raycast(gp.cpu().numpy(), gn.cpu().numpy(), op, on, "big, other view")
