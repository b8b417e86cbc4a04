"""Pins for host swapping (Sec. 5).

* round trip: blocks swapped out to the host store and swapped back in (their
  device copies being fresh) come back bit-identical;
* a run with a small device budget and swapping every frame reproduces the
  voxels of an unbounded run exactly (device or host copy, by position),
  provided the transfer buffer is never full;
* the secondary-integration merge of two copies of one block is the weighted
  average of the two, pinned on a two-source closed form.
"""
import numpy as np

from synth import Intrinsics, configs, look_at, render_depth
from synth.configs import VolumeParams

K_SMALL = Intrinsics(60.0, 60.0, 40.0, 30.0, 80, 60)
VP = VolumeParams(0.02, 0.08, 100, 1 << 14, 1 << 12, 1 << 13)


def walk_frames(n=60):
    """out-and-back walk through the first rooms of the multi-room layout"""
    scene, _ = configs.c3_layout(0)
    poses = configs.c3_poses(1500, 0)
    idx = list(range(0, 10 * n, 10)) + list(range(10 * n - 10, -1, -10))
    out = []
    for i in idx:
        P = poses[i].astype(np.float32)
        out.append((render_depth(scene, poses[i], K_SMALL).astype(np.float32), P))
    return out


def state_by_position(vol):
    """{position: (sdf, w)} from device blocks and the host store"""
    pos, _, ptr = vol.entries()
    res = {}
    dev = np.flatnonzero(ptr >= 0)
    sdf, w = vol.block_voxels(dev)
    for k, i in enumerate(dev):
        res[tuple(pos[i])] = (sdf[k], w[k])
    for i in np.flatnonzero(ptr == -1):
        hb = vol.host_block(i)
        assert hb is not None, "swapped-out entry without host data"
        res[tuple(pos[i])] = hb
    return res


def test_round_trip_is_identity(oracle_mod):
    d, p, K, _ = configs.c1_frames(3)
    vol = oracle_mod.Volume.from_params(configs.C1_VOLUME)
    vol.enable_swap(1 << 14)
    for k in range(3):
        vol.alloc_and_visible(d[k], K.as_array(), p[k])
        vol.integrate(d[k], K.as_array(), p[k])
    before = state_by_position(vol)
    # an empty frame looking at the sky: nothing stays visible, all go out
    sky = look_at([0.0, 0.0, 2.0], [0.0, 0.0, 5.0], up=(0.0, 1.0, 0.0)).astype(np.float32)
    vol.alloc_and_visible(np.zeros_like(d[0]), K.as_array(), sky)
    moved = vol.swap_out()
    pos, _, ptr = vol.entries()
    assert moved == len(before) and (ptr >= 0).sum() == 0
    assert vol.n_free_blocks == configs.C1_VOLUME.n_blocks
    assert state_by_position(vol).keys() == before.keys()
    # the original frame brings every touched block back from the host
    vol.alloc_and_visible(d[2], K.as_array(), p[2])
    assert vol.n_swapped_in > 0
    after = state_by_position(vol)
    for key, (s, w) in before.items():
        assert np.array_equal(after[key][0], s) and np.array_equal(after[key][1], w)
    assert vol.flags == 0


def test_budget_with_swapping_equals_unbounded(oracle_mod):
    frames = walk_frames(40)
    big = oracle_mod.Volume.from_params(VP)
    small = oracle_mod.Volume(VP.voxel_size, VP.mu, VP.max_w, VP.n_buckets, VP.n_excess, 5000)
    small.enable_swap(4096)
    swapped_in = swapped_out = 0
    for depth, P in frames:
        for vol in (big, small):
            vol.alloc_and_visible(depth, K_SMALL.as_array(), P)
            vol.integrate(depth, K_SMALL.as_array(), P)
        swapped_in += small.n_swapped_in
        swapped_out += small.swap_out()
        # the visible sets agree frame by frame
        bp, _, _ = big.entries()
        sp, _, _ = small.entries()
        assert {tuple(x) for x in bp[big.visible()]} == {tuple(x) for x in sp[small.visible()]}
    assert small.flags == 0 and big.flags == 0
    assert swapped_out > 500 and swapped_in > 50
    a = state_by_position(big)
    b = state_by_position(small)
    assert a.keys() == b.keys()
    for key in a:
        assert np.array_equal(a[key][0], b[key][0]) and np.array_equal(a[key][1], b[key][1]), key


def test_secondary_integration_matches_sequential_fusion(oracle_mod):
    """Host data that could not be transferred while the device kept fusing
    is merged later (Sec. 5, O3): the weighted average of the two copies must
    equal fusing all frames in sequence -- weights exactly, SDF within 2 LSB
    (the two evaluation orders round differently)."""
    vp = configs.C1_VOLUME
    K = configs.C1_INTR
    pose = np.eye(4, dtype=np.float32)
    plane = lambda z: np.full((K.height, K.width), z, np.float32)
    seq = [(1.0, 3), (1.02, 2)]
    ref = oracle_mod.Volume.from_params(vp)
    for z, n in seq:
        for _ in range(n):
            ref.alloc_and_visible(plane(z), K.as_array(), pose)
            ref.integrate(plane(z), K.as_array(), pose)
    vol = oracle_mod.Volume.from_params(vp)
    vol.enable_swap(40)                       # far fewer than the blocks in view
    for _ in range(3):
        vol.alloc_and_visible(plane(1.0), K.as_array(), pose)
        vol.integrate(plane(1.0), K.as_array(), pose)
    n_blocks = len(vol.allocated_positions())
    sky = look_at([0.0, 0.0, 0.0], [0.0, 0.0, -5.0], up=(0.0, 1.0, 0.0)).astype(np.float32)
    vol.alloc_and_visible(plane(0.0), K.as_array(), sky)
    out = 0
    while True:                               # empty the device, 40 blocks per call
        moved = vol.swap_out()
        out += moved
        if moved == 0:
            break
    assert out == n_blocks
    merged = 0
    for _ in range(2):
        vol.alloc_and_visible(plane(1.02), K.as_array(), pose)
        merged += vol.n_swapped_in
        vol.integrate(plane(1.02), K.as_array(), pose)
    assert vol.flags & 8                       # the transfer buffer overflowed
    for _ in range(200):                      # empty frames in view drain the backlog
        vol.alloc_and_visible(plane(0.0), K.as_array(), pose)
        merged += vol.n_swapped_in
        if vol.n_swapped_in == 0:
            break
    assert merged == n_blocks
    a = state_by_position(ref)
    b = state_by_position(vol)
    assert a.keys() == b.keys()
    late = 0
    for key in a:
        assert np.array_equal(a[key][1], b[key][1]), key
        d = np.abs(a[key][0].astype(int) - b[key][0].astype(int))
        assert d.max() <= 2, key
        late += int(d.max() > 0)
    assert late > 0                           # some blocks really went through the merge
