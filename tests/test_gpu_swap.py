"""GPU parity of host swapping (Sec. 5): the same small device budget with
swapping after every frame, oracle vs HIP path.  Visible and device-resident
sets must agree frame by frame and the final voxels (device or host copy) by
position.  The transfer buffer is larger than any frame's candidate set, so
the selection of which blocks move does not depend on entry indices (those
differ between the two tables: excess slots are taken in a different order)."""
import numpy as np
import pytest

from gpu_helpers import to_device
from synth.configs import VolumeParams

pytestmark = pytest.mark.gpu


def _walk():
    import test_oracle_swap as S
    return S.walk_frames(40), S.K_SMALL, S.VP


def _state(vol_o=None, vol_g=None):
    res = {}
    if vol_o is not None:
        pos, _, ptr = vol_o.entries()
        dev = np.flatnonzero(ptr >= 0)
        sdf, w = vol_o.block_voxels(dev)
        for k, i in enumerate(dev):
            res[tuple(pos[i])] = (sdf[k], w[k])
        for i in np.flatnonzero(ptr == -1):
            res[tuple(pos[i])] = vol_o.host_block(i)
    else:
        pos, _, ptr = vol_g.entries()
        dev = np.flatnonzero(ptr >= 0)
        sdf, w = vol_g.block_voxels(dev)
        for k, i in enumerate(dev):
            res[tuple(pos[i])] = (sdf[k], w[k])
        out = np.flatnonzero(ptr == -1)
        hs, hw, has = vol_g.host_voxels(out)
        assert has.all()
        for k, i in enumerate(out):
            res[tuple(pos[i])] = (hs[k], hw[k])
    return res


# 2^21 buckets: the ordered swap-out selection scans 513 chunks of 4096
# entries, so its single-workgroup scan carries offsets across two passes of
# 256 chunks (the entries of the walk's blocks spread over all of them)
@pytest.mark.parametrize("n_buckets", [None, 1 << 21])
def test_swapping_parity_walk(n_buckets):
    from oracle import oracle as O
    import paper_1708_00783_amd as T
    frames, K, VP = _walk()
    nb = n_buckets or VP.n_buckets
    print(f"case swap walk, {nb} buckets", flush=True)
    budget = VolumeParams(VP.voxel_size, VP.mu, VP.max_w, nb, VP.n_excess, 5000)
    o = O.Volume.from_params(budget)
    o.enable_swap(4096)
    g = T.Volume(budget, K.width, K.height, swap_transfer_blocks=4096)
    tot_in = tot_out = 0
    for f, (depth, P) in enumerate(frames):
        o.alloc_and_visible(depth, K.as_array(), P)
        o.integrate(depth, K.as_array(), P)
        dd = to_device(depth)
        g.alloc_and_visible(dd, K, P)
        g.integrate(dd, P)
        st = g.stats()
        assert st["n_swapped_in"] == o.n_swapped_in, f
        tot_in += st["n_swapped_in"]
        mo = o.swap_out()
        g.swap_out()
        st = g.stats()
        assert st["n_swapped_out"] == mo, f
        tot_out += mo
        gp, _, gptr = g.entries()
        op, _, optr = o.entries()
        assert {tuple(x) for x in gp[gptr >= 0]} == {tuple(x) for x in op[optr >= 0]}, f
        assert {tuple(x) for x in gp[gptr == -1]} == {tuple(x) for x in op[optr == -1]}, f
        assert {tuple(x) for x in gp[g.visible()]} == {tuple(x) for x in op[o.visible()]}, f
    assert tot_out > 500 and tot_in > 50
    assert g.stats()["flags"] == 0 and o.flags == 0
    a = _state(vol_o=o)
    b = _state(vol_g=g)
    assert a.keys() == b.keys()
    for key in a:
        assert np.array_equal(a[key][1], b[key][1]), key
        assert np.abs(a[key][0].astype(int) - b[key][0].astype(int)).max() <= 1, key


def test_transfer_overflow_merge_parity():
    """tiny transfer buffer: host data waits while the device keeps fusing,
    then merges (secondary integration) -- same weights, SDF within 1 LSB"""
    from oracle import oracle as O
    import paper_1708_00783_amd as T
    from synth import configs, look_at
    vp = configs.C1_VOLUME
    K = configs.C1_INTR
    pose = np.eye(4, dtype=np.float32)
    plane = lambda z: np.full((K.height, K.width), z, np.float32)
    sky = look_at([0.0, 0.0, 0.0], [0.0, 0.0, -5.0], up=(0.0, 1.0, 0.0)).astype(np.float32)
    o = O.Volume.from_params(vp)
    o.enable_swap(40)
    g = T.Volume(vp, K.width, K.height, swap_transfer_blocks=40)
    seq = [(plane(1.0), pose, True)] * 3 + [(plane(0.0), sky, False)] + [(plane(1.02), pose, True)] * 2 + \
          [(plane(0.0), pose, False)] * 60
    for k, (d, P, integ) in enumerate(seq):
        o.alloc_and_visible(d, K.as_array(), P)
        dd = to_device(d)
        g.alloc_and_visible(dd, K, P)
        assert g.stats()["n_swapped_in"] == o.n_swapped_in, k
        if integ:
            o.integrate(d, K.as_array(), P)
            g.integrate(dd, P)
        if k == 3:
            while o.swap_out():
                pass
            for _ in range(200):
                g.swap_out()
                if g.stats()["n_swapped_out"] == 0:
                    break
    assert g.stats()["flags"] & 8 and o.flags & 8
    a = _state(vol_o=o)
    b = _state(vol_g=g)
    assert a.keys() == b.keys()
    for key in a:
        assert np.array_equal(a[key][1], b[key][1]), key
        assert np.abs(a[key][0].astype(int) - b[key][0].astype(int)).max() <= 1, key


def test_swap_out_merges_pending_host_copies():
    """Blocks swapped out, then touched again: they get fresh device blocks
    at once while their host copies come back at most 40 per frame.  Swapping
    everything out again two frames later catches most of them with the host
    copy still pending: the secondary integration (Sec. 5) then fuses the
    device copy into the store copy on the device.  Final voxels by position
    (device or host copy): weights bit-exact, SDF within 1 LSB of the oracle."""
    from oracle import oracle as O
    import paper_1708_00783_amd as T
    from synth import configs, look_at
    vp = configs.C1_VOLUME
    K = configs.C1_INTR
    pose = np.eye(4, dtype=np.float32)
    plane = lambda z: np.full((K.height, K.width), z, np.float32)
    sky = look_at([0.0, 0.0, 0.0], [0.0, 0.0, -5.0], up=(0.0, 1.0, 0.0)).astype(np.float32)
    o = O.Volume.from_params(vp)
    o.enable_swap(40)
    g = T.Volume(vp, K.width, K.height, swap_transfer_blocks=40)
    seq = [(plane(1.0), pose, True)] * 3 + [(plane(0.0), sky, False)] + [(plane(1.02), pose, True)] * 2 + \
          [(plane(0.0), sky, False)] + [(plane(0.0), pose, False)] * 3
    pending_at_swap = 0
    for k, (d, P, integ) in enumerate(seq):
        o.alloc_and_visible(d, K.as_array(), P)
        dd = to_device(d)
        g.alloc_and_visible(dd, K, P)
        assert g.stats()["n_swapped_in"] == o.n_swapped_in, k
        if integ:
            o.integrate(d, K.as_array(), P)
            g.integrate(dd, P)
        if k in (3, 6):
            if k == 6:
                _, _, ptr = g.entries()
                dev = np.flatnonzero(ptr >= 0).astype(np.int32)
                pending_at_swap = int(g.host_voxels(dev)[2].sum())
            while o.swap_out():
                pass
            for _ in range(500):
                g.swap_out()
                if g.stats()["n_swapped_out"] == 0:
                    break
            _, _, ptr = g.entries()
            assert (ptr >= 0).sum() == 0, k
    assert pending_at_swap > 100, pending_at_swap
    a = _state(vol_o=o)
    b = _state(vol_g=g)
    assert a.keys() == b.keys()
    n_lsb = 0
    for key in a:
        assert np.array_equal(a[key][1], b[key][1]), key
        dsdf = np.abs(a[key][0].astype(int) - b[key][0].astype(int))
        assert dsdf.max() <= 1, key
        n_lsb += int((dsdf > 0).sum())
    print(f"pending host copies merged at swap-out: {pending_at_swap}; blocks {len(a)}; "
          f"1-LSB SDF differences {n_lsb}", flush=True)
