"""Persistence of a volume (tf_save / tf_load) and the camera depth of
raycast hits (tf_camera_depth), through the C ABI.

A loaded volume is the saved one: hash entries (positions, chain links,
block indices), visible list, voxels and counters identical; a raycast from
the same pose gives bit-identical points and normals; fusing the same next
frame into both gives the same map (by position) and the same raycast.  With
swapping, the host store's blocks come back too.  A file of other parameters
is refused and leaves the volume untouched."""
import numpy as np
import pytest

from gpu_helpers import to_device
from synth import configs, look_at

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, flush=True)


def _fused(vp, frames, K, swap=0):
    import paper_1708_00783_amd as T
    d, p = frames
    g = T.Volume(vp, K.width, K.height, swap_transfer_blocks=swap)
    for k in range(len(d)):
        g.frame(to_device(d[k]), K, p[k])
    return g


def _same_tables(a, b):
    pa, oa, ra = a.entries()
    pb, ob, rb = b.entries()
    assert np.array_equal(pa, pb) and np.array_equal(oa, ob) and np.array_equal(ra, rb)
    assert np.array_equal(a.visible(), b.visible())
    for x, y in zip(a.voxels_by_position(), b.voxels_by_position()):
        assert np.array_equal(x, y)


def test_save_load_round_trip(tmp_path):
    import paper_1708_00783_amd as T
    d, p, K, _ = configs.c1_frames(6)
    _log("case save/load c1, 5 frames")
    a = _fused(configs.C1_VOLUME, (d[:5], p[:5]), K)
    path = str(tmp_path / "c1.tsdfvol")
    a.save(path)
    b = T.Volume(configs.C1_VOLUME, K.width, K.height)
    b.load(path)
    _same_tables(a, b)
    sa, sb = a.stats(), b.stats()
    assert sa == sb, (sa, sb)
    # another view (every block feeds the search range on both sides)
    pa, na = a.raycast(p[0], K)
    pb, nb = b.raycast(p[0], K)
    assert torch_equal(pa, pb) and torch_equal(na, nb)
    assert (pa.cpu().numpy()[..., 3] == 1).sum() > 1000
    # integration needs an allocation first on a loaded volume
    with pytest.raises(T.TsdfError):
        b.integrate(to_device(d[5]), p[5])
    # the next frame: same map by position, same raycast
    for v in (a, b):
        v.frame(to_device(d[5]), K, p[5])
    for x, y in zip(a.voxels_by_position(), b.voxels_by_position()):
        assert np.array_equal(x, y)
    pa, na = a.raycast(p[5], K)
    pb, nb = b.raycast(p[5], K)
    assert torch_equal(pa, pb) and torch_equal(na, nb)
    # the saved file holds only the blocks in use, not the whole block array
    import os
    n_alloc = a.stats()["n_allocated"]
    assert os.path.getsize(path) < configs.C1_VOLUME.n_blocks * 1536 // 4 + n_alloc * 1536 * 2


def torch_equal(x, y):
    import torch
    return bool(torch.equal(x, y))


def test_save_load_with_host_swapping(tmp_path):
    """blocks in the host store (swapped out) are saved and restored"""
    import paper_1708_00783_amd as T
    from test_gpu_swap import _state
    d, p, K, _ = configs.c1_frames(4)
    a = _fused(configs.C1_VOLUME, (d[:3], p[:3]), K, swap=1 << 12)
    sky = look_at([0.0, 0.0, 2.0], [0.0, 0.0, 5.0], up=(0.0, 1.0, 0.0)).astype(np.float32)
    a.alloc_and_visible(to_device(np.zeros_like(d[0])), K, sky)
    a.swap_out()
    assert a.stats()["n_swapped_out"] > 100
    path = str(tmp_path / "swap.tsdfvol")
    a.save(path)
    b = T.Volume(configs.C1_VOLUME, K.width, K.height, swap_transfer_blocks=1 << 12)
    b.load(path)
    _same_tables(a, b)
    sa, sb = _state(vol_g=a), _state(vol_g=b)
    assert sa.keys() == sb.keys()
    for key in sa:
        assert np.array_equal(sa[key][0], sb[key][0]) and np.array_equal(sa[key][1], sb[key][1])
    # both swap the same blocks back in when the camera returns
    for v in (a, b):
        v.frame(to_device(d[3]), K, p[3])
    assert a.stats()["n_swapped_in"] == b.stats()["n_swapped_in"] > 0
    for x, y in zip(a.voxels_by_position(), b.voxels_by_position()):
        assert np.array_equal(x, y)


def test_load_refuses_other_parameters_and_bad_files(tmp_path):
    import paper_1708_00783_amd as T
    from synth.configs import VolumeParams
    d, p, K, _ = configs.c1_frames(2)
    a = _fused(configs.C1_VOLUME, (d[:2], p[:2]), K)
    path = str(tmp_path / "a.tsdfvol")
    a.save(path)
    vp = configs.C1_VOLUME
    other = T.Volume(VolumeParams(vp.voxel_size, vp.mu, vp.max_w, vp.n_buckets, vp.n_excess, vp.n_blocks // 2),
                     K.width, K.height)
    other.frame(to_device(d[0]), K, p[0])
    before = other.allocated_positions()
    with pytest.raises(T.TsdfError, match="file error"):
        other.load(path)
    assert np.array_equal(other.allocated_positions(), before)   # untouched
    with pytest.raises(T.TsdfError, match="file error"):
        other.load(str(tmp_path / "missing.tsdfvol"))
    # a truncated file: refused, the volume is left empty
    raw = open(path, "rb").read()
    cut = str(tmp_path / "cut.tsdfvol")
    open(cut, "wb").write(raw[: len(raw) // 2])
    b = T.Volume(configs.C1_VOLUME, K.width, K.height)
    b.frame(to_device(d[0]), K, p[0])
    with pytest.raises(T.TsdfError, match="file error"):
        b.load(cut)
    assert len(b.allocated_positions()) == 0 and b.stats()["frames"] == 0


def test_camera_depth_of_raycast_points():
    """((m8 x + m9 y) + m10 z) + m11 at hits, 0 at misses: bit-identical to
    the same float32 expression evaluated on the host"""
    import torch
    import paper_1708_00783_amd as T
    d, p, K, _ = configs.c1_frames(3)
    g = _fused(configs.C1_VOLUME, (d, p), K)
    pts, _ = g.raycast(p[2], K)
    z = torch.empty((K.height, K.width), dtype=torch.float32, device="cuda")
    T.tf_camera_depth(pts, p[2], z)
    P = pts.cpu().numpy()
    M = np.asarray(p[2], np.float32)
    f = np.float32
    want = ((M[2, 0] * P[..., 0] + M[2, 1] * P[..., 1]) + M[2, 2] * P[..., 2]) + M[2, 3]
    want = np.where(P[..., 3] == 1, want, f(0)).astype(np.float32)
    got = z.cpu().numpy()
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    hit = P[..., 3] == 1
    assert hit.sum() > 1000
    # and it is the rendered depth up to the fusion's error (noiseless frames),
    # away from silhouettes, where a ray meets the surface behind the edge
    m = hit & (d[2] > 0)
    e = np.abs(got[m] - d[2][m])
    assert np.median(e) < 0.003 and (e > 0.02).mean() < 0.03
    # a ragged size, misses only
    pts2 = torch.zeros((7, 13, 4), dtype=torch.float32, device="cuda")
    z2 = torch.full((7, 13), 5.0, dtype=torch.float32, device="cuda")
    T.tf_camera_depth(pts2, p[2], z2)
    assert not z2.cpu().numpy().any()
