"""Pins for the combined field of rigid submaps (Sec. 7.2).

* one submap with the identity pose reduces exactly to the plain raycast;
* k identical copies with identity poses give the plain surface (the weighted
  average of equal values), up to float rounding of the average;
* a submap whose voxel grid is rotated and shifted against the world (frames
  fused with the camera composed with the submap pose) reproduces the
  analytic surface -- a transposed or inverted pose would misplace it;
* the composed camera of a submap is M_d P^-1 (closed form in float64).
"""
import numpy as np

from synth import analytic_sdf, configs, look_at

K = configs.C1_INTR
VP = configs.C1_VOLUME


def _plain(oracle_mod, n=6):
    d, p, intr, scene = configs.c1_frames(n)
    vol = oracle_mod.Volume.from_params(VP)
    for k in range(n):
        vol.alloc_and_visible(d[k], intr.as_array(), p[k])
        vol.integrate(d[k], intr.as_array(), p[k])
    return vol, d, p, scene


def test_compose_closed_form(oracle_mod):
    rng = np.random.default_rng(0)
    A = look_at([1.0, -2.0, 1.5], [0.2, 0.3, 0.1])
    P = look_at([-0.7, 0.4, 2.0], [1.0, 1.0, 0.0])
    got = oracle_mod.compose(A.astype(np.float32), P.astype(np.float32)).astype(np.float64)
    want = A.astype(np.float32).astype(np.float64) @ np.linalg.inv(P.astype(np.float32).astype(np.float64))
    assert np.abs(got - want).max() < 1e-6
    # identity pose: the composition is exact
    A32 = A.astype(np.float32)
    assert np.array_equal(oracle_mod.compose(A32, np.eye(4, dtype=np.float32)), A32)


def test_single_identity_submap_equals_plain(oracle_mod):
    vol, d, p, _ = _plain(oracle_mod)
    V = p[-1]
    pts0, nrm0 = vol.raycast(K.width, K.height, K.as_array(), V, blocks="all")
    m = oracle_mod.Multi([vol], [np.eye(4, dtype=np.float32)])
    pts1, nrm1 = m.raycast(K.width, K.height, K.as_array(), V)
    assert np.array_equal(pts0, pts1) and np.array_equal(nrm0, nrm1)
    z0, z1 = vol.range_image(K.width, K.height, K.as_array(), V, blocks="all")
    m0, m1 = m.range_image(K.width, K.height, K.as_array(), V)
    assert np.array_equal(z0, m0) and np.array_equal(z1, m1)


def test_identical_copies_average_to_plain(oracle_mod):
    a, d, p, _ = _plain(oracle_mod)
    b, _, _, _ = _plain(oracle_mod)
    V = p[-1]
    pts0, _ = a.raycast(K.width, K.height, K.as_array(), V, blocks="all")
    m = oracle_mod.Multi([a, b], [np.eye(4, dtype=np.float32)] * 2)
    pts1, nrm1 = m.raycast(K.width, K.height, K.as_array(), V)
    h0 = pts0[..., 3] == 1
    h1 = pts1[..., 3] == 1
    assert (h0 != h1).mean() < 1e-3
    both = h0 & h1
    assert np.abs(pts0[both][:, :3] - pts1[both][:, :3]).max() < 1e-4


def test_rotated_submap_reproduces_analytic_surface(oracle_mod):
    d, p, intr, scene = configs.c1_frames(10)
    # submap frame: rotated 30 deg about z and shifted (world -> submap)
    c, s = np.cos(0.5236), np.sin(0.5236)
    P = np.eye(4)
    P[:3, :3] = [[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]]
    P[:3, 3] = [0.137, -0.081, 0.029]
    P = P.astype(np.float32)
    vol = oracle_mod.Volume.from_params(VP)
    m = oracle_mod.Multi([vol], [P])
    for k in range(10):
        m.integrate_frame(0, d[k], intr.as_array(), p[k])
    pts, nrm = m.raycast(K.width, K.height, K.as_array(), p[-1])
    hit = pts[..., 3] == 1
    assert hit.mean() > 0.5
    e = analytic_sdf(scene, pts[hit][:, :3])
    assert np.sqrt(np.mean(e ** 2)) < 0.5 * VP.voxel_size
    # the grid really is rotated: its blocks are not those of the plain map
    plain, _, _, _ = _plain(oracle_mod, 10)
    assert {tuple(x) for x in vol.allocated_positions()} != {tuple(x) for x in plain.allocated_positions()}


def _plane_submap(oracle_mod, z0, frames):
    """a volume fused from `frames` identical frames of the fronto-parallel
    plane z = z0 seen by the identity camera"""
    depth = np.full((K.height, K.width), z0, np.float32)
    pose = np.eye(4, dtype=np.float32)
    vol = oracle_mod.Volume.from_params(VP)
    for _ in range(frames):
        vol.alloc_and_visible(depth, K.as_array(), pose)
        vol.integrate(depth, K.as_array(), pose)
    return vol


def test_combined_field_is_weight_averaged(oracle_mod):
    """Reading R27 (the combined field of Sec. 7.2, normalised): submap A
    holds 9 observations of the plane z = 1.000 m, submap B 3 observations
    of z = 1.016 m, both with identity poses.  Inside both truncation bands
    F_A = (z_A - z) / mu and F_B = (z_B - z) / mu with weights 9 and 3, so
    the weighted mean field vanishes at z* = (9 z_A + 3 z_B) / 12 = 1.004 m.
    The raycast hit must sit there up to the plane raycast's own bound
    (refinement residual v (1 - dir_z)^2 plus quantisation).  Weighting by
    submap count puts the zero at 1.008 m, swapping the weights at 1.012 m,
    and an unnormalised sum (F scaled by 12) breaks the distance-scaled
    steps: each of these misses the bound by millimetres."""
    za, na, zb, nb = 1.000, 9, 1.016, 3
    a = _plane_submap(oracle_mod, za, na)
    b = _plane_submap(oracle_mod, zb, nb)
    # the premise: every voxel near z* carries exactly na (resp. nb) observations
    _, _, wa = a.voxels_by_position()
    _, _, wb = b.voxels_by_position()
    assert wa.max() == na and wb.max() == nb
    z_star = (na * za + nb * zb) / (na + nb)
    pose = np.eye(4, dtype=np.float32)
    m = oracle_mod.Multi([a, b], [pose, pose])
    pts, nrm = m.raycast(K.width, K.height, K.as_array(), pose)
    ys, xs = np.mgrid[0:K.height, 0:K.width]
    ax = (xs - K.cx) / K.fx
    by = (ys - K.cy) / K.fy
    dir_z = 1.0 / np.sqrt(ax * ax + by * by + 1.0)
    interior = (xs >= 6) & (xs < K.width - 6) & (ys >= 6) & (ys < K.height - 6)
    hit = pts[..., 3] == 1
    assert hit[interior].all()
    # each submap's stored F drifts by at most one truncation per frame
    quant = (na + nb) * VP.mu / 32767.0 + 1e-6
    bound = VP.voxel_size * (1 - dir_z) ** 2 + quant
    err = np.abs(pts[..., 2] - z_star)
    assert np.all(err[interior] <= bound[interior]), float(err[interior].max())
    # the alternatives are far outside the bound at every interior pixel
    for wrong in ((za + zb) / 2, (nb * za + na * zb) / (na + nb)):
        assert np.all(np.abs(pts[..., 2] - wrong)[interior] > bound[interior])
    assert np.all(nrm[interior] == np.array([0, 0, -1, 1], np.float32))


def test_partition_into_two_submaps_equals_plain(oracle_mod):
    """Two identity-posed submaps that partition the plain map's blocks
    (blocks with x < 0 in one, the rest in the other) give the plain raycast
    wherever a hit's trilinear reads and normal taps stay on one side of the
    cut: there a single submap contributes and the combined field is its
    field.  The union of their blocks is the plain map's, so the allocation
    test and the search range are the plain ones."""
    plain, d, p, _ = _plain(oracle_mod)
    pos, _, ptr = plain.entries()
    ids = np.flatnonzero(ptr >= 0)
    sdf, w = plain.block_voxels(ids)
    parts = [oracle_mod.Volume.from_params(VP), oracle_mod.Volume.from_params(VP)]
    for k, i in enumerate(ids):
        bx, byy, bz = (int(c) for c in pos[i])
        vol = parts[0] if bx < 0 else parts[1]
        e = vol.insert(bx, byy, bz)
        assert e >= 0
        vol.set_block_voxels(e, sdf[k], w[k])
    assert len(parts[0].allocated_positions()) > 50 and len(parts[1].allocated_positions()) > 50
    V = p[-1]
    pts0, nrm0 = plain.raycast(K.width, K.height, K.as_array(), V, blocks="all")
    eye = np.eye(4, dtype=np.float32)
    m = oracle_mod.Multi(parts, [eye, eye])
    z0, z1 = plain.range_image(K.width, K.height, K.as_array(), V, blocks="all")
    m0, m1 = m.range_image(K.width, K.height, K.as_array(), V)
    assert np.array_equal(z0, m0) and np.array_equal(z1, m1)
    pts1, nrm1 = m.raycast(K.width, K.height, K.as_array(), V)
    h0 = pts0[..., 3] == 1
    h1 = pts1[..., 3] == 1
    # world x of the cut in voxel units is 0; keep hits whose reads (cell, +-1
    # voxel normal taps, refinement) stay at least 3 voxels from it
    xv = pts0[..., 0] / VP.voxel_size
    away = h0 & (np.abs(xv) >= 3.0)
    assert away.sum() > 1000
    assert (h1[away]).mean() > 0.999
    both = away & h1
    dp = np.abs(pts0[both][:, :3] - pts1[both][:, :3]).max(axis=1)
    assert np.mean(dp <= 1e-4) > 0.99, float(np.mean(dp <= 1e-4))
    dn = np.abs(nrm0[both][:, :3] - nrm1[both][:, :3]).max(axis=1)
    assert np.mean(dn <= 1e-3) > 0.99


def test_masked_raycast_marches_only_the_masked_pixels(oracle_mod):
    """The mask only empties the other pixels' ranges: masked pixels equal the
    full raycast bit for bit, the others have no hit (used to sample pixels of
    large views)."""
    vol, d, p, _ = _plain(oracle_mod)
    m = oracle_mod.Multi([vol], [np.eye(4, dtype=np.float32)])
    V = p[-1]
    full_p, full_n = m.raycast(K.width, K.height, K.as_array(), V)
    mask = np.zeros((K.height, K.width), bool)
    mask.flat[np.random.default_rng(3).choice(K.width * K.height, 500, replace=False)] = True
    mp, mn = m.raycast(K.width, K.height, K.as_array(), V, mask=mask)
    assert np.array_equal(mp[mask], full_p[mask]) and np.array_equal(mn[mask], full_n[mask])
    assert not (mp[~mask][:, 3] == 1).any() and not (mn[~mask][:, 3] == 1).any()
    assert (full_p[mask][:, 3] == 1).sum() > 100
