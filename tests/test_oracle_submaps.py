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
