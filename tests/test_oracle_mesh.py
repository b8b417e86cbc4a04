"""Pins of the marching-cubes oracle against what the geometry fixes: the
derived case table (0 and 255 empty, a lone corner cut by one triangle on its
three edges, every active edge used once, loops of at least three edges,
consistent orientation), a plane reproduced exactly by the linear
interpolation, a sphere meshed into a closed, consistently oriented manifold
of genus 0 whose vertices lie on the sphere, whose area and enclosed volume
match the closed forms, and unobserved voxels leaving no triangles."""
import itertools

import numpy as np

from oracle import mesh as M


def _volume(fn, lo, hi, observed=None):
    """blocks covering voxel box [lo, hi) with s = trunc(F * 32767) of F = clip(fn(x, y, z)),
    weight 1 (0 where observed(x, y, z) is False)"""
    blo = np.floor_divide(lo, 8)
    bhi = -np.floor_divide(-np.asarray(hi), 8)
    pos, sdf, w = [], [], []
    lz, ly, lx = np.meshgrid(np.arange(8), np.arange(8), np.arange(8), indexing="ij")
    for bx, by, bz in itertools.product(range(blo[0], bhi[0]), range(blo[1], bhi[1]), range(blo[2], bhi[2])):
        X, Y, Z = bx * 8 + lx, by * 8 + ly, bz * 8 + lz
        F = np.clip(fn(X.astype(np.float64), Y.astype(np.float64), Z.astype(np.float64)), -1.0, 1.0)
        pos.append((bx, by, bz))
        sdf.append(np.trunc(F * 32767).astype(np.int16).reshape(-1))
        ww = np.ones_like(F, np.uint8) if observed is None else observed(X, Y, Z).astype(np.uint8)
        w.append(ww.reshape(-1))
    return np.array(pos), np.array(sdf), np.array(w)


def test_case_table_from_its_definition():
    assert M.TABLE[0] == [] and M.TABLE[255] == []
    for c in range(8):
        tris = M.TABLE[1 << c]
        assert len(tris) == 1
        assert sorted(tris[0]) == sorted(e for e, (a, b, _) in enumerate(M.EDGES) if c in (a, b))
    for m in range(256):
        inside = [(m >> c) & 1 for c in range(8)]
        active = {e for e, (a, b, _) in enumerate(M.EDGES) if inside[a] != inside[b]}
        loops = M.cell_loops(m)
        used = [e for lp in loops for e in lp]
        assert sorted(used) == sorted(active) and len(used) == len(set(used)), m
        assert all(len(lp) >= 3 for lp in loops)
        assert len(M.TABLE[m]) == sum(len(lp) - 2 for lp in loops)


def test_plane_is_reproduced_exactly():
    z0 = 12.37

    def fn(x, y, z):
        return (z - z0) * 0.1
    pos, sdf, w = _volume(fn, (0, 0, 0), (24, 16, 24))
    V, K = M.mesh(pos, sdf, w, 0.005)
    # cells crossing the plane: x in 0..22, y in 0..14 (the +1 corner must exist), two triangles each
    assert len(V) == 2 * 23 * 15
    # vertices on the plane up to the short quantisation of F (1 / 32767 over a slope of 0.1 per voxel)
    assert np.abs(V[..., 2] / 0.005 - z0).max() < 1e-3
    n = np.cross(V[:, 1] - V[:, 0], V[:, 2] - V[:, 0])
    assert np.all(n[:, 2] > 0)                        # facing +z, towards F > 0


def test_sphere_is_a_closed_oriented_genus0_surface():
    c, R = np.array([20.3, 19.7, 20.1]), 9.6

    def fn(x, y, z):
        return (np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2) - R) * 0.25
    pos, sdf, w = _volume(fn, (0, 0, 0), (40, 40, 40))
    V, K = M.mesh(pos, sdf, w, 1.0)
    assert len(V) > 1000
    # every directed mesh edge appears once and its reverse once: closed and consistently oriented
    directed = {}
    for k in K:
        for i in range(3):
            e = (int(k[i]), int(k[(i + 1) % 3]))
            assert e not in directed
            directed[e] = 1
    assert all((b, a) in directed for a, b in directed)
    nv = len({int(x) for x in K.reshape(-1)})
    ne = len(directed) // 2
    assert nv - ne + len(K) == 2                       # Euler characteristic of a sphere
    r = np.linalg.norm(V.reshape(-1, 3) - c, axis=1)
    assert np.abs(r - R).max() < 0.03                  # linear interpolation of a curved surface
    n = np.cross(V[:, 1] - V[:, 0], V[:, 2] - V[:, 0])
    area = 0.5 * np.linalg.norm(n, axis=1).sum()
    vol = np.einsum("ij,ij->i", V[:, 0] - c, n).sum() / 6.0
    assert abs(area / (4 * np.pi * R * R) - 1) < 0.01
    assert abs(vol / (4 / 3 * np.pi * R ** 3) - 1) < 0.01       # positive: normals point outwards


def test_unobserved_voxels_leave_no_triangles():
    c, R = np.array([20.3, 19.7, 20.1]), 9.6

    def fn(x, y, z):
        return (np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2) - R) * 0.25

    def obs(x, y, z):
        return z < 22
    pos, sdf, w = _volume(fn, (0, 0, 0), (40, 40, 40), obs)
    V, K = M.mesh(pos, sdf, w, 1.0)
    assert len(V) > 500
    assert V[..., 2].max() <= 21.0 + 1e-9              # every cell needs all 8 corners observed
    # the open rim: edges used by one triangle only, all at the last observed cell layer
    directed = {}
    for k in K:
        for i in range(3):
            directed[(int(k[i]), int(k[(i + 1) % 3]))] = 1
    rim = [e for e in directed if (e[1], e[0]) not in directed]
    assert len(rim) > 20
    z_of = {int(x): z for x, z in zip(K.reshape(-1), V.reshape(-1, 3)[:, 2])}
    assert all(z_of[a] >= 20.0 and z_of[b] >= 20.0 for a, b in rim)
