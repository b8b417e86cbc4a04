"""CPU oracle of marching-cubes meshing of the voxel-hashed volume.

TEST INFRASTRUCTURE ONLY: tests/, the smoke check and the bench's CPU
baseline may use this module; the library never does, and nothing here is
shared with it (the library derives its own case table).

The paper's meshing engine turns the fused volume into a triangle mesh by
the Marching-Cubes algorithm of Lorensen and Cline (Sec. 4, the meshing
engine; Sec. 6, createMeshingEngine).  The paper gives no further detail.
Reading used here (each also in the design notes):

  * cells: every voxel cell whose 8 corner voxels (x..x+1, y..y+1, z..z+1,
    corners possibly in neighbouring blocks) are all observed (weight > 0);
    a corner is inside when its stored SDF is negative (F < 0, the same
    decision as the raycast's).
  * vertices: one per active cell edge, at the zero crossing of the linear
    interpolation of F between its two corners, t = F0 / (F0 - F1) from the
    lower corner, F = s / 32767; world position = voxel coordinates x voxel
    size (lattice points at p v, no half-voxel offset).
  * case table: derived, not tabulated: on each cube face the active edges are
    paired into segments (two active edges: one segment; four, the ambiguous
    face: each inside corner is cut off by the segment joining its two
    edges); the segments close into loops; each loop is oriented so that its
    normal points from the inside corners to the outside ones (towards free
    space) and fanned into triangles from its smallest edge index.  The face
    rule depends only on the face, so neighbouring cells agree on shared
    faces and the mesh is closed where every cell is observed.

Corner c of a cell is at (c & 1, c >> 1 & 1, c >> 2 & 1); edge e = 4 a + k runs
along axis a from the k-th corner (ascending) whose bit a is 0.
"""
from __future__ import annotations

import numpy as np

CORNER_POS = np.array([[(c >> 0) & 1, (c >> 1) & 1, (c >> 2) & 1] for c in range(8)], np.float64)


def _edges():
    out = []
    for a in range(3):
        for c in range(8):
            if not (c >> a) & 1:
                out.append((c, c | (1 << a), a))
    return out


EDGES = _edges()


def _faces():
    out = []
    for a in range(3):
        for s in (0, 1):
            corners = [c for c in range(8) if ((c >> a) & 1) == s]
            edges = [e for e, (c0, c1, ax) in enumerate(EDGES)
                     if ax != a and ((c0 >> a) & 1) == s and ((c1 >> a) & 1) == s]
            out.append((corners, edges))
    return out


FACES = _faces()


def cell_loops(mask: int) -> list:
    """oriented loops of edge indices for the inside-corner set `mask`"""
    inside = [(mask >> c) & 1 for c in range(8)]
    active = {e for e, (c0, c1, _) in enumerate(EDGES) if inside[c0] != inside[c1]}
    adj = {e: [] for e in active}
    for corners, fedges in FACES:
        fa = [e for e in fedges if e in active]
        if len(fa) == 2:
            pairs = [(fa[0], fa[1])]
        elif len(fa) == 4:
            pairs = []
            for c in corners:
                if inside[c]:
                    inc = [e for e in fa if c in EDGES[e][:2]]
                    pairs.append((inc[0], inc[1]))
        else:
            pairs = []
        for a, b in pairs:
            adj[a].append(b)
            adj[b].append(a)
    loops, seen = [], set()
    for e0 in sorted(active):
        if e0 in seen:
            continue
        loop, prev, cur = [e0], None, e0
        seen.add(e0)
        while True:
            nxt = adj[cur][0] if adj[cur][0] != prev else adj[cur][1]
            if nxt == e0:
                break
            loop.append(nxt)
            seen.add(nxt)
            prev, cur = cur, nxt
        # orientation: the polygon normal (Newell, on edge midpoints) must point
        # from the loop's inside corners towards its outside corners
        P = [CORNER_POS[EDGES[e][0]] + 0.5 * (CORNER_POS[EDGES[e][1]] - CORNER_POS[EDGES[e][0]]) for e in loop]
        n = np.zeros(3)
        for i in range(len(P)):
            n += np.cross(P[i], P[(i + 1) % len(P)])
        d = np.zeros(3)
        for e in loop:
            c0, c1, _ = EDGES[e]
            d += (CORNER_POS[c1] - CORNER_POS[c0]) * (1.0 if inside[c0] else -1.0)
        if float(n @ d) < 0:
            loop = [loop[0]] + loop[1:][::-1]
        loops.append(loop)
    return loops


def cell_triangles(mask: int) -> list:
    """triangles (edge-index triples) of the inside-corner set `mask`"""
    tris = []
    for loop in cell_loops(mask):
        for i in range(1, len(loop) - 1):
            tris.append((loop[0], loop[i], loop[i + 1]))
    return tris


TABLE = [cell_triangles(m) for m in range(256)]

KEY_OFF = 1 << 19


def edge_key(gx, gy, gz, axis):
    """64-bit key of the cell edge starting at global voxel (gx, gy, gz) along axis"""
    return (((int(gx) + KEY_OFF) << 42) | ((int(gy) + KEY_OFF) << 22) | ((int(gz) + KEY_OFF) << 2) | int(axis))


def mesh(block_pos, sdf, weight, voxel_size: float):
    """Triangles of the volume given as block positions (n, 3), SDF shorts and
    weights (n, 512) with in-block index lx + 8 ly + 64 lz.  Returns
    (vertices (m, 3, 3) float64 world metres, keys (m, 3) int64 edge keys) in
    a deterministic order (blocks as given, cells x-fastest, table order)."""
    block_pos = np.asarray(block_pos, np.int64).reshape(-1, 3)
    index = {tuple(p): i for i, p in enumerate(block_pos)}
    sdf = np.asarray(sdf, np.int16).reshape(-1, 8, 8, 8)      # [z][y][x]
    weight = np.asarray(weight, np.uint8).reshape(-1, 8, 8, 8)
    verts, keys = [], []
    for b, (bx, by, bz) in enumerate(block_pos):
        S = np.zeros((9, 9, 9), np.int32)                       # [z][y][x] over the block and +1 halo
        Wt = np.zeros((9, 9, 9), np.int32)
        for dz in (0, 1):
            for dy in (0, 1):
                for dx in (0, 1):
                    j = index.get((bx + dx, by + dy, bz + dz))
                    if j is None:
                        continue
                    zs = slice(0, 8) if dz == 0 else slice(0, 1)
                    ys = slice(0, 8) if dy == 0 else slice(0, 1)
                    xs = slice(0, 8) if dx == 0 else slice(0, 1)
                    tz = slice(0, 8) if dz == 0 else slice(8, 9)
                    ty = slice(0, 8) if dy == 0 else slice(8, 9)
                    tx = slice(0, 8) if dx == 0 else slice(8, 9)
                    S[tz, ty, tx] = sdf[j][zs, ys, xs]
                    Wt[tz, ty, tx] = weight[j][zs, ys, xs]
        # corner c of cell (lz, ly, lx) is S[lz + cz, ly + cy, lx + cx]
        cs = np.stack([S[(c >> 2) & 1:8 + ((c >> 2) & 1), (c >> 1) & 1:8 + ((c >> 1) & 1), c & 1:8 + (c & 1)]
                       for c in range(8)])
        cw = np.stack([Wt[(c >> 2) & 1:8 + ((c >> 2) & 1), (c >> 1) & 1:8 + ((c >> 1) & 1), c & 1:8 + (c & 1)]
                       for c in range(8)])
        case = sum((cs[c] < 0).astype(np.int32) << c for c in range(8))
        live = (cw > 0).all(axis=0) & (case != 0) & (case != 255)
        for lz, ly, lx in np.argwhere(live):                   # cells x-fastest
            m = int(case[lz, ly, lx])
            g0 = np.array([bx * 8 + lx, by * 8 + ly, bz * 8 + lz], np.int64)
            for tri in TABLE[m]:
                tv, tk = [], []
                for e in tri:
                    c0, c1, a = EDGES[e]
                    f0 = float(cs[c0][lz, ly, lx]) / 32767.0
                    f1 = float(cs[c1][lz, ly, lx]) / 32767.0
                    t = f0 / (f0 - f1)
                    g = g0 + CORNER_POS[c0].astype(np.int64)
                    p = g.astype(np.float64)
                    p[a] += t
                    tv.append(p * voxel_size)
                    tk.append(edge_key(g[0], g[1], g[2], a))
                verts.append(tv)
                keys.append(tk)
    if not verts:
        return np.zeros((0, 3, 3)), np.zeros((0, 3), np.int64)
    return np.array(verts, np.float64), np.array(keys, np.int64)
