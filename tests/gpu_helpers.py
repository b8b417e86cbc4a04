"""Shared helpers of the GPU parity tests: run the oracle and the HIP path on
the same frames and compare what the method fixes."""
from __future__ import annotations

import numpy as np

# parity bars (the method's stated tolerances)
SDF_LSB = 1            # stored short SDF
PT_TOL = 1e-4          # metres, raycast points
NRM_TOL = 1e-3         # raycast normals
HITMISS_FRAC = 1e-3    # hit/miss disagreement


def to_device(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def oracle_depth(depth):
    from oracle import oracle as O
    if depth.dtype == np.uint16:
        return O.depth_from_mm(depth)
    return np.ascontiguousarray(depth, np.float32)


def compare_tables(gv, ov, tag=""):
    """allocated sets equal; voxels: weights bit-exact, SDF within 1 LSB"""
    gp = gv.allocated_positions()
    op = ov.allocated_positions()
    assert gp.shape == op.shape and np.array_equal(gp, op), \
        f"{tag}: allocated sets differ ({len(gp)} gpu vs {len(op)} oracle)"
    g_pos, g_sdf, g_w = gv.voxels_by_position()
    o_pos, o_sdf, o_w = ov.voxels_by_position()
    assert np.array_equal(g_pos, o_pos)
    wdiff = int((g_w != o_w).sum())
    assert wdiff == 0, f"{tag}: {wdiff} voxel weights differ"
    sd = np.abs(g_sdf.astype(np.int32) - o_sdf.astype(np.int32))
    assert sd.max(initial=0) <= SDF_LSB, f"{tag}: SDF differs by {sd.max()} LSB"
    return len(gp), int((sd > 0).sum())


def compare_visible(gv, ov, tag=""):
    gpos, _, _ = gv.entries()
    opos, _, _ = ov.entries()
    gs = {tuple(p) for p in gpos[gv.visible()]}
    os_ = {tuple(p) for p in opos[ov.visible()]}
    assert gs == os_, f"{tag}: visible sets differ ({len(gs)} gpu vs {len(os_)} oracle, " \
                      f"{len(gs - os_)} extra, {len(os_ - gs)} missing)"
    return len(gs)


def compare_raycast(g_pts, g_nrm, o_pts, o_nrm, tag=""):
    gh = g_pts[..., 3] == 1
    oh = o_pts[..., 3] == 1
    flips = int((gh != oh).sum())
    assert flips <= HITMISS_FRAC * gh.size, f"{tag}: {flips} hit/miss disagreements"
    both = gh & oh
    if both.any():
        dp = np.abs(g_pts[both][:, :3] - o_pts[both][:, :3]).max()
        assert dp <= PT_TOL, f"{tag}: point error {dp}"
        gn = g_nrm[both]
        on = o_nrm[both]
        valid = (gn[:, 3] == 1) & (on[:, 3] == 1)
        assert int(((gn[:, 3] == 1) != (on[:, 3] == 1)).sum()) <= HITMISS_FRAC * gh.size
        if valid.any():
            dn = np.abs(gn[valid][:, :3] - on[valid][:, :3]).max()
            assert dn <= NRM_TOL, f"{tag}: normal error {dn}"
    return int(gh.sum()), flips


class Pair:
    """an oracle volume and a GPU volume fed the same frames"""

    def __init__(self, vp, W, H):
        from oracle import oracle as O
        import paper_1708_00783_amd as T
        self.o = O.Volume.from_params(vp)
        self.g = T.Volume(vp, W, H)

    def alloc(self, depth, intr, pose):
        self.o.alloc_and_visible(oracle_depth(depth), intr.as_array(), pose)
        self.g.alloc_and_visible(to_device(depth), intr, pose)
        self._last = (np.asarray(pose, np.float32).copy(),
                      (intr.fx, intr.fy, intr.cx, intr.cy, intr.width, intr.height))

    def integrate(self, depth, intr, pose):
        self.o.integrate(oracle_depth(depth), intr.as_array(), pose)
        self.g.integrate(to_device(depth), pose)

    def raycast(self, intr, pose):
        op, on = self.o.raycast(intr.width, intr.height, intr.as_array(), pose,
                                blocks=None if self._same(pose, intr) else "all")
        gp, gn = self.g.raycast(pose, intr)
        return gp.cpu().numpy(), gn.cpu().numpy(), op, on

    _last = None

    def _same(self, pose, intr):
        return self._last is not None and np.array_equal(self._last[0], np.asarray(pose, np.float32)) \
            and self._last[1] == (intr.fx, intr.fy, intr.cx, intr.cy, intr.width, intr.height)

    def frame(self, depth, intr, pose):
        self.alloc(depth, intr, pose)
        self.integrate(depth, intr, pose)
