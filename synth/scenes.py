"""Seeded synthetic scenes, camera trajectories and depth rendering.

Input generation only: nothing here performs any step of the fusion method
(allocation, integration, raycasting).  The same frames feed the CPU oracle
and the GPU library, so both sides see bit-identical inputs.

Conventions
-----------
* World frame: right-handed, z up, metres.
* Camera frame: x right, y down, z forward (the pinhole projection of the
  integration step in Sec. 4.3 of the paper, u = fx*x/z + cx, v = fy*y/z + cy).
* A pose is the 4x4 world->camera matrix M_d of Sec. 4.3, row-major.
* Depth is the camera-frame z of the first surface hit through the integer
  pixel coordinate (x, y), computed in float64 by exact ray/primitive
  intersection; 0 means no return.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Intrinsics:
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int

    def as_array(self) -> np.ndarray:
        return np.array([self.fx, self.fy, self.cx, self.cy], dtype=np.float32)


@dataclasses.dataclass
class Scene:
    """Union of solids; free space is inside every `rooms` box and outside
    every other primitive."""
    rooms: list = dataclasses.field(default_factory=list)      # (lo[3], hi[3]) inside-out boxes
    floors: list = dataclasses.field(default_factory=list)     # z = h, solid below
    spheres: list = dataclasses.field(default_factory=list)    # (centre[3], radius)
    boxes: list = dataclasses.field(default_factory=list)      # (centre[3], half[3], yaw)

    def n_primitives(self) -> int:
        return len(self.rooms) + len(self.floors) + len(self.spheres) + len(self.boxes)


# ----------------------------------------------------------------------------
# camera helpers
# ----------------------------------------------------------------------------

def look_at(eye, target, up=(0.0, 0.0, 1.0)) -> np.ndarray:
    """World->camera 4x4 (float64) for a camera at `eye` looking at `target`."""
    eye = np.asarray(eye, np.float64)
    target = np.asarray(target, np.float64)
    z = target - eye
    z /= np.linalg.norm(z)
    x = np.cross(z, np.asarray(up, np.float64))
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    R = np.stack([x, y, z])
    M = np.eye(4)
    M[:3, :3] = R
    M[:3, 3] = -R @ eye
    return M


def pixel_rays(intr: Intrinsics) -> np.ndarray:
    """Camera-frame ray directions with unit z, shape (H, W, 3), float64."""
    xs = (np.arange(intr.width, dtype=np.float64) - intr.cx) / intr.fx
    ys = (np.arange(intr.height, dtype=np.float64) - intr.cy) / intr.fy
    r = np.empty((intr.height, intr.width, 3))
    r[..., 0] = xs[None, :]
    r[..., 1] = ys[:, None]
    r[..., 2] = 1.0
    return r


# ----------------------------------------------------------------------------
# ray casting against the analytic primitives (ray parameter = camera z)
# ----------------------------------------------------------------------------

def _hit_room(o, d, lo, hi):
    lam = np.full(d.shape[0], np.inf)
    for a in range(3):
        da = d[:, a]
        with np.errstate(divide="ignore", invalid="ignore"):
            t_hi = (hi[a] - o[a]) / da
            t_lo = (lo[a] - o[a]) / da
        ta = np.where(da > 0, t_hi, np.where(da < 0, t_lo, np.inf))
        lam = np.minimum(lam, ta)
    return lam


def _hit_floor(o, d, h):
    dz = d[:, 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        t = (h - o[2]) / dz
    return np.where((dz < 0) & (t > 0), t, np.inf)


def _hit_sphere(o, d, c, r):
    oc = o - np.asarray(c)
    a = np.einsum("ij,ij->i", d, d)
    b = 2.0 * (d @ oc)
    cc = oc @ oc - r * r
    disc = b * b - 4 * a * cc
    sq = np.sqrt(np.maximum(disc, 0.0))
    t = (-b - sq) / (2 * a)
    return np.where((disc >= 0) & (t > 0), t, np.inf)


def _yaw_matrix(yaw):
    c, s = math.cos(yaw), math.sin(yaw)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def _hit_box(o, d, centre, half, yaw):
    Rb = _yaw_matrix(yaw)             # local -> world
    ol = Rb.T @ (o - np.asarray(centre))
    dl = d @ Rb                       # (Rb^T d) row-wise
    tn = np.full(d.shape[0], -np.inf)
    tf = np.full(d.shape[0], np.inf)
    for a in range(3):
        da = dl[:, a]
        with np.errstate(divide="ignore", invalid="ignore"):
            t1 = (-half[a] - ol[a]) / da
            t2 = (half[a] - ol[a]) / da
        lo = np.minimum(t1, t2)
        hi = np.maximum(t1, t2)
        par = da == 0
        inside = np.abs(ol[a]) <= half[a]
        lo = np.where(par, np.where(inside, -np.inf, np.inf), lo)
        hi = np.where(par, np.where(inside, np.inf, -np.inf), hi)
        tn = np.maximum(tn, lo)
        tf = np.minimum(tf, hi)
    return np.where((tn <= tf) & (tn > 0), tn, np.inf)


def _cull(o, d, c, radius):
    """Indices of rays whose line passes within `radius` of `c` (bounding sphere)."""
    oc = np.asarray(c, np.float64) - o
    dd = np.einsum("ij,ij->i", d, d)
    proj = d @ oc
    dist2 = oc @ oc - proj * proj / dd
    return np.flatnonzero((dist2 <= radius * radius * 1.0001) & (proj > -radius * np.sqrt(dd)))


def render_depth(scene: Scene, pose_w2c: np.ndarray, intr: Intrinsics,
                 zrange=(0.3, 4.0)) -> np.ndarray:
    """Noiseless depth (camera z, metres, float64, shape (H, W)); 0 = no return
    or outside `zrange`."""
    M = np.asarray(pose_w2c, np.float64)
    R, t = M[:3, :3], M[:3, 3]
    eye = -R.T @ t
    rays = pixel_rays(intr).reshape(-1, 3) @ R      # world directions, camera z = 1
    lam = np.full(rays.shape[0], np.inf)
    for lo, hi in scene.rooms:
        lam = np.minimum(lam, _hit_room(eye, rays, np.asarray(lo), np.asarray(hi)))
    for h in scene.floors:
        lam = np.minimum(lam, _hit_floor(eye, rays, h))
    for c, r in scene.spheres:
        sel = _cull(eye, rays, c, r)
        if sel.size:
            lam[sel] = np.minimum(lam[sel], _hit_sphere(eye, rays[sel], c, r))
    for c, half, yaw in scene.boxes:
        sel = _cull(eye, rays, c, float(np.linalg.norm(half)))
        if sel.size:
            lam[sel] = np.minimum(lam[sel], _hit_box(eye, rays[sel], c, half, yaw))
    z = np.where(np.isfinite(lam), lam, 0.0)
    z = np.where((z >= zrange[0]) & (z <= zrange[1]), z, 0.0)
    return z.reshape(intr.height, intr.width)


# ----------------------------------------------------------------------------
# analytic signed distance of free space (positive in free space)
# ----------------------------------------------------------------------------

def analytic_sdf(scene: Scene, pts: np.ndarray) -> np.ndarray:
    """Signed distance (metres, float64) of points (N, 3) to the scene surface:
    positive in free space, negative inside solids."""
    p = np.asarray(pts, np.float64).reshape(-1, 3)
    s = np.full(p.shape[0], np.inf)
    for lo, hi in scene.rooms:
        lo = np.asarray(lo)
        hi = np.asarray(hi)
        inner = np.minimum(p - lo, hi - p).min(axis=1)          # >0 inside the room
        # outside the room the free-space distance is minus the box distance
        q = np.maximum(np.maximum(lo - p, p - hi), 0.0)
        outer = -np.linalg.norm(q, axis=1)
        s = np.minimum(s, np.where(inner >= 0, inner, np.minimum(outer, inner)))
    for h in scene.floors:
        s = np.minimum(s, p[:, 2] - h)
    for c, r in scene.spheres:
        s = np.minimum(s, np.linalg.norm(p - np.asarray(c), axis=1) - r)
    for c, half, yaw in scene.boxes:
        Rb = _yaw_matrix(yaw)
        ql = np.abs((p - np.asarray(c)) @ Rb) - np.asarray(half)
        out = np.linalg.norm(np.maximum(ql, 0.0), axis=1)
        ins = np.minimum(ql.max(axis=1), 0.0)
        s = np.minimum(s, out + ins)
    return s


def render_points_normals(scene: Scene, pose_w2c: np.ndarray, intr: Intrinsics, h: float = 1e-5):
    """Exact surface point and normal maps of a view, float32 (H, W, 4) each,
    world frame, w = 1 where the noiseless depth is valid: the point is the
    rendered depth's ray point, the normal the normalised gradient of the
    analytic signed distance there (central differences, step h).  A synthetic
    stand-in for a perfect model's raycast."""
    M = np.asarray(pose_w2c, np.float64)
    R, t = M[:3, :3], M[:3, 3]
    z = render_depth(scene, M, intr)
    cam = pixel_rays(intr) * z[..., None]
    world = (cam.reshape(-1, 3) - t) @ R          # R^T (X - t), row-wise
    ok = z.reshape(-1) > 0
    g = np.zeros_like(world)
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        g[:, a] = (analytic_sdf(scene, world + e) - analytic_sdf(scene, world - e)) / (2 * h)
    nrm = np.linalg.norm(g, axis=1)
    ok &= nrm > 0
    n = g / np.where(nrm > 0, nrm, 1.0)[:, None]
    V = np.zeros((world.shape[0], 4), np.float32)
    N = np.zeros((world.shape[0], 4), np.float32)
    V[ok, :3] = world[ok]
    V[ok, 3] = 1.0
    N[ok, :3] = n[ok]
    N[ok, 3] = 1.0
    return V.reshape(intr.height, intr.width, 4), N.reshape(intr.height, intr.width, 4)


# ----------------------------------------------------------------------------
# sensor noise
# ----------------------------------------------------------------------------

def kinect_noise(depth: np.ndarray, rng: np.random.Generator,
                 dropout=0.02, edge_jump=0.05, zrange=(0.3, 4.0)) -> np.ndarray:
    """Kinect-like corruption of a noiseless depth map (float64 metres).

    * axial Gaussian noise, sigma(z) = 0.0012 + 0.0019 (z - 0.4)^2 m;
    * edge dropout: pixels within 1 px of a 4-neighbour depth jump larger than
      `edge_jump` (or next to a hole) form the edge region; a seeded random
      subset of it, of size `dropout` x (number of valid pixels) or the whole
      region if it is smaller, is zeroed;
    * depths outside `zrange` become 0.
    """
    z = np.asarray(depth, np.float64)
    valid = z > 0
    sigma = 0.0012 + 0.0019 * (z - 0.4) ** 2
    noisy = np.where(valid, z + rng.standard_normal(z.shape) * sigma, 0.0)

    jump = np.zeros_like(valid)
    dx = np.abs(np.diff(z, axis=1)) > edge_jump
    dy = np.abs(np.diff(z, axis=0)) > edge_jump
    jump[:, :-1] |= dx
    jump[:, 1:] |= dx
    jump[:-1, :] |= dy
    jump[1:, :] |= dy
    region = np.zeros_like(jump)
    region[:, :] = jump
    region[:, :-1] |= jump[:, 1:]
    region[:, 1:] |= jump[:, :-1]
    region[:-1, :] |= jump[1:, :]
    region[1:, :] |= jump[:-1, :]
    region &= valid
    idx = np.flatnonzero(region)
    k = min(int(round(dropout * int(valid.sum()))), idx.size)
    if k > 0:
        drop = rng.choice(idx, size=k, replace=False)
        noisy.reshape(-1)[drop] = 0.0
    noisy = np.where((noisy >= zrange[0]) & (noisy <= zrange[1]), noisy, 0.0)
    return noisy


def to_mm_u16(depth_m: np.ndarray) -> np.ndarray:
    """Quantise metres to uint16 millimetres, round half to even; 0 stays 0."""
    mm = np.rint(np.asarray(depth_m, np.float64) * 1000.0)
    return np.clip(mm, 0, 65535).astype(np.uint16)
