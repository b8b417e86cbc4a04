"""The five seeded workloads (volume parameters, scenes, trajectories, frames).

C1 tiny     160x120 float32 depth, sphere on a floor, 10 poses, noiseless.
C2 full     640x480 uint16 mm depth, 4x4x3 m room with 20 primitives, 300
            poses, Kinect-like noise.
C3 large    640x480 uint16 mm depth, 12x12x3 m layout of 3x3 rooms with doors
            and 200 primitives, 1500 poses, same noise (host swapping).
C4 batched  64 rigid submaps over the C3 layout with log-uniform block counts,
            frames of the C3 walk fused into the 4-12 submaps they overlap,
            8 views of mixed resolution per frame.
Seeds: numpy PCG64, seed = 1000 * config + index.
"""
from __future__ import annotations

import dataclasses
import functools
import math

import numpy as np

from .scenes import (Intrinsics, Scene, kinect_noise, look_at, render_depth,
                     to_mm_u16)


@dataclasses.dataclass
class VolumeParams:
    voxel_size: float
    mu: float
    max_w: int
    n_buckets: int
    n_excess: int
    n_blocks: int


C1_VOLUME = VolumeParams(0.01, 0.04, 100, 1 << 16, 1 << 12, 1 << 14)
C2_VOLUME = VolumeParams(0.005, 0.02, 100, 1 << 20, 1 << 17, 1 << 18)
C3_VOLUME = VolumeParams(0.004, 0.016, 100, 1 << 22, 1 << 19, 1 << 20)

C1_INTR = Intrinsics(120.0, 120.0, 80.0, 60.0, 160, 120)
KINECT_INTR = Intrinsics(525.0, 525.0, 319.5, 239.5, 640, 480)


def rng_for(config: int, index: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(1000 * config + index))


# ----------------------------------------------------------------------------
# C1
# ----------------------------------------------------------------------------

def c1_scene() -> Scene:
    return Scene(floors=[0.0], spheres=[((0.0, 0.0, 0.25), 0.25)])


def c1_poses(n: int = 10, seed_index: int = 0) -> list:
    """n poses evenly spaced along a 0.3 m arc of the 1.2 m-radius circle about
    the sphere centre, 15 degrees above the horizontal, looking at the centre."""
    rng = rng_for(1, seed_index)
    phi0 = rng.uniform(0.0, 2 * math.pi)
    span = 0.3 / 1.2
    S = np.array([0.0, 0.0, 0.25])
    el = math.radians(15.0)
    poses = []
    for k in range(n):
        phi = phi0 + span * k / max(1, n - 1)
        eye = S + 1.2 * np.array([math.cos(el) * math.cos(phi),
                                  math.cos(el) * math.sin(phi), math.sin(el)])
        poses.append(look_at(eye, S))
    return poses


def c1_frames(n: int = 10, seed_index: int = 0):
    """(depths float32 (n,H,W) metres, poses float32 (n,4,4), intrinsics, scene)."""
    scene = c1_scene()
    poses = c1_poses(n, seed_index)
    depths = np.stack([render_depth(scene, P, C1_INTR) for P in poses]).astype(np.float32)
    return depths, np.stack(poses).astype(np.float32), C1_INTR, scene


# ----------------------------------------------------------------------------
# C2
# ----------------------------------------------------------------------------

def random_primitives(rng, n, region_lo, region_hi, zmax=2.0):
    spheres, boxes = [], []
    for _ in range(n):
        size = rng.uniform(0.1, 0.6)
        c = np.array([rng.uniform(region_lo[0] + 0.4, region_hi[0] - 0.4),
                      rng.uniform(region_lo[1] + 0.4, region_hi[1] - 0.4),
                      rng.uniform(size / 2, zmax)])
        if rng.uniform() < 0.5:
            spheres.append((tuple(c), size / 2))
        else:
            boxes.append((tuple(c), (size / 2,) * 3, rng.uniform(0, math.pi / 2)))
    return spheres, boxes


def c2_scene(seed_index: int = 0, n_prims: int = 20) -> Scene:
    rng = rng_for(2, seed_index)
    spheres, boxes = random_primitives(rng, n_prims, (0, 0), (4, 4))
    return Scene(rooms=[((0.0, 0.0, 0.0), (4.0, 4.0, 3.0))], spheres=spheres, boxes=boxes)


def c2_poses(n: int = 300, seed_index: int = 0) -> list:
    """Smooth loop around the room centre; each camera looks 1.5 m ahead along
    the chord to a phase-lagged point of the same curve."""
    rng = rng_for(2, 500 + seed_index)
    th0 = rng.uniform(0, 2 * math.pi)
    ph = rng.uniform(0, 2 * math.pi, size=3)
    centre = np.array([2.0, 2.0, 1.5])

    def C(th):
        return centre + np.array([1.2 * math.cos(th) + 0.2 * math.sin(3 * th + ph[0]),
                                  1.2 * math.sin(th) + 0.2 * math.cos(2 * th + ph[1]),
                                  -0.2 + 0.2 * math.sin(2 * th + ph[2])])

    poses = []
    for f in range(n):
        th = th0 + 2 * math.pi * f / 300.0 * 0.8
        eye = C(th)
        ahead = C(th + 0.5) - eye + np.array([0.0, 0.0, -0.3])
        ahead /= np.linalg.norm(ahead)
        poses.append(look_at(eye, eye + 1.5 * ahead))
    return poses


def noisy_u16_frames(scene, poses, intr, config, seed_index=0, noise=True):
    out = np.empty((len(poses), intr.height, intr.width), np.uint16)
    for k, P in enumerate(poses):
        z = render_depth(scene, P, intr)
        if noise:
            z = kinect_noise(z, rng_for(config, 100000 + 1000 * seed_index + k))
        out[k] = to_mm_u16(z)
    return out


def c2_frames(n: int = 300, seed_index: int = 0, first: int = 0, noise: bool = True):
    """(depth uint16 mm (n,H,W), poses float32 (n,4,4), intrinsics, scene) for
    trajectory frames first .. first+n-1."""
    scene = c2_scene(seed_index)
    poses = c2_poses(max(300, first + n), seed_index)[first:first + n]
    depth = noisy_u16_frames(scene, poses, KINECT_INTR, 2, seed_index, noise)
    return depth, np.stack(poses).astype(np.float32), KINECT_INTR, scene


def c2_frame(k: int, seed_index: int = 0, noise: bool = True) -> np.ndarray:
    """Trajectory frame k of C2 as uint16 mm (same values as c2_frames)."""
    scene = c2_scene(seed_index)
    P = c2_poses(max(300, k + 1), seed_index)[k]
    z = render_depth(scene, P, KINECT_INTR)
    if noise:
        z = kinect_noise(z, rng_for(2, 100000 + 1000 * seed_index + k))
    return to_mm_u16(z)


# ----------------------------------------------------------------------------
# C3: 12x12x3 m layout of 3x3 rooms (4x4 m) with one door per shared wall
# ----------------------------------------------------------------------------

WALL = 0.1
DOOR_W, DOOR_H = 1.0, 2.1


@functools.lru_cache(maxsize=4)
def c3_layout(seed_index: int = 0):
    """(scene, doors) -- doors as {(room_a, room_b): (x, y)} door centres at
    floor level.  Rooms are (i, j) with x in [4i, 4i+4], y in [4j, 4j+4]."""
    rng = rng_for(3, seed_index)
    boxes = []
    doors = {}
    h = WALL / 2
    # walls between room columns (x = 4, 8) and room rows (y = 4, 8)
    for axis in (0, 1):
        for k in (1, 2):
            c = 4.0 * k
            for seg in range(3):
                lo, hi = 4.0 * seg, 4.0 * seg + 4.0
                d = rng.uniform(lo + 0.8, hi - 0.8)          # door centre along the wall
                parts = [(lo, d - DOOR_W / 2, 0.0, 3.0), (d + DOOR_W / 2, hi, 0.0, 3.0),
                         (d - DOOR_W / 2, d + DOOR_W / 2, DOOR_H, 3.0)]
                for a, b, z0, z1 in parts:
                    if b - a <= 1e-6:
                        continue
                    mid = ((a + b) / 2, (z0 + z1) / 2)
                    half_along, half_z = (b - a) / 2, (z1 - z0) / 2
                    if axis == 0:   # wall at x = c, spanning y
                        boxes.append(((c, mid[0], mid[1]), (h, half_along, half_z), 0.0))
                    else:           # wall at y = c, spanning x
                        boxes.append(((mid[0], c, mid[1]), (half_along, h, half_z), 0.0))
                if axis == 0:
                    doors[((k - 1, seg), (k, seg))] = (c, d)
                else:
                    doors[((seg, k - 1), (seg, k))] = (d, c)
    spheres = []
    for _ in range(200):
        ri, rj = rng.integers(0, 3, size=2)
        size = rng.uniform(0.1, 0.6)
        cx = rng.uniform(4 * ri + 0.5, 4 * ri + 3.5)
        cy = rng.uniform(4 * rj + 0.5, 4 * rj + 3.5)
        cz = rng.uniform(size / 2, 2.0)
        if rng.uniform() < 0.5:
            spheres.append(((cx, cy, cz), size / 2))
        else:
            boxes.append(((cx, cy, cz), (size / 2,) * 3, rng.uniform(0, math.pi / 2)))
    scene = Scene(rooms=[((0.0, 0.0, 0.0), (12.0, 12.0, 3.0))], spheres=spheres, boxes=boxes)
    return scene, doors


def _catmull_rom(points, n):
    P = np.asarray(points, np.float64)
    P = np.vstack([P[0], P, P[-1]])
    seg = np.linalg.norm(np.diff(P[1:-1], axis=0), axis=1)
    cum = np.concatenate([[0.0], np.cumsum(seg)])
    s = np.linspace(0.0, cum[-1], n)
    out = np.empty((n, 3))
    for k, sk in enumerate(s):
        i = min(np.searchsorted(cum, sk, side="right") - 1, len(seg) - 1)
        u = (sk - cum[i]) / max(seg[i], 1e-12)
        p0, p1, p2, p3 = P[i], P[i + 1], P[i + 2], P[i + 3]
        out[k] = 0.5 * ((2 * p1) + (-p0 + p2) * u + (2 * p0 - 5 * p1 + 4 * p2 - p3) * u * u +
                        (-p0 + 3 * p1 - 3 * p2 + p3) * u ** 3)
    return out


@functools.lru_cache(maxsize=4)
def c3_poses(n: int = 1500, seed_index: int = 0) -> list:
    """A smoothed walk through the rooms in snake order, passing every shared
    door on the way at 1.5 m height, facing forward (slightly down)."""
    _, doors = c3_layout(seed_index)
    order = [(0, 0), (1, 0), (2, 0), (2, 1), (1, 1), (0, 1), (0, 2), (1, 2), (2, 2)]
    way = []
    for a, b in zip(order[:-1], order[1:]):
        way.append((4 * a[0] + 2.0, 4 * a[1] + 2.0))
        key = (a, b) if (a, b) in doors else (b, a)
        dx, dy = doors[key]
        # approach and leave the door perpendicular to its wall
        if a[0] != b[0]:
            way += [(dx - 0.6, dy), (dx + 0.6, dy)] if b[0] > a[0] else [(dx + 0.6, dy), (dx - 0.6, dy)]
        else:
            way += [(dx, dy - 0.6), (dx, dy + 0.6)] if b[1] > a[1] else [(dx, dy + 0.6), (dx, dy - 0.6)]
    way.append((4 * order[-1][0] + 2.0, 4 * order[-1][1] + 2.0))
    pts = _catmull_rom([(x, y, 1.5) for x, y in way], n + 1)
    poses = []
    for k in range(n):
        fwd = pts[k + 1] - pts[k]
        fwd[2] = 0.0
        fwd /= max(np.linalg.norm(fwd), 1e-9)
        target = pts[k] + 1.5 * fwd + np.array([0.0, 0.0, -0.25])
        poses.append(look_at(pts[k], target))
    return poses


def c3_frame(k: int, seed_index: int = 0, noise: bool = True, intr: Intrinsics = KINECT_INTR):
    scene, _ = c3_layout(seed_index)
    P = c3_poses(1500, seed_index)[k]
    z = render_depth(scene, P, intr)
    if noise:
        z = kinect_noise(z, rng_for(3, 100000 + 1000 * seed_index + k))
    return to_mm_u16(z)


# ---- C4: batched rigid submaps ------------------------------------------------------
C4_VOLUME = VolumeParams(0.005, 0.02, 100, 1 << 19, 1 << 17, 1 << 18)
C4_N_SUBMAPS = 64
C4_BLOCKS = (2000, 60000)                  # log-uniform target block counts
C4_PREFILL_INTR = Intrinsics(262.5, 262.5, 159.5, 119.5, 320, 240)
C4_VIEW_SIZES = ((320, 240), (320, 240), (640, 480), (640, 480), (960, 540), (960, 540), (1280, 720), (1280, 720))
C4_N_FRAMES = 300                         # every 5th pose of the C3 walk
C4_MAX_SEL, C4_MIN_SEL = 12, 4


def random_rotation(rng) -> np.ndarray:
    """uniform rotation from a normalised 4-d Gaussian quaternion"""
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


@dataclasses.dataclass(frozen=True)
class Submap:
    pose: np.ndarray       # 4x4 float32, world -> submap
    centre: tuple          # region centre (world, m)
    radius: float          # region radius (m)
    target: int            # block count the prefill aims at


@functools.lru_cache(maxsize=2)
def c4_submaps(seed_index: int = 0) -> tuple:
    """64 submaps: a uniform random rotation and a translation within the
    layout for the pose, a region (ball) inside the layout, and a log-uniform
    block-count target."""
    rng = rng_for(4, seed_index)
    lo, hi = math.log(C4_BLOCKS[0]), math.log(C4_BLOCKS[1])
    out = []
    for _ in range(C4_N_SUBMAPS):
        R = random_rotation(rng)
        origin = rng.uniform([0.0, 0.0, 0.0], [12.0, 12.0, 3.0])
        P = np.eye(4)
        P[:3, :3] = R
        P[:3, 3] = -R @ origin                # X_submap = R (X_world - origin)
        centre = tuple(rng.uniform([0.6, 0.6, 0.8], [11.4, 11.4, 2.2]))
        radius = float(rng.uniform(1.0, 2.0))
        target = int(round(math.exp(rng.uniform(lo, hi))))
        out.append(Submap(P.astype(np.float32), centre, radius, target))
    return tuple(out)


def c4_prefill_pose(i: int, j: int, seed_index: int = 0) -> np.ndarray:
    """j-th prefill viewpoint of submap i: a point of its region (kept inside
    the layout), a random heading, a slight random pitch"""
    sm = c4_submaps(seed_index)[i]
    rng = rng_for(4, 10000 + 1000 * i + j)
    c = np.asarray(sm.centre)
    while True:
        d = rng.uniform(-1.0, 1.0, size=3)
        if np.dot(d, d) <= 1.0:
            break
    eye = np.clip(c + sm.radius * d, [0.25, 0.25, 0.4], [11.75, 11.75, 2.6])
    yaw = rng.uniform(0.0, 2 * math.pi)
    pitch = rng.uniform(-0.45, 0.2)
    fwd = np.array([math.cos(yaw) * math.cos(pitch), math.sin(yaw) * math.cos(pitch), math.sin(pitch)])
    return look_at(eye, eye + fwd)


def c4_prefill_frame(i: int, j: int, seed_index: int = 0) -> np.ndarray:
    """noiseless float32 depth (m) of prefill viewpoint j of submap i"""
    scene, _ = c3_layout(seed_index)
    return render_depth(scene, c4_prefill_pose(i, j, seed_index), C4_PREFILL_INTR).astype(np.float32)


def c4_poses(seed_index: int = 0) -> list:
    return [np.asarray(P, np.float32) for P in c3_poses(1500, seed_index)[::5]]


def c4_frame(k: int, seed_index: int = 0) -> np.ndarray:
    """640x480 uint16 mm depth with Kinect-like noise at the k-th C4 pose"""
    scene, _ = c3_layout(seed_index)
    P = c4_poses(seed_index)[k % C4_N_FRAMES]
    z = kinect_noise(render_depth(scene, P, KINECT_INTR), rng_for(4, 200000 + 1000 * seed_index + k))
    return to_mm_u16(z)


def c4_select(pose_w2c, seed_index: int = 0, intr: Intrinsics = KINECT_INTR, near: float = 0.3,
              far: float = 4.0) -> list:
    """Submaps whose region meets the viewing frustum [near, far], nearest
    first, at most 12; fewer than 4 are topped up with the nearest regions."""
    subs = c4_submaps(seed_index)
    M = np.asarray(pose_w2c, np.float64)
    planes = []
    for n in ((intr.fx, 0.0, intr.cx), (-intr.fx, 0.0, intr.width - 1 - intr.cx),
              (0.0, intr.fy, intr.cy), (0.0, -intr.fy, intr.height - 1 - intr.cy)):
        n = np.asarray(n)
        planes.append(n / np.linalg.norm(n))
    eye = -M[:3, :3].T @ M[:3, 3]
    meet, dist = [], []
    for i, sm in enumerate(subs):
        c = M[:3, :3] @ np.asarray(sm.centre) + M[:3, 3]
        r = sm.radius
        ok = c[2] + r >= near and c[2] - r <= far and all(np.dot(n, c) >= -r for n in planes)
        d = float(np.linalg.norm(np.asarray(sm.centre) - eye))
        dist.append(d)
        if ok:
            meet.append((d, i))
    meet.sort()
    sel = [i for _, i in meet[:C4_MAX_SEL]]
    if len(sel) < C4_MIN_SEL:
        for i in np.argsort(dist):
            if int(i) not in sel:
                sel.append(int(i))
            if len(sel) == C4_MIN_SEL:
                break
    return sel


def c4_views(k: int, seed_index: int = 0) -> list:
    """the 8 views of frame k: (intrinsics, pose); view j looks from the walk
    pose 37 j frames ahead, at its own size (focal length scaled with width)"""
    poses = c4_poses(seed_index)
    out = []
    for j, (W, H) in enumerate(C4_VIEW_SIZES):
        f = 525.0 * W / 640.0
        intr = Intrinsics(f, f, (W - 1) / 2.0, (H - 1) / 2.0, W, H)
        out.append((intr, poses[(k + 37 * j) % C4_N_FRAMES]))
    return out
