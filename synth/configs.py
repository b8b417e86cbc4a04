"""The five seeded workloads (volume parameters, scenes, trajectories, frames).

C1 tiny     160x120 float32 depth, sphere on a floor, 10 poses, noiseless.
C2 full     640x480 uint16 mm depth, 4x4x3 m room with 20 primitives, 300
            poses, Kinect-like noise.
C3 large    640x480 uint16 mm depth, 12x12x3 m layout of 3x3 rooms with doors
            and 200 primitives, 1500 poses, same noise (host swapping).
Seeds: numpy PCG64, seed = 1000 * config + index.
"""
from __future__ import annotations

import dataclasses
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
