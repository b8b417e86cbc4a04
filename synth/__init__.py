"""Seeded synthetic inputs (scenes, trajectories, depth frames, noise).

Shared by the oracle tests, the GPU tests and the benchmark; contains none of
the fusion method's arithmetic."""
from .scenes import (Intrinsics, Scene, analytic_sdf, kinect_noise, look_at,  # noqa: F401
                     pixel_rays, render_depth, to_mm_u16)
from . import configs, scenes  # noqa: F401
