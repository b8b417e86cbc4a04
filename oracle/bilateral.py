"""CPU oracle of the bilateral depth filter -- test infrastructure only.

TEST INFRASTRUCTURE ONLY: tests/, the smoke check and the bench's CPU
baseline may use this module; the library never does, and nothing here is
shared with it.

The paper's view builder optionally applies a bilateral filter to the
processed depth image before it is used (Sec. 4, image preparation; the
scene setting useBilateralFilter of Sec. 6), and says nothing more about
it.  This is the textbook bilateral filter (Tomasi and Manduchi, 1998)
restricted to valid depths, in float64:

    out(p) = sum_q w(p, q) d(q) / sum_q w(p, q),
    w(p, q) = exp(-|p - q|^2 / (2 sigma_s^2)) * exp(-(d(p) - d(q))^2 / (2 sigma_r^2)),

over the (2r + 1)^2 window of pixels q inside the image with a valid depth
(d > 0); out(p) = 0 where d(p) is not valid (no hole filling).
"""
from __future__ import annotations

import numpy as np


def bilateral(depth: np.ndarray, radius: int, sigma_space: float, sigma_range: float) -> np.ndarray:
    """depth (H, W) in metres (0 = invalid) -> filtered depth, float64"""
    d = np.asarray(depth, np.float64)
    H, W = d.shape
    valid = d > 0
    num = np.zeros((H, W))
    den = np.zeros((H, W))
    for dy in range(-radius, radius + 1):
        for dx in range(-radius, radius + 1):
            ws = np.exp(-(dx * dx + dy * dy) / (2.0 * sigma_space * sigma_space))
            # q = p + (dx, dy), for every p whose q lies inside the image
            ys = slice(max(0, -dy), min(H, H - dy))
            xs = slice(max(0, -dx), min(W, W - dx))
            yq = slice(max(0, dy), min(H, H + dy))
            xq = slice(max(0, dx), min(W, W + dx))
            dq = d[yq, xq]
            dp = d[ys, xs]
            w = ws * np.exp(-((dp - dq) ** 2) / (2.0 * sigma_range * sigma_range))
            w = np.where(valid[yq, xq], w, 0.0)
            num[ys, xs] += w * dq
            den[ys, xs] += w
    with np.errstate(invalid="ignore", divide="ignore"):
        out = np.where(valid, num / np.where(den > 0, den, 1.0), 0.0)
    return out
