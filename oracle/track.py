"""CPU oracle of the depth tracker (Sec. 4.1.1, ITMDepthTracker).

TEST INFRASTRUCTURE ONLY: tests/, the smoke check and the bench's CPU
baseline may use this module; the library never does, and nothing here is
shared with it.

The tracker aligns a new depth image with the surface point map V and normal
map N that the raycast (Sec. 4.4) rendered from a reference pose.  Every live
depth pixel p is moved into the world by the current estimate (R, t), projected
into the reference image to the pixel p_bar, and scored by its distance from
the plane through V(p_bar) with normal N(p_bar):
    d = (R p + t - V(p_bar))^T N(p_bar).
(R, t) minimises the sum of d^2 through a linear system, the two steps repeat,
and a resolution hierarchy of the depth image runs from the coarsest level to
the finest (Sec. 4.1.1).  Following Sec. 4.1.1's split, the per-pixel terms
and their sums are the data-parallel part; the 6x6 solve is a few dozen
operations.

Readings where the paper is silent (each also in the design notes):
  * pose: the estimate is the camera->world transform (R, t), kept in float64;
    per-pixel arithmetic uses its float32 rounding.  The caller passes
    world->camera matrices (the integration's M_d); the initial one is
    inverted in float64.
  * linear system: the residual is linearised in a world-frame increment
    xi = (omega, delta_t): R p + t -> Exp(omega) (R p + t) + delta_t, so a
    pair's Jacobian row is (q x n, n) with q = R p + t, n = N(p_bar); the
    normal equations A xi = -g with A = sum J^T J, g = sum J^T d; the update
    R <- Exp(omega) R, t <- Exp(omega) t + delta_t (Rodrigues' formula).
  * association: nearest reference pixel, floor(u + 0.5), of the projection
    of q with the reference pose and intrinsics (u = (fx c_x) / c_z + cx);
    a pair needs c_z > 0, the pixel inside the reference image, valid V and
    N (w = 1), and |q - V| <= tau_l, a per-level distance threshold.
  * hierarchy: level l + 1 halves level l; each coarse pixel is the mean of
    the valid (> 0) depths of its 2x2 block (summed in raster order in
    float32, divided by their count), 0 if none.  Level-l intrinsics:
    fx / 2^l, fy / 2^l, (cx + 0.5) / 2^l - 0.5, (cy + 0.5) / 2^l - 0.5, so that
    a coarse pixel centre is the mean of the centres it covers.  The
    reference maps stay at their own resolution at every level.
  * iterations: a fixed count per level; a level may stop early once
    |xi|_2 falls below a threshold (applied after the update); a level with
    fewer than 6 pairs or a matrix that is not positive definite stops
    without an update.

Per-pixel operations are float32, evaluated in the written order (no fused
multiply-add), so that every decision (pixel rounding, image bounds, the
distance test) is the one the GPU takes; the sums are float64.
"""
from __future__ import annotations

import numpy as np

f32 = np.float32


def pyramid(depth: np.ndarray, levels: int) -> list:
    """[level 0, level 1, ...]: level 0 is `depth` (float32 metres, 0 =
    invalid); each further level is the mean of the valid depths of 2x2
    blocks (raster order, float32), size floor(W / 2) x floor(H / 2)."""
    out = [np.ascontiguousarray(depth, f32)]
    for _ in range(1, levels):
        s = out[-1]
        h, w = s.shape[0] // 2, s.shape[1] // 2
        a = s[0:2 * h:2, 0:2 * w:2]
        b = s[0:2 * h:2, 1:2 * w:2]
        c = s[1:2 * h:2, 0:2 * w:2]
        d = s[1:2 * h:2, 1:2 * w:2]
        tot = np.zeros((h, w), f32)
        cnt = np.zeros((h, w), f32)
        for q in (a, b, c, d):              # raster order of the block
            v = q > 0
            tot = np.where(v, tot + q, tot).astype(f32)
            cnt = cnt + v.astype(f32)
        with np.errstate(invalid="ignore", divide="ignore"):
            out.append(np.where(cnt > 0, tot / cnt, f32(0)).astype(f32))
    return out


def level_intrinsics(K, level: int) -> np.ndarray:
    """(fx, fy, cx, cy) of pyramid level `level` (float64 arithmetic, rounded
    once to float32)"""
    fx, fy, cx, cy = (float(v) for v in K[:4])
    s = 2.0 ** level
    return np.array([fx / s, fy / s, (cx + 0.5) / s - 0.5, (cy + 0.5) / s - 0.5], f32)


def pair_terms(depth_l, K_l, V, N, K_r, M_r, R, t, tau):
    """Per live pixel of one level: (mask of pixels with a pair, J (n, 6)
    float32, d (n,) float32, q (n, 3) float32, and the matched reference
    points and normals (n, 3)) at the float32 pose (R, t).
    V, N: (Hr, Wr, 4) world points and normals of the reference view (w = 1
    valid); K_r = (fx, fy, cx, cy) and M_r (4x4 world->camera) of that view."""
    depth_l = np.asarray(depth_l, f32)
    H, W = depth_l.shape
    Hr, Wr = V.shape[0], V.shape[1]
    fx, fy, cx, cy = (f32(v) for v in K_l)
    rfx, rfy, rcx, rcy = (f32(v) for v in K_r[:4])
    R = np.asarray(R, f32)
    t = np.asarray(t, f32)
    M = np.asarray(M_r, f32)
    ys, xs = np.mgrid[0:H, 0:W]
    xs = xs.astype(f32)
    ys = ys.astype(f32)
    d = depth_l
    ok = d > 0
    px = d * ((xs - cx) / fx)
    py = d * ((ys - cy) / fy)
    pz = d
    qx = ((R[0, 0] * px + R[0, 1] * py) + R[0, 2] * pz) + t[0]
    qy = ((R[1, 0] * px + R[1, 1] * py) + R[1, 2] * pz) + t[1]
    qz = ((R[2, 0] * px + R[2, 1] * py) + R[2, 2] * pz) + t[2]
    ccx = ((M[0, 0] * qx + M[0, 1] * qy) + M[0, 2] * qz) + M[0, 3]
    ccy = ((M[1, 0] * qx + M[1, 1] * qy) + M[1, 2] * qz) + M[1, 3]
    ccz = ((M[2, 0] * qx + M[2, 1] * qy) + M[2, 2] * qz) + M[2, 3]
    ok &= ccz > 0
    with np.errstate(invalid="ignore", divide="ignore", over="ignore"):
        u = (rfx * ccx) / ccz + rcx
        v = (rfy * ccy) / ccz + rcy
        ui = np.floor(u + f32(0.5))
        vi = np.floor(v + f32(0.5))
    ok &= (ui >= 0) & (ui <= Wr - 1) & (vi >= 0) & (vi <= Hr - 1)
    iy, ix = np.nonzero(ok)
    ru = ui[iy, ix].astype(np.int64)
    rv = vi[iy, ix].astype(np.int64)
    Vp = np.asarray(V, f32)[rv, ru]
    Np = np.asarray(N, f32)[rv, ru]
    q = np.stack([qx[iy, ix], qy[iy, ix], qz[iy, ix]], axis=1)
    keep = (Vp[:, 3] == 1) & (Np[:, 3] == 1)
    dx = q[:, 0] - Vp[:, 0]
    dy = q[:, 1] - Vp[:, 1]
    dz = q[:, 2] - Vp[:, 2]
    dist2 = (dx * dx + dy * dy) + dz * dz
    tau = f32(tau)
    keep &= dist2 <= tau * tau
    dx, dy, dz, q, Np = dx[keep], dy[keep], dz[keep], q[keep], Np[keep]
    nx, ny, nz = Np[:, 0], Np[:, 1], Np[:, 2]
    r = (dx * nx + dy * ny) + dz * nz
    J = np.stack([q[:, 1] * nz - q[:, 2] * ny, q[:, 2] * nx - q[:, 0] * nz, q[:, 0] * ny - q[:, 1] * nx,
                  nx, ny, nz], axis=1).astype(f32)
    mask = np.zeros((H, W), bool)
    mask[iy[keep], ix[keep]] = True
    return mask, J, r.astype(f32), q, Vp[keep][:, :3], Np[:, :3]


def normal_equations(J: np.ndarray, r: np.ndarray):
    """(A = sum J^T J, g = sum J^T d, sum d^2, n) in float64"""
    J64 = np.asarray(J, np.float64)
    r64 = np.asarray(r, np.float64)
    return J64.T @ J64, J64.T @ r64, float(r64 @ r64), int(len(r64))


def exp_rotation(w) -> np.ndarray:
    """rotation matrix of the rotation vector w (Rodrigues' formula, float64)"""
    w = np.asarray(w, np.float64)
    th = float(np.sqrt(w @ w))
    Wx = np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])
    if th < 1e-12:
        return np.eye(3) + Wx
    return np.eye(3) + (np.sin(th) / th) * Wx + ((1.0 - np.cos(th)) / (th * th)) * (Wx @ Wx)


def solve_step(A, g):
    """xi = A^-1 (-g), or None when A is not positive definite"""
    try:
        np.linalg.cholesky(A)
    except np.linalg.LinAlgError:
        return None
    return np.linalg.solve(A, -g)


def apply_update(R, t, xi):
    dR = exp_rotation(xi[:3])
    return dR @ R, dR @ t + np.asarray(xi[3:], np.float64)


def invert_pose(M) -> tuple:
    """(R, t) of the inverse of a rigid 4x4 (float64)"""
    M = np.asarray(M, np.float64)
    R = M[:3, :3].T
    return R, -(R @ M[:3, 3])


def track(depth, K, V, N, K_r, M_r, M_init, iterations, taus, min_update: float = 0.0):
    """Align `depth` (float32 metres at level 0, intrinsics K = (fx, fy, cx,
    cy)) with the reference maps V, N (intrinsics K_r, world->camera M_r),
    starting from the world->camera guess M_init.  iterations[l] and taus[l]
    per level, index 0 = finest; levels run coarsest first.  Returns
    (world->camera float32 4x4, per-level info dicts: iterations done, pairs
    and sums of the level's last evaluated system)."""
    levels = len(iterations)
    R, t = invert_pose(M_init)
    pyr = pyramid(depth, levels)
    info = [dict(iterations=0, pairs=0, A=None, g=None, rr=0.0, degenerate=False) for _ in range(levels)]
    for l in reversed(range(levels)):
        Kl = level_intrinsics(K, l)
        for _ in range(int(iterations[l])):
            _, J, r, _, _, _ = pair_terms(pyr[l], Kl, V, N, K_r, M_r, R.astype(f32), t.astype(f32), taus[l])
            A, g, rr, n = normal_equations(J, r)
            info[l].update(pairs=n, A=A, g=g, rr=rr)
            xi = solve_step(A, g) if n >= 6 else None
            if xi is None:
                info[l]["degenerate"] = True
                break
            R, t = apply_update(R, t, xi)
            info[l]["iterations"] += 1
            if float(np.sqrt(xi @ xi)) < min_update:
                break
    out = np.eye(4)
    out[:3, :3] = R.T
    out[:3, 3] = -(R.T @ t)
    return out.astype(f32), info
