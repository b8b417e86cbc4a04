"""CPU oracle of surfel fusion (Sec. 7.3, Keller et al.'s surfel-based
reconstruction as the paper summarises it).

TEST INFRASTRUCTURE ONLY: tests/, the smoke check and the bench's CPU
baseline may use this module; the library never does, and nothing here is
shared with it.

A surfel is a point with position v, normal n, radius r, confidence c and
time stamp t.  Per frame (Sec. 7.3): every input pixel u gives a world point
v^g(u) and normal n^g(u); all surfels are forward-projected into the image as
circles and their indices written into an index map; the corresponding surfel
of a point is the one whose index is at its pixel; it is updated by the
weighted average
    v <- (c v + alpha v^g) / (c + alpha),  n <- (c n + alpha n^g) / (c + alpha),
    c <- c + alpha,  t <- now,
and a point without a corresponding surfel becomes a new surfel with c = alpha.

Readings where the paper is silent (each also in the design notes):
  S1 input point: v^c = d ((x - cx) / fx, (y - cy) / fy, 1), world v^g = R v^c + t
     with (R, t) the camera->world inverse of M_d (float64, rounded to float32).
  S2 input normal: n^c = normalise((v^c(x+1, y) - v^c(x, y)) x (v^c(x, y+1) - v^c(x, y))),
     turned towards the camera (n^c . v^c < 0); needs the three depths valid,
     so the last row and column have none; a pixel is an input point only with
     both a depth and a normal.  World normal R n^c.
  S3 alpha = exp(-gamma^2 / (2 sigma^2)), gamma = |(x - cx, y - cy)| / |(cx, cy)|
     (distance from the principal point, normalised), sigma = 0.6 (Keller et al.).
  S4 radius r = d sqrt(2) / (2 fx): the circle around the pixel's footprint,
     set when the surfel is made; the update leaves it unchanged (the
     paper's update lists v, n, c, t).
  S5 index map: a surfel with camera z_s > 0 projects to (u_s, v_s) = (fx X / Z + cx,
     fy Y / Z + cy) with pixel radius rho = min(fx r / z_s, 8); it covers the
     pixels (x, y) with (x - u_s)^2 + (y - v_s)^2 <= rho^2; a pixel keeps the
     covering surfel of least z_s, ties to the smaller index.
  S6 correspondence: the pixel's surfel s, if |d(u) - z_s| <= delta_z and
     n^g . n_s >= tau_n |n_s| (the paper's test is only the index map; without
     a gate a pixel at a silhouette would average two surfaces).
  S7 a surfel with several corresponding points in one frame takes all of
     them: (c v + sum alpha_i v_i) / (c + sum alpha_i), which is the paper's
     update applied to them one after another in any order.
  S8 new surfels are appended in pixel raster order; beyond the capacity they
     are dropped and an overflow flag is raised.
  Removal, merging and the stable/unstable distinction of Keller et al. are
  not described in the paper and not done.

Decisions that pick integers (coverage, z order, gates, validity) are taken in
float32 in a fixed operation order, as the GPU takes them; sums and the
update are float64, stored as float32.
"""
from __future__ import annotations

import numpy as np

f32 = np.float32
RHO_MAX = f32(8.0)


class SurfelMap:
    def __init__(self, capacity: int, sigma: float = 0.6, delta_z: float = 0.05, tau_n: float = 0.5):
        self.capacity = int(capacity)
        self.sigma, self.delta_z, self.tau_n = sigma, delta_z, tau_n
        self.pos = np.zeros((0, 4), f32)      # x, y, z, radius
        self.nrm = np.zeros((0, 4), f32)      # nx, ny, nz, confidence
        self.time = np.zeros(0, np.int32)
        self.frames = 0
        self.overflow = False
        self.index_map = None

    @classmethod
    def from_state(cls, pos, nrm, time, frames, capacity, **kw):
        m = cls(capacity, **kw)
        m.pos = np.array(pos, f32).reshape(-1, 4)
        m.nrm = np.array(nrm, f32).reshape(-1, 4)
        m.time = np.array(time, np.int32).reshape(-1)
        m.frames = int(frames)
        return m


def input_points(depth, K, pose_w2c, sigma=0.6):
    """(valid (H, W), world points (H, W, 3), world normals (H, W, 3), alpha
    (H, W), camera z (H, W)), float32"""
    d = np.asarray(depth, f32)
    H, W = d.shape
    fx, fy, cx, cy = (f32(v) for v in K[:4])
    M = np.asarray(pose_w2c, np.float64)
    Rd = M[:3, :3].T
    td = -(Rd @ M[:3, 3])
    R, t = Rd.astype(f32), td.astype(f32)
    ys, xs = np.mgrid[0:H, 0:W]
    xs = xs.astype(f32)
    ys = ys.astype(f32)
    vx = d * ((xs - cx) / fx)
    vy = d * ((ys - cy) / fy)
    vz = d
    ok = d > 0
    # forward differences to the right and down neighbours
    okn = np.zeros((H, W), bool)
    okn[:-1, :-1] = ok[:-1, :-1] & ok[:-1, 1:] & ok[1:, :-1]
    ax = np.zeros((H, W), f32)
    ay = np.zeros((H, W), f32)
    az = np.zeros((H, W), f32)
    bx = np.zeros((H, W), f32)
    by = np.zeros((H, W), f32)
    bz = np.zeros((H, W), f32)
    ax[:, :-1] = vx[:, 1:] - vx[:, :-1]
    ay[:, :-1] = vy[:, 1:] - vy[:, :-1]
    az[:, :-1] = vz[:, 1:] - vz[:, :-1]
    bx[:-1, :] = vx[1:, :] - vx[:-1, :]
    by[:-1, :] = vy[1:, :] - vy[:-1, :]
    bz[:-1, :] = vz[1:, :] - vz[:-1, :]
    nx = ay * bz - az * by
    ny = az * bx - ax * bz
    nz = ax * by - ay * bx
    nn = (nx * nx + ny * ny) + nz * nz
    okn &= nn > 0
    with np.errstate(invalid="ignore", divide="ignore"):
        inv = f32(1.0) / np.sqrt(nn)
        nx, ny, nz = nx * inv, ny * inv, nz * inv
    flip = ((nx * vx + ny * vy) + nz * vz) > 0
    nx = np.where(flip, -nx, nx)
    ny = np.where(flip, -ny, ny)
    nz = np.where(flip, -nz, nz)
    valid = ok & okn
    wx = ((R[0, 0] * vx + R[0, 1] * vy) + R[0, 2] * vz) + t[0]
    wy = ((R[1, 0] * vx + R[1, 1] * vy) + R[1, 2] * vz) + t[1]
    wz = ((R[2, 0] * vx + R[2, 1] * vy) + R[2, 2] * vz) + t[2]
    gx = (R[0, 0] * nx + R[0, 1] * ny) + R[0, 2] * nz
    gy = (R[1, 0] * nx + R[1, 1] * ny) + R[1, 2] * nz
    gz = (R[2, 0] * nx + R[2, 1] * ny) + R[2, 2] * nz
    rx, ry = xs - cx, ys - cy
    norm = f32(np.sqrt(f32(cx * cx + cy * cy)))
    gam = np.sqrt(rx * rx + ry * ry) / norm
    alpha = np.exp(-(gam * gam) / f32(2.0 * sigma * sigma)).astype(f32)
    P = np.stack([wx, wy, wz], axis=-1).astype(f32)
    N = np.stack([gx, gy, gz], axis=-1).astype(f32)
    return valid, P, N, alpha, d


def project(m: SurfelMap, K, pose_w2c, W, H):
    """per surfel: (in front, u, v, rho, z), float32"""
    fx, fy, cx, cy = (f32(v) for v in K[:4])
    M = np.asarray(pose_w2c, f32)
    p = m.pos
    X = ((M[0, 0] * p[:, 0] + M[0, 1] * p[:, 1]) + M[0, 2] * p[:, 2]) + M[0, 3]
    Y = ((M[1, 0] * p[:, 0] + M[1, 1] * p[:, 1]) + M[1, 2] * p[:, 2]) + M[1, 3]
    Z = ((M[2, 0] * p[:, 0] + M[2, 1] * p[:, 1]) + M[2, 2] * p[:, 2]) + M[2, 3]
    front = Z > 0
    with np.errstate(invalid="ignore", divide="ignore", over="ignore"):
        u = (fx * X) / Z + cx
        v = (fy * Y) / Z + cy
        rho = np.minimum((fx * p[:, 3]) / Z, RHO_MAX)
    return front, u, v, rho, Z


def index_map(m: SurfelMap, K, pose_w2c, W, H):
    """(H, W) int32: the covering surfel of least camera z (ties: smaller index), -1 if none"""
    front, u, v, rho, Z = project(m, K, pose_w2c, W, H)
    best = np.full(H * W, np.iinfo(np.uint64).max, np.uint64)
    idx = np.arange(len(u), dtype=np.uint64)
    with np.errstate(invalid="ignore", over="ignore"):
        ok = front & (u + rho >= 0) & (u - rho <= W - 1) & (v + rho >= 0) & (v - rho <= H - 1)
    s = np.flatnonzero(ok)
    if len(s) == 0:
        return np.full((H, W), -1, np.int32)
    u, v, rho, Z = u[s], v[s], rho[s], Z[s]
    x0 = np.ceil(u - rho).astype(np.int64)
    y0 = np.ceil(v - rho).astype(np.int64)
    key = (Z.view(np.uint32).astype(np.uint64) << np.uint64(32)) | idx[s]
    span = int(2 * RHO_MAX) + 2
    for dy in range(span):
        for dx in range(span):
            x = x0 + dx
            y = y0 + dy
            fxp = x.astype(f32) - u
            fyp = y.astype(f32) - v
            inside = ((fxp * fxp + fyp * fyp) <= rho * rho) & (x >= 0) & (x < W) & (y >= 0) & (y < H)
            if not inside.any():
                continue
            pix = y[inside] * W + x[inside]
            np.minimum.at(best, pix, key[inside])
    out = np.where(best == np.iinfo(np.uint64).max, -1, (best & np.uint64(0xffffffff)).astype(np.int64))
    return out.reshape(H, W).astype(np.int32)


def fuse(m: SurfelMap, depth, K, pose_w2c):
    """one frame into the map (in place); returns the correspondence of every
    pixel: surfel index, -1 for a new surfel, -2 for no input point"""
    H, W = np.asarray(depth).shape
    valid, P, N, alpha, d = input_points(depth, K, pose_w2c, m.sigma)
    imap = index_map(m, K, pose_w2c, W, H)
    m.index_map = imap
    corr = np.full((H, W), -2, np.int64)
    corr[valid] = -1
    cand = valid & (imap >= 0)
    if cand.any():
        _, _, _, _, Z = project(m, K, pose_w2c, W, H)
        s = imap[cand]
        zs = Z[s]
        ns = m.nrm[s, :3]
        ng = N[cand]
        dz = np.abs(d[cand] - zs)
        dot = (ng[:, 0] * ns[:, 0] + ng[:, 1] * ns[:, 1]) + ng[:, 2] * ns[:, 2]
        nlen = np.sqrt((ns[:, 0] * ns[:, 0] + ns[:, 1] * ns[:, 1]) + ns[:, 2] * ns[:, 2])
        ok = (dz <= f32(m.delta_z)) & (dot >= f32(m.tau_n) * nlen)
        c = corr[cand]
        c[ok] = s[ok]
        corr[cand] = c
    # updates (S7): sums over each surfel's corresponding points
    sel = corr >= 0
    if sel.any():
        s = corr[sel]
        a = alpha[sel].astype(np.float64)
        n_s = len(m.pos)
        sa = np.zeros(n_s)
        sv = np.zeros((n_s, 3))
        sn = np.zeros((n_s, 3))
        np.add.at(sa, s, a)
        np.add.at(sv, s, a[:, None] * P[sel].astype(np.float64))
        np.add.at(sn, s, a[:, None] * N[sel].astype(np.float64))
        hit = np.flatnonzero(sa > 0)
        c = m.nrm[hit, 3].astype(np.float64)
        den = c + sa[hit]
        m.pos[hit, :3] = ((c[:, None] * m.pos[hit, :3].astype(np.float64) + sv[hit]) / den[:, None]).astype(f32)
        m.nrm[hit, :3] = ((c[:, None] * m.nrm[hit, :3].astype(np.float64) + sn[hit]) / den[:, None]).astype(f32)
        m.nrm[hit, 3] = den.astype(f32)
        m.time[hit] = m.frames
    # new surfels (S8), raster order
    new = np.flatnonzero((corr == -1).reshape(-1))
    room = m.capacity - len(m.pos)
    if len(new) > room:
        m.overflow = True
        new = new[:max(0, room)]
    if len(new):
        fx = f32(K[0])
        dd = d.reshape(-1)[new]
        r = (dd * f32(np.sqrt(2.0) / 2.0)) / fx
        pos = np.concatenate([P.reshape(-1, 3)[new], r[:, None]], axis=1).astype(f32)
        nrm = np.concatenate([N.reshape(-1, 3)[new], alpha.reshape(-1)[new][:, None]], axis=1).astype(f32)
        m.pos = np.concatenate([m.pos, pos])
        m.nrm = np.concatenate([m.nrm, nrm])
        m.time = np.concatenate([m.time, np.full(len(new), m.frames, np.int32)])
    m.frames += 1
    return corr.astype(np.int32)
