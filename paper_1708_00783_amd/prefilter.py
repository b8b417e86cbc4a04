"""Training data, training loop and evaluation of the learned depth prefilter.

Training pairs are produced by the method itself: the noisy frames of a room
are fused, the fused model is raycast from every frame's pose, and the camera
depth of the raycast hits is the target for that frame's raw depth (0 where
the ray misses).  The analytic scene never enters training; it only serves
the evaluation, the surface error of a fused model: the root mean square of
the analytic signed distance at the raycast hit points of a set of
evaluation poses.

Everything numeric on the path runs in the library's kernels (fusion,
raycast, the network's forward, backward and Adam); torch only moves and
slices device buffers.
"""
from __future__ import annotations

import time

import numpy as np

from . import NN_LAYERS, Denoiser, Volume, tf_camera_depth

FRAME_W, FRAME_H = 640, 480


def init_params(seed: int = 0) -> np.ndarray:
    """fp32 parameter vector: He-normal conv weights (std sqrt(2 / (9 cin))),
    zero biases, zero head -- the prefilter starts as the identity"""
    rng = np.random.default_rng(seed)
    parts = []
    for name, cin, cout in NN_LAYERS:
        n = cout * 9 * cin
        w = np.zeros(n) if name == "head" else rng.standard_normal(n) * np.sqrt(2.0 / (9 * cin))
        parts += [w.astype(np.float32), np.zeros(cout, np.float32)]
    return np.concatenate(parts)


def _render(args):
    from synth import configs
    seed_index, k = args
    return configs.c2_frame(k, seed_index)


def render_room(seed_index: int, n: int, workers: int = 1) -> np.ndarray:
    """uint16 mm frames 0..n-1 of the seeded room's trajectory"""
    items = [(seed_index, k) for k in range(n)]
    if workers <= 1:
        return np.stack([_render(a) for a in items])
    import multiprocessing as mp
    with mp.get_context("fork").Pool(workers) as pool:
        return np.stack(pool.map(_render, items, chunksize=max(1, n // (4 * workers))))


def room_poses(seed_index: int, n: int) -> np.ndarray:
    from synth import configs
    return np.stack(configs.c2_poses(max(300, n), seed_index)[:n]).astype(np.float32)


def camera_depth(points, pose, out=None):
    """camera z of world hit points (H, W, 4 device tensor; w = 1 on a hit), 0
    on a miss, by the library's tf_camera_depth"""
    import torch
    if out is None:
        out = torch.empty(points.shape[:2], dtype=torch.float32, device=points.device)
    tf_camera_depth(points, pose, out)
    return out


def fuse_frame(vol: Volume, depth, intr, pose, net: Denoiser | None = None, den_out=None):
    """one frame into the volume, through the prefilter when `net` is given"""
    if net is not None:
        depth = net.forward(depth[None], out=den_out)[0]
    vol.alloc_and_visible(depth, intr, pose)
    vol.integrate(depth, pose)
    return depth


def make_pairs(seed_index: int, n_frames: int, workers: int = 1, vp=None):
    """(raw uint16 frames, target depth in metres), both (n, H, W) device tensors"""
    import torch
    from synth import configs
    vp = vp or configs.C2_VOLUME
    K = configs.KINECT_INTR
    frames = render_room(seed_index, n_frames, workers)
    poses = room_poses(seed_index, n_frames)
    d = torch.from_numpy(frames).cuda()
    vol = Volume(vp, K.width, K.height)
    for k in range(n_frames):
        fuse_frame(vol, d[k], K, poses[k])
    targets = torch.empty((n_frames, K.height, K.width), dtype=torch.float32, device="cuda")
    pts = torch.empty((K.height, K.width, 4), dtype=torch.float32, device="cuda")
    nrm = torch.empty_like(pts)
    for k in range(n_frames):
        vol.raycast(poses[k], K, pts, nrm)
        camera_depth(pts, poses[k], out=targets[k])
    vol.close()
    return d, targets


def train(net: Denoiser, inputs, targets, steps: int, lr: float = 2e-4, seed: int = 0, crop: int = 256,
          log_every: int = 0):
    """Adam on random crops: inputs / targets are lists of (n, H, W) device
    tensors (one per room); batch = the denoiser's batch size."""
    import torch
    rng = np.random.default_rng(seed)
    B = net.B
    assert net.H == crop and net.W == crop
    xin = torch.empty((B, crop, crop), dtype=inputs[0].dtype, device="cuda")
    tgt = torch.empty((B, crop, crop), dtype=torch.float32, device="cuda")
    losses = []
    t0 = time.perf_counter()
    for it in range(steps):
        for b in range(B):
            r = int(rng.integers(len(inputs)))
            k = int(rng.integers(inputs[r].shape[0]))
            y0 = int(rng.integers(inputs[r].shape[1] - crop + 1))
            x0 = int(rng.integers(inputs[r].shape[2] - crop + 1))
            xin[b] = inputs[r][k, y0:y0 + crop, x0:x0 + crop]
            tgt[b] = targets[r][k, y0:y0 + crop, x0:x0 + crop]
        net.forward(xin)
        loss = net.backward(tgt)
        net.adam_step(lr)
        if log_every and (it % log_every == 0 or it == steps - 1):
            losses.append((it, float(loss[0].item()), time.perf_counter() - t0))
    torch.cuda.synchronize()
    return losses, time.perf_counter() - t0


def surface_rms(vol: Volume, scene, poses, intr, stride: int = 4):
    """RMS of the analytic signed distance at the raycast hits of `poses`
    (every `stride`-th pixel in x and y), and the hit count"""
    import torch
    from synth import analytic_sdf
    pts = torch.empty((intr.height, intr.width, 4), dtype=torch.float32, device="cuda")
    nrm = torch.empty_like(pts)
    errs, n = [], 0
    for P in poses:
        vol.raycast(P, intr, pts, nrm)
        p = pts[::stride, ::stride].reshape(-1, 4).cpu().numpy()
        p = p[p[:, 3] == 1.0][:, :3].astype(np.float64)
        if len(p):
            errs.append(analytic_sdf(scene, p))
            n += len(p)
    return rms_of(np.concatenate(errs) if errs else []), n


def rms_of(errors) -> float:
    """surface RMS of signed distances (the evaluation's statistic): sqrt(mean e^2)"""
    e = np.asarray(errors, np.float64).reshape(-1)
    return float(np.sqrt(np.mean(e * e))) if e.size else float("nan")


def equal_error(ns, rms_plain, rms_path, hits_plain, hits_path, t_plain, t_path, coverage=0.95):
    """The equal-error comparison: e* = the plain path's RMS with the most
    frames (the last of `ns`, ascending frame counts); N_d = the smallest N
    at which the other path's RMS <= e* while its evaluation hits reach
    `coverage` of the plain path's with every frame (the RMS is over hits
    only, so a sparse model must also cover the room); ratio = T_plain(all) /
    T_path(N_d).  Returns (e*, N_d, ratio), N_d and ratio None if never."""
    e_star = float(rms_plain[-1])
    h_star = float(hits_plain[-1])
    for j, n in enumerate(ns):
        if rms_path[j] <= e_star and hits_path[j] >= coverage * h_star:
            return e_star, n, float(t_plain[-1]) / float(t_path[j])
    return e_star, None, None


EVAL_STRIDES = (60, 30, 20, 15, 10, 6, 5, 4, 3, 2, 1)   # every k-th frame: N = 300 / k frames


def evaluate_room(seed_index: int, frames, net: Denoiser | None, strides=EVAL_STRIDES, vp=None,
                  eval_every: int = 10, stride: int = 4):
    """Equal-coverage evaluation: for each k, fuse every k-th frame of the
    whole trajectory (raw, or through `net`) into a fresh volume and record
    the surface RMS at every `eval_every`-th trajectory pose and the
    device-synchronised wall time of the fusion (prefilter + allocation +
    integration + raycast per frame).  Returns {N: (rms, seconds, hits)}:
    the RMS is over the evaluation hits only, so `hits` tells how much of
    the room the fused model covers."""
    import torch
    from synth import configs
    vp = vp or configs.C2_VOLUME
    K = configs.KINECT_INTR
    n = frames.shape[0]
    poses = room_poses(seed_index, n)
    scene = configs.c2_scene(seed_index)
    eval_poses = poses[::eval_every]
    pts = torch.empty((K.height, K.width, 4), dtype=torch.float32, device="cuda")
    nrm = torch.empty_like(pts)
    den = torch.empty((1, K.height, K.width), dtype=torch.float32, device="cuda") if net is not None else None
    out = {}
    vol = Volume(vp, K.width, K.height)
    # one untimed frame first: the first launch of a kernel loads its code object
    fuse_frame(vol, frames[0], K, poses[0], net, den)
    vol.raycast(poses[0], K, pts, nrm)
    torch.cuda.synchronize()
    for k in strides:
        vol.reset()
        idx = list(range(0, n, k))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in idx:
            fuse_frame(vol, frames[i], K, poses[i], net, den)
            vol.raycast(poses[i], K, pts, nrm)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        rms, hits = surface_rms(vol, scene, eval_poses, K, stride)
        out[len(idx)] = (rms, dt, hits)
    vol.close()
    return out
