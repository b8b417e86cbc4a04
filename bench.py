"""Benchmark of the fusion hot path on one MI355X.

One step = one depth frame through the whole path: tf_alloc_and_visible
(allocation + visible list), tf_integrate and tf_raycast (points + normals)
from the frame's pose.  Workload: the full-frame configuration -- 640x480
uint16 depth of a seeded 4x4x3 m room with 20 primitives and Kinect-like
noise, voxel 5 mm, mu 2 cm, 2^20 buckets + 2^17 excess slots, 2^18 blocks,
along a 300-frame seeded trajectory.

Inputs are generated and uploaded to HBM before timing.  The whole trajectory
is fused in order: an untimed prefix, W warm-up frames, then the K timed
frames (the trajectory's last K, so the map has its configured size),
bracketed by device synchronisation.  Per-kernel device time comes from HIP
events the library records on its launch stream during the timed frames;
algorithmic bytes from the library's device-side work counters.  The CPU
baseline times the oracle on a bounded prefix of the same trajectory on the
host cores, with all granted threads and with one.

The second half of the metric (denoised vs plain at equal surface error)
follows in `extra.c5`: the prefilter is trained on pairs the method makes
from seeded rooms and both paths fuse held-out rooms (`--no-c5` skips it).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "frames/s integrate+raycast 640x480 @5mm; denoised vs plain at equal RMS error"
HBM_PEAK_GBS = 8000.0
N_TRAJ = 300
PROFILE_EVERY = 8


# the sources the single-volume kernels are built from (the traffic figures of
# profiles/ are keyed by their hash)
KERNEL_SOURCES = ("paper_1708_00783_amd/csrc/tsdf_device.h", "paper_1708_00783_amd/csrc/tsdf_kernels.hip",
                  "paper_1708_00783_amd/csrc/tsdf_internal.h")


def measured_traffic(kernel, timed=None):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 summaries
    (FETCH_SIZE + WRITE_SIZE, copy-calibrated, averaged over the dispatches of
    the timed frames), only if they were taken with the current kernel sources
    and over the same timed frame range `timed` = (first, last); else None"""
    import glob
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    sha = h.hexdigest()[:16]
    want = f"{timed[0]}-{timed[1]}" if timed else None
    for f in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(f):
            m = re.match(r"traffic (\S+) ([0-9a-f]{16}) (\d+)(?: frames=(\d+-\d+))?$", line.strip())
            # the trace names a template instance (k_raycast<true>); match the kernel
            if m and m.group(1).split("<")[0] == kernel and m.group(2) == sha and m.group(4) == want:
                return int(m.group(3))
    return None


def _gen(k):
    from synth import configs
    return configs.c2_frame(k)


def _gen_c4(k):
    from synth import configs
    return configs.c4_frame(k)


def _gen_c3(k):
    from synth import configs
    return configs.c3_frame(k)


def _gen_prefill(ij):
    from synth import configs
    return configs.c4_prefill_frame(*ij)


def _one_thread():
    """render workers: one BLAS/OpenMP thread each (the pool supplies the parallelism)"""
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:
        pass


def pmap(fn, items, workers):
    if workers <= 1:
        return [fn(x) for x in items]
    import multiprocessing as mp
    with mp.get_context("fork").Pool(workers, initializer=_one_thread) as pool:
        return pool.map(fn, items, chunksize=max(1, len(items) // (4 * workers)))


def make_frames(n, workers, cache=None, gen=_gen):
    """frames 0..n-1 (read from / written to `cache`, an .npy path, if given)"""
    if cache and os.path.exists(cache):
        a = np.load(cache)
        if len(a) >= n:
            return a[:n]
    a = np.stack(pmap(gen, list(range(n)), workers))
    if cache:
        np.save(cache, a)
    return a


def cpu_cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_threads():
    """threads for the oracle: the cores this process may run on, capped by
    OMP_NUM_THREADS when the host sets it (a shared GPU host grants a share)"""
    n = cpu_cores()
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return n


def _oracle_fps(frames, poses, K, threads, budget_s, max_frames):
    from oracle import oracle as O
    from synth import configs
    O.set_threads(threads)
    vol = O.Volume.from_params(configs.C2_VOLUME)
    intr = K.as_array()
    t0 = time.perf_counter()
    n = 0
    while n < max_frames and n < len(frames):
        d = O.depth_from_mm(frames[n])
        vol.alloc_and_visible(d, intr, poses[n])
        vol.integrate(d, intr, poses[n])
        vol.raycast(K.width, K.height, intr, poses[n])
        n += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return n / dt, n, dt, O.get_threads()


def cpu_baseline(frames, poses, K, budget_s=12.0, max_frames=150):
    """Oracle frames/s on a prefix of the trajectory (bounded wall time), with
    all granted host threads and with one thread."""
    fps, n, dt, used = _oracle_fps(frames, poses, K, cpu_threads(), budget_s, max_frames)
    fps1, n1, dt1, _ = _oracle_fps(frames, poses, K, 1, budget_s, max_frames)
    return {"value": fps, "unit": "frames/s", "cores": used, "kind": "oracle",
            "sample": f"first {n} frames of the same trajectory (alloc+integrate+raycast each), "
                      f"{dt:.1f} s on the host",
            "one_thread": {"value": fps1, "cores": 1,
                           "sample": f"first {n1} frames of the same trajectory, {dt1:.1f} s"},
            "host_cores_visible": cpu_cores(),
            "omp_num_threads_env": os.environ.get("OMP_NUM_THREADS"),
            "cpu_model": _cpu_model()}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


C4_BIN_CAP = 1 << 27      # (block, tile) entries of one raycast call over its 8 views (4 GiB)


def c4_prefill(mm, workers, max_frames=48, batch=4):
    """Fill every submap from noiseless viewpoints in its region until it
    holds its target block count (or max_frames frames)."""
    import torch
    from synth import configs
    subs = configs.c4_submaps()
    counts = [0] * len(subs)
    nxt = [0] * len(subs)
    need = list(range(len(subs)))
    used = 0
    while need:
        items = [(i, nxt[i] + b) for i in need for b in range(batch)]
        depths = pmap(_gen_prefill, items, workers)
        for (i, j), dep in zip(items, depths):
            if counts[i] >= subs[i].target:
                continue
            mm.integrate(torch.from_numpy(dep).cuda(), configs.C4_PREFILL_INTR, configs.c4_prefill_pose(i, j), [i])
            counts[i] = mm.submap(i).stats()["n_allocated"]
            used += 1
        for i in need:
            nxt[i] += batch
        need = [i for i in need if counts[i] < subs[i].target and nxt[i] < max_frames]
        print(f"[bench] prefill: {used} frames, {sum(counts)} blocks, {len(need)} submaps below target",
              file=sys.stderr, flush=True)
    return counts, used


C3_TRANSFER = 8192          # blocks per swap-in / swap-out call (12.6 MB of transfer buffer)


def run_c3(args):
    """C3: the large multi-room walk (4 mm voxels, 2^20 device blocks) with host
    swapping every frame: allocation + swap-in, integration, raycast, swap-out.
    Both swap calls synchronise with the host (it needs the candidate counts),
    so each frame is timed from its first launch to the end of its swap-out."""
    import torch
    import paper_1708_00783_amd as T
    from synth import configs
    K = configs.KINECT_INTR
    n = min(1500, args.warmup + args.steps)
    frames = make_frames(n, args.workers, args.frames_cache, gen=_gen_c3)
    poses = np.stack(configs.c3_poses(1500)[:n]).astype(np.float32)
    torch.cuda.set_device(0)
    d = torch.from_numpy(frames).cuda()
    vol = T.Volume(configs.C3_VOLUME, K.width, K.height, swap_transfer_blocks=C3_TRANSFER)
    pts = torch.empty((K.height, K.width, 4), dtype=torch.float32, device="cuda")
    nrm = torch.empty_like(pts)

    def frame(k):
        vol.alloc_and_visible(d[k], K, poses[k])
        vol.integrate(d[k], poses[k])
        vol.raycast(poses[k], K, pts, nrm)
        vol.swap_out()

    for k in range(args.warmup):
        frame(k)
    torch.cuda.synchronize()
    vol.profile_enable(True)
    vol.profile_select(("integrate", "raycast", "swap"), PROFILE_EVERY)
    vol.profile_read(reset=True)
    s0 = vol.stats()
    dt, sw_in, sw_out, hits, dev_blocks = 0.0, 0, 0, 0, []
    for k in range(args.warmup, n):
        t0 = time.perf_counter()
        frame(k)
        torch.cuda.synchronize()
        dt += time.perf_counter() - t0
        st = vol.stats()
        sw_in += st["n_swapped_in"]
        sw_out += st["n_swapped_out"]
        dev_blocks.append(st["n_allocated"])
    s1 = vol.stats()
    prof = vol.profile_read()
    assert s1["flags"] == 0, f"capacity flags raised: {s1['flags']:#x}"
    steps = n - args.warmup
    WH = K.width * K.height
    d_rec = s1["total_range_records"] - s0["total_range_records"]
    ray_ms = prof["raycast"]["ms"] / max(1, prof["raycast"]["launches"])
    ray_bytes = d_rec * (1024 + 16) / steps + 32 * WH
    gbs = ray_bytes / (ray_ms * 1e-3) / 1e9 if ray_ms > 0 else 0.0
    out = {
        "metric": "frames/s: alloc + swap-in + integrate + raycast + swap-out, large multi-room walk",
        "value": round(steps / dt, 3), "unit": "frames/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * dt / steps, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "large scene: 640x480 uint16 depth walking a 12x12x3 m 3x3-room layout with 200 "
                               "primitives, voxel 4 mm, mu 1.6 cm, 2^22 buckets + 2^19 excess, 2^20 device blocks, "
                               f"host store per entry, {C3_TRANSFER}-block transfer buffer, swap-out every frame",
                   "frames": n},
        "roofline": {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 5), "traffic": None, "kernel": "raycast",
                     "algorithmic_bytes_per_launch": int(ray_bytes), "avg_launch_ms": round(ray_ms, 5)},
        "cpu_baseline": None,
        "extra": {"swapped_in_per_frame": round(sw_in / steps, 1), "swapped_out_per_frame": round(sw_out / steps, 1),
                  "pcie_mb_per_frame": round((sw_in + sw_out) * (1536 + 4) / steps / 1e6, 3),
                  "device_blocks_last": dev_blocks[-1], "device_blocks_max": max(dev_blocks),
                  "kernel_ms_per_launch": {k: round(v["ms"] / max(1, v["launches"]), 5) for k, v in prof.items()
                                           if v["launches"]},
                  "avg_visible_blocks": round((s1["total_integrated_blocks"] - s0["total_integrated_blocks"]) / steps, 1),
                  "hit_fraction": round((s1["total_rays_hit"] - s0["total_rays_hit"]) / (steps * WH), 4)},
    }
    print(json.dumps(out), flush=True)


def run_c4(args):
    """64 batched submaps: per frame one 640x480 depth fused into the submaps it
    overlaps and 8 views raycast on the combined field, as one graph replay."""
    from synth import configs
    K = configs.KINECT_INTR
    n_frames = args.warmup + args.steps
    print(f"[bench] c4: generating {n_frames} frames", file=sys.stderr, flush=True)
    frames = make_frames(n_frames, args.workers, args.frames_cache, gen=_gen_c4)
    poses = configs.c4_poses()
    import torch
    import paper_1708_00783_amd as T
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    subs = configs.c4_submaps()
    mm = T.MultiMap(configs.C4_VOLUME, np.stack([s.pose for s in subs]), K.width, K.height, 1280, 720, C4_BIN_CAP)
    counts, used = c4_prefill(mm, args.workers)
    d_frames = torch.from_numpy(frames).cuda()
    outs = [(torch.empty((H, W, 4), dtype=torch.float32, device="cuda"),
             torch.empty((H, W, 4), dtype=torch.float32, device="cuda")) for W, H in configs.C4_VIEW_SIZES]
    sels = [configs.c4_select(poses[k % configs.C4_N_FRAMES]) for k in range(n_frames)]

    def views_of(k):
        return [(intr, pose, o[0], o[1]) for (intr, pose), o in zip(configs.c4_views(k), outs)]

    def step(k, graph=True):
        mm.frame(d_frames[k], K, poses[k % configs.C4_N_FRAMES], sels[k], views_of(k), use_graph=graph, stream=stream)

    step(0, graph=False)
    for k in range(1, args.warmup):
        step(k)
    if args.c4_tile:
        tw, th = (int(x) for x in args.c4_tile.split("x"))
        mm.set_config(tile_w=tw, tile_h=th)
        best = mm.get_config().as_dict()
        print(f"[bench] c4 fixed shape: {best}", file=sys.stderr, flush=True)
    else:
        # tuned on the first timed frame: the submaps grow over the run, so an
        # early frame would pick for a lighter workload
        w = args.warmup
        best, best_ms = mm.autotune(d_frames[w], K, poses[w % configs.C4_N_FRAMES], sels[w], views_of(w), reps=3,
                                    stream=stream)
        print(f"[bench] c4 autotune: {best} ({best_ms:.3f} ms)", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    s0 = mm.stats()
    t0 = time.perf_counter()
    for k in range(args.warmup, n_frames):
        step(k)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    s1 = mm.stats()
    assert s1["flags"] == 0, f"capacity flags raised: {s1['flags']:#x}"
    # raycast phase alone (binning + combined-field raycast), HIP events on the stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    nr = min(20, args.steps)
    r0 = mm.stats()
    e0.record(stream)
    for k in range(nr):
        mm.raycast(views_of(args.warmup + k), stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    r1 = mm.stats()
    ray_ms = e0.elapsed_time(e1) / nr
    steps = args.steps
    d_blocks = s1["total_integrated_blocks"] - s0["total_integrated_blocks"]
    d_cols = s1["total_written_columns"] - s0["total_written_columns"]
    pix = sum(W * H for W, H in configs.C4_VIEW_SIZES)
    bv = (r1["total_block_views"] - r0["total_block_views"]) / nr
    be = (r1["total_bin_entries"] - r0["total_bin_entries"]) / nr
    ray_bytes = bv * (1536 + 16) + be * 32 * 2 + 32 * pix
    gbs = ray_bytes / (ray_ms * 1e-3) / 1e9
    out = {
        "metric": "frames/s: fuse into overlapping submaps + raycast 8 views on the combined field",
        "value": round(steps / dt, 3), "unit": "frames/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * dt / steps, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batched submaps: 64 rigid submaps (log-uniform 2k-60k blocks, voxel 5 mm, "
                               "mu 2 cm) over a 12x12x3 m multi-room layout; per frame one 640x480 uint16 depth "
                               "fused into its 4-12 overlapping submaps and 8 views (2 each 320x240, 640x480, "
                               "960x540, 1280x720) raycast, one HIP graph replay per frame",
                   "submaps": len(subs), "views": len(configs.C4_VIEW_SIZES)},
        "roofline": {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 5), "traffic": None, "kernel": "raycast phase",
                     "algorithmic_bytes_per_launch": int(ray_bytes), "avg_launch_ms": round(ray_ms, 5)},
        "cpu_baseline": None,
        "extra": {"prefill_frames": used, "blocks_after_prefill": int(sum(counts)),
                  "allocated_blocks": s1["allocated_blocks"], "autotuned": best,
                  "avg_selected_submaps": float(np.mean([len(x) for x in sels[args.warmup:]])),
                  "voxel_updates_per_s": d_blocks * 512 / dt,
                  "avg_integrated_blocks": d_blocks / steps, "avg_written_columns": d_cols / steps,
                  "raycast_phase_ms": round(ray_ms, 4), "avg_block_views": bv, "avg_bin_entries": be,
                  "hit_fraction": (s1["total_rays_hit"] - s0["total_rays_hit"]) / (steps * pix)},
    }
    print(json.dumps(out), flush=True)


def _render_c5(item):
    from synth import configs
    seed, k = item
    return configs.c2_frame(k, seed)


def render_rooms(seeds, n, workers, tag):
    """uint16 frames 0..n-1 of every seeded room, rendered before any GPU work"""
    import multiprocessing as mp
    items = [(s, k) for s in seeds for k in range(n)]
    out = []
    with mp.get_context("fork").Pool(max(1, workers), initializer=_one_thread) as pool:
        for i, f in enumerate(pool.imap(_render_c5, items, chunksize=8)):
            out.append(f)
            if (i + 1) % 500 == 0:
                print(f"[bench] c5 {tag}: {i + 1}/{len(items)} frames", file=sys.stderr, flush=True)
    a = np.stack(out)
    return [a[i * n:(i + 1) * n] for i in range(len(seeds))]


C5_COVERAGE = 0.95
C5_BILATERAL = (2, 2.5, 0.025)     # radius (px), sigma_space (px), sigma_range (m)


def run_c5(args):
    print(json.dumps(c5_result(args)), flush=True)


def c5_result(args):
    """Train the prefilter on pairs the method makes itself (fused-model
    raycasts as targets), then fuse held-out rooms with raw and with denoised
    depth: e* = raw surface RMS with all frames fused; N_d = the smallest
    frame count (every k-th frame of the whole trajectory) at which the
    denoised RMS <= e*; report the time each path takes."""
    from synth import configs
    t_all = time.perf_counter()
    tr_seeds = list(range(5000, 5000 + args.c5_rooms))
    ev_seeds = list(range(6000, 6000 + args.c5_eval_rooms))
    nf, ne = args.c5_frames, args.c5_eval_frames
    t_render = time.perf_counter()
    train_frames = render_rooms(tr_seeds, nf, args.workers, "training")
    eval_frames = render_rooms(ev_seeds, ne, args.workers, "evaluation")
    t_render = time.perf_counter() - t_render
    import torch
    import paper_1708_00783_amd as T
    from paper_1708_00783_amd import prefilter as PF
    torch.cuda.set_device(0)
    K = configs.KINECT_INTR
    # training pairs: fuse each room, raycast the model at every pose
    t0 = time.perf_counter()
    inputs, targets = [], []
    for i, s in enumerate(tr_seeds):
        d = torch.from_numpy(train_frames[i]).cuda()
        vol = T.Volume(configs.C2_VOLUME, K.width, K.height)
        poses = PF.room_poses(s, nf)
        for k in range(nf):
            PF.fuse_frame(vol, d[k], K, poses[k])
        tg = torch.empty((nf, K.height, K.width), dtype=torch.float32, device="cuda")
        pts = torch.empty((K.height, K.width, 4), dtype=torch.float32, device="cuda")
        nrm = torch.empty_like(pts)
        for k in range(nf):
            vol.raycast(poses[k], K, pts, nrm)
            PF.camera_depth(pts, poses[k], out=tg[k])
        vol.close()
        inputs.append(d)
        targets.append(tg)
    torch.cuda.synchronize()
    t_pairs = time.perf_counter() - t0
    print(f"[bench] c5: {len(tr_seeds) * nf} training pairs in {t_pairs:.1f} s", file=sys.stderr, flush=True)
    net = T.Denoiser(8, 256, 256, training=True)
    net.set_params(PF.init_params(0))
    losses, t_train = PF.train(net, inputs, targets, args.c5_steps, lr=args.c5_lr, seed=0, log_every=100)
    print(f"[bench] c5: trained {args.c5_steps} steps in {t_train:.1f} s, loss {losses[0][1]:.5f} -> "
          f"{losses[-1][1]:.5f}", file=sys.stderr, flush=True)
    params = net.get_params()
    if args.c5_save:
        np.save(args.c5_save, params.cpu().numpy())
    del inputs, targets
    inf = T.Denoiser(1, K.height, K.width)
    inf.set_params(params)
    # held-out rooms, equal-coverage protocol (every k-th frame of the whole trajectory)
    # the paper's own prefilter, the bilateral filter, as the comparator
    bil = T.Bilateral(K.height, K.width, *C5_BILATERAL)
    res = {"raw": [], "denoised": [], "bilateral": []}
    for i, s in enumerate(ev_seeds):
        d = torch.from_numpy(eval_frames[i]).cuda()
        for name, nn in (("raw", None), ("denoised", inf), ("bilateral", bil)):
            res[name].append(PF.evaluate_room(s, d, nn))
        print(f"[bench] c5: room {s}: raw {res['raw'][-1][ne][0] * 1e3:.3f} mm, denoised "
              f"{res['denoised'][-1][ne][0] * 1e3:.3f} mm with all {ne} frames", file=sys.stderr, flush=True)
    ns = sorted(res["raw"][0])
    raw = np.array([np.mean([r[n][0] for r in res["raw"]]) for n in ns])
    den = np.array([np.mean([r[n][0] for r in res["denoised"]]) for n in ns])
    traw = np.array([np.mean([r[n][1] for r in res["raw"]]) for n in ns])
    tden = np.array([np.mean([r[n][1] for r in res["denoised"]]) for n in ns])
    hraw = np.array([np.mean([r[n][2] for r in res["raw"]]) for n in ns])
    hden = np.array([np.mean([r[n][2] for r in res["denoised"]]) for n in ns])
    # the same with the median over rooms (one room with a large error on both
    # paths should not decide the comparison)
    raw_md = np.array([np.median([r[n][0] for r in res["raw"]]) for n in ns])
    den_md = np.array([np.median([r[n][0] for r in res["denoised"]]) for n in ns])
    # equal error at equal coverage: the RMS is over evaluation hits only, so a
    # model fused from few frames must also cover the room (>= 95% of the raw
    # path's hits with every frame) before its error counts
    e_star, nd, ratio = PF.equal_error(ns, raw, den, hraw, hden, traw, tden, C5_COVERAGE)
    _, nd_md, ratio_md = PF.equal_error(ns, raw_md, den_md, hraw, hden, traw, tden, C5_COVERAGE)
    bl = np.array([np.mean([r[n][0] for r in res["bilateral"]]) for n in ns])
    tbl = np.array([np.mean([r[n][1] for r in res["bilateral"]]) for n in ns])
    hbl = np.array([np.mean([r[n][2] for r in res["bilateral"]]) for n in ns])
    _, nd_bl, ratio_bl = PF.equal_error(ns, raw, bl, hraw, hbl, traw, tbl, C5_COVERAGE)
    t_plain = float(traw[-1])
    t_den = float(tden[list(ns).index(nd)]) if nd is not None else None
    cps = ns
    out = {
        "metric": "denoised vs plain at equal surface RMS error (time to reach the plain path's error)",
        "value": round(ratio, 4) if ratio is not None else None, "unit": "x (T_plain(300) / T_denoised(N_d))",
        "n_gpus": 1, "higher_is_better": True, "vs_baseline": None, "dtype": "bf16 prefilter, f32 fusion",
        "data": "synthetic",
        "config": {"workload": "learned prefilter: 4-level 3x3 conv encoder-decoder (32/64/64/128), bf16 on "
                               "matrix cores, trained on (raw depth, fused-model raycast) pairs of seeded C2 rooms; "
                               "evaluated on held-out rooms fused raw vs denoised",
                   "train_rooms": len(tr_seeds), "frames_per_room": nf, "pairs": len(tr_seeds) * nf,
                   "steps": args.c5_steps, "batch": 8, "crop": 256, "eval_rooms": len(ev_seeds),
                   "eval_frames": ne, "eval_pose_every": 10, "eval_pixel_stride": 4},
        "e_star_mm": round(e_star * 1e3, 4), "n_d": nd, "t_plain_s": round(t_plain, 4),
        "t_denoised_s": round(t_den, 4) if t_den else None,
        "frames_per_s_plain": round(ne / t_plain, 2),
        "frames_per_s_denoised": round(float(ns[-1] / tden[-1]), 2),
        "rms_mm": {"frames_fused": cps, "raw": [round(v * 1e3, 4) for v in raw],
                   "denoised": [round(v * 1e3, 4) for v in den]},
        "bilateral": {"params": {"radius": C5_BILATERAL[0], "sigma_space_px": C5_BILATERAL[1],
                                 "sigma_range_m": C5_BILATERAL[2]},
                      "n_d": nd_bl, "ratio": round(ratio_bl, 4) if ratio_bl is not None else None,
                      "rms_mm": [round(v * 1e3, 4) for v in bl],
                      "frames_per_s": round(float(ns[-1] / tbl[-1]), 2)},
        "median_over_rooms": {"e_star_mm": round(float(raw_md[-1]) * 1e3, 4),
                              "n_d": nd_md, "ratio": round(ratio_md, 4) if ratio_md is not None else None,
                              "raw_mm": [round(v * 1e3, 4) for v in raw_md],
                              "denoised_mm": [round(v * 1e3, 4) for v in den_md]},
        "per_room_mm_at_300": {"raw": [round(r[ns[-1]][0] * 1e3, 4) for r in res["raw"]],
                               "denoised": [round(r[ns[-1]][0] * 1e3, 4) for r in res["denoised"]]},
        "eval_hits": {"raw": [int(v) for v in hraw], "denoised": [int(v) for v in hden],
                      "coverage_required": C5_COVERAGE},
        "protocol": "each N fuses every (300/N)-th frame of the whole trajectory into a fresh volume (equal "
                    "coverage); RMS of the analytic SDF at the hits of every 10th pose, every 4th pixel; N_d "
                    "also needs >= 95% of the raw path's evaluation hits at N = 300",
        "train": {"loss_curve": [(a, round(b, 6)) for a, b, _ in losses], "seconds": round(t_train, 2),
                  "pairs_seconds": round(t_pairs, 2), "render_seconds": round(t_render, 2)},
        "seconds": round(time.perf_counter() - t_all, 1),
    }
    return out


# the equal-error half of the headline, run after the frame-rate half: a
# protocol sized to finish in about two minutes on a 16-core host share
C5_IN_C2 = {"c5_rooms": 50, "c5_frames": 40, "c5_steps": 2000, "c5_eval_rooms": 4, "c5_eval_frames": 300}


def c5_summary(args):
    a = argparse.Namespace(**vars(args))
    for k, v in C5_IN_C2.items():
        setattr(a, k, v)
    a.c5_save = None
    r = c5_result(a)
    keep = ("value", "unit", "config", "e_star_mm", "n_d", "t_plain_s", "t_denoised_s", "frames_per_s_plain",
            "frames_per_s_denoised", "rms_mm", "bilateral", "median_over_rooms", "eval_hits", "protocol", "seconds")
    out = {k: r[k] for k in keep}
    out["metric"] = "denoised vs plain at equal surface RMS error: T_plain(300 frames) / T_denoised(N_d frames)"
    out["train_seconds"] = r["train"]["seconds"]
    out["final_loss"] = r["train"]["loss_curve"][-1][1] if r["train"]["loss_curve"] else None
    return out


def run_track(args):
    """The tracking loop of Sec. 4.1.1 on the full-frame room trajectory: each
    frame is tracked against the raycast of the model at the previous estimate
    (tf_track, 3 levels, 4/5/10 iterations), then fused and raycast at the new
    estimate.  One step = track + allocate + integrate + raycast."""
    import torch
    import paper_1708_00783_amd as T
    from synth import configs
    K = configs.KINECT_INTR
    n = min(N_TRAJ, args.warmup + args.steps + 1)
    frames = make_frames(n, args.workers, args.frames_cache)
    truth = np.stack(configs.c2_poses(N_TRAJ)).astype(np.float32)
    torch.cuda.set_device(0)
    d = torch.from_numpy(frames).cuda()
    vol = T.Volume(configs.C2_VOLUME, K.width, K.height)
    trk = T.Tracker(K.width, K.height, 3)
    prm = T.make_track_params((4, 5, 10), (0.1, 0.2, 0.3))
    pts = torch.empty((K.height, K.width, 4), dtype=torch.float32, device="cuda")
    nrm = torch.empty_like(pts)
    est = [truth[0]]
    vol.frame(d[0], K, truth[0], pts, nrm)
    ev = []

    def step(k, timed):
        if timed:
            e = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            e[0].record()
        trk.track_async(d[k], K, pts, nrm, K, est[-1], est[-1], prm)
        if timed:
            e[1].record()
            ev.append(e)
        # the estimate is read back for the host-side pose arguments of fusion
        r = T.parse_track_result(trk.result.cpu().numpy())
        est.append(r["pose_w2c"])
        vol.frame(d[k], K, est[-1], pts, nrm)
        return r

    for k in range(1, 1 + args.warmup):
        step(k, False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pairs = []
    for k in range(1 + args.warmup, n):
        r = step(k, True)
        pairs.append(r["pairs"][:3])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    steps = n - 1 - args.warmup
    ms_track = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    Ra, Rb = est[-1][:3, :3].T, truth[n - 1][:3, :3].T
    ta, tb = -(Ra @ est[-1][:3, 3]), -(Rb @ truth[n - 1][:3, 3])
    drift_mm = float(np.linalg.norm(ta - tb) * 1e3)
    # algorithmic bytes of one tracking call: per sums launch the level's depth
    # (4 B per pixel) and the V and N gathers of every pair (32 B)
    WH = [K.width * K.height >> (2 * l) for l in range(3)]
    p_mean = np.mean(np.array(pairs, np.float64), axis=0)
    its = (4, 5, 10)
    call_bytes = sum(its[l] * (4 * WH[l] + 32 * p_mean[l]) for l in range(3)) + 6 * WH[0]
    gbs = call_bytes / (ms_track * 1e-3) / 1e9
    # the oracle's tracking call on a bounded sample of the same inputs
    from oracle import track as OT
    V, N = pts.cpu().numpy(), nrm.cpu().numpy()
    dm = frames[n - 1].astype(np.float32) / np.float32(1000.0)
    t0 = time.perf_counter()
    m = 0
    while m < 5 and time.perf_counter() - t0 < 15.0:
        OT.track(dm, K.as_array(), V, N, K.as_array(), est[-2], est[-2], [4, 5, 10], [0.1, 0.2, 0.3])
        m += 1
    cpu = m / (time.perf_counter() - t0)
    out = {
        "metric": "tracked frames/s (point-to-plane tracking + alloc + integrate + raycast, 640x480 @5mm)",
        "value": round(steps / dt, 3), "unit": "frames/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * dt / steps, 4), "higher_is_better": True, "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "full-frame room trajectory, each frame tracked against the raycast at the previous "
                               "estimate (3 levels, 4/5/10 iterations, 0.1/0.2/0.3 m gates) and fused at the estimate",
                   "frames": n},
        "roofline": {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 5), "traffic": None, "kernel": "tf_track (whole call)",
                     "algorithmic_bytes_per_call": int(call_bytes), "avg_call_ms": round(ms_track, 5)},
        "cpu_baseline": {"value": round(cpu, 3), "unit": "tracking calls/s", "cores": 1, "kind": "oracle",
                         "sample": f"{m} calls of the numpy oracle on the last frame's inputs"},
        "extra": {"tf_track_ms": round(ms_track, 5), "avg_pairs_per_level": [int(v) for v in p_mean],
                  "drift_mm_at_end": round(drift_mm, 3),
                  "host_readback": "the estimate is copied to the host after each call (fusion takes host poses)"},
    }
    print(json.dumps(out), flush=True)


def _events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def run_filter(args):
    """The bilateral depth filter (radius 2, sigma 2.5 px / 25 mm) on 640x480
    uint16 frames; the oracle filters a bounded sample on the host."""
    import torch
    import paper_1708_00783_amd as T
    from oracle.bilateral import bilateral
    frames = make_frames(8, args.workers, args.frames_cache)
    torch.cuda.set_device(0)
    d = torch.from_numpy(frames).cuda()
    out = torch.empty(frames.shape[1:], dtype=torch.float32, device="cuda")
    for k in range(args.warmup):
        T.tf_bilateral(d[k % 8], out, *C5_BILATERAL)
    torch.cuda.synchronize()
    e0, e1 = _events()
    e0.record()
    for k in range(args.steps):
        T.tf_bilateral(d[k % 8], out, *C5_BILATERAL)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    H, W = frames.shape[1:]
    nbytes = (2 + 4) * W * H
    t0 = time.perf_counter()
    n = 0
    while n < 8 and time.perf_counter() - t0 < 10.0:
        bilateral(frames[n].astype(np.float32) / np.float32(1000.0), *C5_BILATERAL)
        n += 1
    cpu = n / (time.perf_counter() - t0)
    out_line = {
        "metric": "bilateral-filtered frames/s (640x480 uint16 in, float32 out)", "value": round(1e3 / ms, 2),
        "unit": "frames/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": True,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "bilateral filter of full-frame room depth frames", "radius": C5_BILATERAL[0],
                   "sigma_space_px": C5_BILATERAL[1], "sigma_range_m": C5_BILATERAL[2]},
        "roofline": {"bound": "hbm", "achieved": round(nbytes / (ms * 1e-3) / 1e9, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 5), "traffic": None,
                     "kernel": "k_bilateral", "algorithmic_bytes_per_launch": nbytes, "avg_launch_ms": round(ms, 5)},
        "cpu_baseline": {"value": round(cpu, 3), "unit": "frames/s", "cores": 1, "kind": "oracle",
                         "sample": f"{n} frames, float64 numpy oracle (vectorised over pixels)"},
    }
    print(json.dumps(out_line), flush=True)


def run_mesh(args):
    """Marching-cubes meshing of the full-frame room after fusing its
    300-frame trajectory; the oracle meshes a bounded sample of the blocks."""
    import ctypes
    import torch
    import paper_1708_00783_amd as T
    from oracle import mesh as OM
    from synth import configs
    K = configs.KINECT_INTR
    frames = make_frames(N_TRAJ, args.workers, args.frames_cache)
    poses = np.stack(configs.c2_poses(N_TRAJ)).astype(np.float32)
    torch.cuda.set_device(0)
    d = torch.from_numpy(frames).cuda()
    vol = T.Volume(configs.C2_VOLUME, K.width, K.height)
    for k in range(N_TRAJ):
        vol.frame(d[k], K, poses[k])
    torch.cuda.synchronize()
    nb = vol.stats()["n_allocated"]
    nbytes_ws = int(T.lib().tf_mesh_workspace_bytes(ctypes.byref(vol.params)))
    ws = torch.empty(nbytes_ws, dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    T.check(T.lib().tf_mesh(vol.ctx, None, None, 0, ctypes.c_void_p(cnt.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                            nbytes_ws, T._stream_ptr(None)), "tf_mesh")
    ntri = int(cnt.item())
    verts = torch.empty((ntri, 3, 3), dtype=torch.float32, device="cuda")
    keys = torch.empty((ntri, 3), dtype=torch.int64, device="cuda")

    def call():
        T.check(T.lib().tf_mesh(vol.ctx, ctypes.c_void_p(verts.data_ptr()), ctypes.c_void_p(keys.data_ptr()), ntri,
                                ctypes.c_void_p(cnt.data_ptr()), ctypes.c_void_p(ws.data_ptr()), nbytes_ws,
                                T._stream_ptr(None)), "tf_mesh")
    for _ in range(args.warmup):
        call()
    torch.cuda.synchronize()
    e0, e1 = _events()
    e0.record()
    for _ in range(args.steps):
        call()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    n_entries = configs.C2_VOLUME.n_buckets + configs.C2_VOLUME.n_excess
    # two walks over the entries, each reading every allocated block and its
    # halo (217 voxels of 3 bytes), plus the triangles written (9 floats + 3 keys)
    nbytes = 2 * (16 * n_entries + nb * (1536 + 217 * 3)) + ntri * (36 + 24)
    # oracle: a bounded sample of blocks (it needs the neighbours of each)
    pos, sdf, w = vol.voxels_by_position()
    t0 = time.perf_counter()
    m = 0
    step = 256
    while m < len(pos) and time.perf_counter() - t0 < 15.0:
        OM.mesh(pos[m:m + step], sdf[m:m + step], w[m:m + step], configs.C2_VOLUME.voxel_size)
        m += step
    cpu = m / (time.perf_counter() - t0)
    out = {
        "metric": "blocks meshed per second (marching cubes over every allocated block)",
        "value": round(nb / (ms * 1e-3), 1), "unit": "blocks/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "higher_is_better": True, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "mesh of the full-frame room after its 300-frame trajectory (voxel 5 mm)",
                   "allocated_blocks": nb, "triangles": ntri},
        "roofline": {"bound": "hbm", "achieved": round(nbytes / (ms * 1e-3) / 1e9, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 5), "traffic": None,
                     "kernel": "tf_mesh (count, scan, emit)", "algorithmic_bytes_per_call": int(nbytes),
                     "avg_call_ms": round(ms, 5)},
        "cpu_baseline": {"value": round(cpu, 1), "unit": "blocks/s", "cores": 1, "kind": "oracle",
                         "sample": f"{m} of {len(pos)} blocks in groups of {step} (neighbours outside a group "
                                   "count as absent)"},
    }
    print(json.dumps(out), flush=True)


def run_surfel(args):
    """Surfel fusion (Sec. 7.3) along the full-frame room trajectory: W
    warm-up frames, then K timed frames (each: input points, index map of
    every surfel, association, update, new surfels); the oracle fuses a
    bounded sample on the host."""
    import torch
    import paper_1708_00783_amd as T
    from oracle import surfel as OS
    from synth import configs
    K = configs.KINECT_INTR
    n = min(N_TRAJ, args.warmup + args.steps)
    frames = make_frames(n, args.workers, args.frames_cache)
    poses = np.stack(configs.c2_poses(N_TRAJ)).astype(np.float32)
    torch.cuda.set_device(0)
    d = torch.from_numpy(frames).cuda()
    g = T.SurfelMap(1 << 24, K.width, K.height)
    for k in range(args.warmup):
        g.fuse(d[k], K, poses[k])
    torch.cuda.synchronize()
    n0 = g.stats()["count"]
    e0, e1 = _events()
    e0.record()
    for k in range(args.warmup, n):
        g.fuse(d[k], K, poses[k])
    e1.record()
    torch.cuda.synchronize()
    steps = n - args.warmup
    ms = e0.elapsed_time(e1) / steps
    st = g.stats()
    n1 = st["count"]
    WH = K.width * K.height
    mean_surfels = 0.5 * (n0 + n1)
    # per frame: each pixel's depth (2 B) read, its point and normal written and
    # read back (2 x 32 B), z-buffer word written, set and read (3 x 8 B),
    # correspondence written and read (2 x 4 B); each surfel's position read
    # twice (2 x 16 B) and its normal once (16 B); new surfels written (36 B)
    nbytes = WH * (2 + 64 + 24 + 8) + mean_surfels * 48 + (n1 - n0) / steps * 36
    # oracle: the first frames from an empty map
    t0 = time.perf_counter()
    o = OS.SurfelMap(1 << 24)
    m = 0
    while m < 3 and time.perf_counter() - t0 < 15.0:
        OS.fuse(o, frames[m].astype(np.float32) / np.float32(1000.0), K.as_array(), poses[m])
        m += 1
    cpu = m / (time.perf_counter() - t0)
    out = {
        "metric": "surfel-fused frames/s (640x480, index map of every surfel per frame)", "value": round(1e3 / ms, 2),
        "unit": "frames/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup, "higher_is_better": True,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "full-frame room trajectory fused into a surfel map", "frames": n,
                   "surfels_at_start": n0, "surfels_at_end": n1},
        "roofline": {"bound": "hbm", "achieved": round(nbytes / (ms * 1e-3) / 1e9, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 5), "traffic": None,
                     "kernel": "tf_surfel_fuse (whole frame)", "algorithmic_bytes_per_frame": int(nbytes),
                     "avg_frame_ms": round(ms, 5)},
        "cpu_baseline": {"value": round(cpu, 3), "unit": "frames/s", "cores": 1, "kind": "oracle",
                         "sample": f"the first {m} frames from an empty map (numpy oracle)"},
        "extra": {"flags": st["flags"]},
    }
    print(json.dumps(out), flush=True)


MFMA_BF16_PEAK_TFLOPS = 2500.0


def prefilter_flop(h, w, n):
    """forward multiply-add flops of the conv stack for n frames of h x w"""
    convs = ((3, 32, 1), (32, 64, 2), (64, 64, 4), (64, 128, 8), (128, 64, 4), (64, 64, 2), (64, 32, 1), (32, 1, 1))
    return n * sum(2.0 * 9 * ci * co * (h // s) * (w // s) for ci, co, s in convs)


def run_prefilter(args):
    """The prefilter's kernels alone: 640x480 inference and batch-8 256x256
    training steps (forward, loss, backward, Adam) on seeded inputs."""
    import torch
    import paper_1708_00783_amd as T
    from paper_1708_00783_amd import prefilter as PF
    from synth import configs
    torch.cuda.set_device(0)
    frames = make_frames(8, args.workers, args.frames_cache)
    d = torch.from_numpy(frames).cuda()
    inf = T.Denoiser(1, 480, 640)
    inf.set_params(PF.init_params(0))
    out = torch.empty((1, 480, 640), dtype=torch.float32, device="cuda")
    for k in range(args.warmup):
        inf.forward(d[k % 8][None], out=out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(args.steps):
        inf.forward(d[k % 8][None], out=out)
    e1.record()
    torch.cuda.synchronize()
    ms_inf = e0.elapsed_time(e1) / args.steps
    tr = T.Denoiser(8, 256, 256, training=True)
    tr.set_params(PF.init_params(0))
    xin = torch.stack([d[k, 100:356, 200:456] for k in range(8)]).contiguous()
    tgt = xin.to(torch.float32) / 1000.0
    for _ in range(args.warmup):
        tr.forward(xin)
        tr.backward(tgt)
        tr.adam_step()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        tr.forward(xin)
        tr.backward(tgt)
        tr.adam_step()
    e1.record()
    torch.cuda.synchronize()
    ms_tr = e0.elapsed_time(e1) / args.steps
    f_inf = prefilter_flop(480, 640, 1)
    f_tr = 3.0 * prefilter_flop(256, 256, 8)     # forward + backward-data + weight gradient
    tf_inf = f_inf / (ms_inf * 1e-3) / 1e12
    out = {
        "metric": "prefilter inference ms per 640x480 frame (bf16 matrix cores)", "value": round(ms_inf, 4),
        "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": False,
        "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "learned prefilter kernels: 640x480 inference; training steps at batch 8 of 256x256"},
        "roofline": {"bound": "mfma", "achieved": round(tf_inf, 2), "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(tf_inf / MFMA_BF16_PEAK_TFLOPS, 5), "traffic": None,
                     "kernel": "whole forward pass", "flop_per_launch": int(f_inf)},
        "extra": {"train_step_ms": round(ms_tr, 4), "train_tflops": round(f_tr / (ms_tr * 1e-3) / 1e12, 2),
                  "train_flop_per_step": int(f_tr)},
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=270)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c5", action="store_true", help="c2: skip the equal-error (prefilter) half")
    ap.add_argument("--workers", type=int, default=min(16, cpu_cores()))
    ap.add_argument("--frames-cache", default=None,
                    help="npy file holding the generated depth frames (written if absent)")
    ap.add_argument("--c4-tile", default="", help="c4: fixed raycast tile shape WxH instead of autotuning")
    ap.add_argument("--workload", choices=("c2", "c3", "c4", "c5", "prefilter", "track", "filter", "mesh", "surfel"), default="c2",
                    help="c2: one volume, the headline metric; c3: the large walk with host swapping; "
                         "c4: 64 batched submaps, 8 views; "
                         "c5: train the depth prefilter, then denoised vs plain at equal surface error")
    ap.add_argument("--c5-rooms", type=int, default=50, help="training rooms (seeds 5000..)")
    ap.add_argument("--c5-frames", type=int, default=100, help="training frames per room")
    ap.add_argument("--c5-steps", type=int, default=1500, help="Adam steps (batch 8 of 256x256 crops)")
    ap.add_argument("--c5-eval-rooms", type=int, default=10, help="held-out rooms (seeds 6000..)")
    ap.add_argument("--c5-eval-frames", type=int, default=300)
    ap.add_argument("--c5-lr", type=float, default=2e-4)
    ap.add_argument("--c5-save", default=None, help="write the trained parameters (npy) here")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 256 MiB device copy (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        n = 256 << 20
        src = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n, "copies": 5}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "layout of the path is described in the design notes but not run.", file=sys.stderr)
        sys.exit(2)

    if args.workload == "c3":
        return run_c3(args)
    if args.workload == "c4":
        return run_c4(args)
    if args.workload == "c5":
        return run_c5(args)
    if args.workload == "prefilter":
        return run_prefilter(args)
    if args.workload == "track":
        return run_track(args)
    if args.workload == "filter":
        return run_filter(args)
    if args.workload == "mesh":
        return run_mesh(args)
    if args.workload == "surfel":
        return run_surfel(args)
    line = run_c2(args)
    if not args.no_c5:
        print("[bench] equal-error half: training and evaluating the prefilter", file=sys.stderr, flush=True)
        line["extra"]["c5"] = c5_summary(args)
    print(json.dumps(line), flush=True)


def c2_schedule(warmup, steps, n_traj=N_TRAJ):
    """trajectory frame index of every fused frame: an untimed prefix so that
    the timed frames are the trajectory's last `steps` (the map at its
    configured size), then `warmup`, then the timed frames; with more than
    n_traj frames in all, indices wrap (the pose jumps back to the start)"""
    prefill = max(0, n_traj - warmup - steps)
    order = [i % n_traj for i in range(prefill + warmup + steps)]
    return prefill, order


def run_c2(args):
    from synth import configs
    K = configs.KINECT_INTR
    prefill, order = c2_schedule(args.warmup, args.steps)
    print(f"[bench] generating {N_TRAJ} frames", file=sys.stderr, flush=True)
    frames = make_frames(N_TRAJ, args.workers, args.frames_cache)
    poses = np.stack(configs.c2_poses(N_TRAJ)).astype(np.float32)

    import torch
    import paper_1708_00783_amd as T
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    d_frames = torch.from_numpy(frames).cuda()
    vol = T.Volume(configs.C2_VOLUME, K.width, K.height)
    pts = torch.empty((K.height, K.width, 4), dtype=torch.float32, device="cuda")
    nrm = torch.empty_like(pts)

    def step(i):
        f = order[i]
        vol.frame(d_frames[f], K, poses[f], pts, nrm, stream)

    for i in range(prefill + args.warmup):
        step(i)
    torch.cuda.synchronize()
    s0 = vol.stats()
    # kernel durations: HIP events around the integration and raycast launches
    # of every PROFILE_EVERY-th frame of the timed region (each timed launch
    # costs two event records on the stream; sampling keeps that out of the
    # frame rate)
    vol.profile_enable(True)
    vol.profile_select(("integrate", "raycast"), PROFILE_EVERY)
    vol.profile_read(reset=True)
    t_first, t_last = order[prefill + args.warmup], order[-1]
    print(f"[bench] prefix {prefill} + warm-up {args.warmup} frames fused, timing {args.steps} "
          f"(trajectory frames {t_first}..{t_last})", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(prefill + args.warmup, len(order)):
        step(i)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = vol.profile_read()
    vol.profile_enable(False)
    s1 = vol.stats()
    assert s1["flags"] == 0, f"capacity flags raised: {s1['flags']:#x}"

    steps = args.steps
    fps = steps / dt
    d_blocks = s1["total_integrated_blocks"] - s0["total_integrated_blocks"]
    d_cols = s1["total_written_columns"] - s0["total_written_columns"]
    d_rec = s1["total_range_records"] - s0["total_range_records"]
    d_hits = s1["total_rays_hit"] - s0["total_rays_hit"]
    WH = K.width * K.height
    # algorithmic bytes per launch (see the design notes for the per-unit figures)
    bytes_integrate = (d_blocks * (1536 + 16 + 4) + d_cols * 24) / steps + 4 * WH
    bytes_raycast = (d_rec * (1024 + 16)) / steps + 32 * WH
    kern = {}
    for k, b in (("integrate", bytes_integrate), ("raycast", bytes_raycast)):
        ms = prof[k]["ms"] / max(1, prof[k]["launches"])
        kern[k] = {"avg_ms": ms, "bytes": b, "gbs": b / (ms * 1e-3) / 1e9 if ms > 0 else 0.0}
    total_ms = {k: v["ms"] for k, v in prof.items()}
    dominant = max(("integrate", "raycast"), key=lambda k: total_ms[k])
    rk = kern[dominant]
    timed = (t_first, t_last)
    roofline = {"bound": "hbm", "achieved": round(rk["gbs"], 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(rk["gbs"] / HBM_PEAK_GBS, 5),
                "traffic": measured_traffic("k_" + dominant, timed),
                "kernel": dominant,
                "algorithmic_bytes_per_launch": int(rk["bytes"]),
                "avg_launch_ms": round(rk["avg_ms"], 5)}

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        cpu = cpu_baseline(frames, poses, K)

    return {
        "metric": METRIC, "value": round(fps, 3), "unit": "frames/s", "n_gpus": 1,
        "steps": steps, "warmup": args.warmup, "ms_per_step": round(1e3 * dt / steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "full frame: 640x480 uint16 depth, 4x4x3 m room with 20 primitives, "
                               "Kinect-like noise, voxel 5 mm, mu 2 cm, 2^20 buckets + 2^17 excess, "
                               "2^18 blocks; alloc+integrate+raycast per frame",
                   "trajectory_frames": N_TRAJ, "frames_fused": len(order), "prefill_frames": prefill,
                   "warmup_frames": args.warmup, "timed_frames": [t_first, t_last],
                   "width": K.width, "height": K.height},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": {
            # voxel visits per second of integration-kernel time
            "voxel_updates_per_s": (d_blocks * 512) / (kern["integrate"]["avg_ms"] * 1e-3 * steps)
            if kern["integrate"]["avg_ms"] > 0 else None,
            "voxel_updates_per_s_wall": (d_blocks * 512) / dt,
            "avg_visible_blocks": d_blocks / steps,
            "avg_range_records": d_rec / steps,
            "hit_fraction": d_hits / (steps * WH),
            "kernel_ms_per_launch": {k: round(v["ms"] / v["launches"], 5) for k, v in prof.items() if v["launches"]},
            "profiled_frames": f"every {PROFILE_EVERY}th frame of the timed region",
            "kernel_gbs": {k: round(v["gbs"], 1) for k, v in kern.items()},
            "allocated_blocks": s1["n_allocated"],
        },
    }


if __name__ == "__main__":
    main()
