"""Python binding of libtsdf.so (the gfx950 TSDF fusion hot path).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  PyTorch supplies device memory (tensors) and streams.  The module
refuses to load without the built library: there is no fallback path.

The functions keep the C names of include/tsdf.h; `Volume` wraps one context
and its workspace tensor.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libtsdf.so")

TF_OK, TF_E_INVAL, TF_E_HIP, TF_E_ORDER, TF_E_SPACE, TF_E_IO = 0, -1, -2, -3, -4, -5
TF_DEPTH_F32_M, TF_DEPTH_U16_MM = 0, 1
TF_FLAG_BLOCKS_EXHAUSTED = 0x1
TF_FLAG_EXCESS_EXHAUSTED = 0x2
TF_FLAG_REQUEST_OVERFLOW = 0x4
TF_FLAG_TRANSFER_OVERFLOW = 0x8
TF_FLAG_BIN_OVERFLOW = 0x10

# every symbol include/tsdf.h declares
EXPORTS = (
    "tf_workspace_bytes", "tf_host_store_bytes", "tf_host_transfer_bytes", "tf_create",
    "tf_destroy", "tf_reset", "tf_alloc_and_visible", "tf_integrate", "tf_raycast",
    "tf_range_image", "tf_swap_out", "tf_get_stats", "tf_export_entries", "tf_export_visible",
    "tf_export_voxels", "tf_status_string", "tf_profile_enable", "tf_profile_read",
    "tf_export_host_voxels", "tf_profile_select", "tf_save", "tf_load", "tf_camera_depth",
    "tf_multi_workspace_bytes", "tf_multi_host_bytes", "tf_multi_create", "tf_multi_destroy",
    "tf_multi_submap", "tf_multi_set_config", "tf_multi_get_config", "tf_multi_integrate",
    "tf_multi_raycast", "tf_multi_frame", "tf_multi_range_image", "tf_multi_autotune",
    "tf_multi_get_stats",
    # include/tsdf_nn.h
    "tf_nn_param_count", "tf_nn_workspace_bytes", "tf_nn_create", "tf_nn_destroy", "tf_nn_set_params",
    "tf_nn_get_params", "tf_nn_forward", "tf_nn_backward", "tf_nn_adam_step", "tf_nn_tensor",
    # include/tsdf_track.h
    "tf_track_workspace_bytes", "tf_track", "tf_track_noalloc",
    # include/tsdf_filter.h
    "tf_bilateral",
    # include/tsdf_mesh.h
    "tf_mesh_workspace_bytes", "tf_mesh",
    # include/tsdf_surfel.h
    "tf_surfel_workspace_bytes", "tf_surfel_create", "tf_surfel_destroy", "tf_surfel_reset", "tf_surfel_fuse",
    "tf_surfel_stats", "tf_surfel_export", "tf_surfel_export_frame",
)


class tf_intrinsics(ctypes.Structure):
    _fields_ = [("fx", ctypes.c_float), ("fy", ctypes.c_float), ("cx", ctypes.c_float),
                ("cy", ctypes.c_float), ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


class tf_params(ctypes.Structure):
    _fields_ = [("voxel_size", ctypes.c_float), ("mu", ctypes.c_float), ("max_w", ctypes.c_int32),
                ("n_buckets", ctypes.c_uint32), ("n_excess", ctypes.c_uint32),
                ("n_blocks", ctypes.c_uint32), ("max_width", ctypes.c_uint32),
                ("max_height", ctypes.c_uint32), ("swap_transfer_blocks", ctypes.c_uint32)]


class tf_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint32) for n in (
        "flags", "n_allocated", "n_visible", "n_new", "n_free_excess", "n_swapped_in",
        "n_swapped_out", "frames")] + [(n, ctypes.c_uint64) for n in (
        "total_integrated_blocks", "total_written_columns", "total_range_records",
        "total_rays_hit", "total_requests", "total_new_blocks", "integrate_calls",
        "raycast_calls")]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


KERNEL_CLASSES = ("alloc_rays", "insert", "visible", "integrate", "range_bin", "raycast", "swap")


class tf_profile(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_uint64 * 8), ("ms", ctypes.c_double * 8)]

    def as_dict(self):
        return {k: {"launches": int(self.launches[i]), "ms": float(self.ms[i])}
                for i, k in enumerate(KERNEL_CLASSES)}


class tf_view(ctypes.Structure):
    _fields_ = [("intr", tf_intrinsics), ("pose_w2c", ctypes.c_float * 16),
                ("d_points", ctypes.c_void_p), ("d_normals", ctypes.c_void_p)]


class tf_multi_config(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in (
        "tile_w", "tile_h", "integrate_threads", "integrate_groups", "bin_groups")]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


class tf_multi_stats(ctypes.Structure):
    _fields_ = [("flags", ctypes.c_uint32), ("n_submaps", ctypes.c_uint32)] + [(n, ctypes.c_uint64) for n in (
        "allocated_blocks", "total_integrated_blocks", "total_written_columns", "total_bin_entries",
        "total_block_views", "total_rays_hit", "raycast_calls")]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


class tf_track_params(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int32), ("iterations", ctypes.c_int32 * 4),
                ("dist_thresh", ctypes.c_float * 4), ("min_update", ctypes.c_float)]


class tf_track_result(ctypes.Structure):
    _fields_ = [("pose_w2c", ctypes.c_float * 16), ("iterations", ctypes.c_int32 * 4), ("pairs", ctypes.c_int32 * 4),
                ("status", ctypes.c_int32), ("pad", ctypes.c_int32), ("sums", (ctypes.c_double * 28) * 4)]


class tf_bilateral_params(ctypes.Structure):
    _fields_ = [("radius", ctypes.c_int32), ("sigma_space", ctypes.c_float), ("sigma_range", ctypes.c_float)]


class tf_surfel_params(ctypes.Structure):
    _fields_ = [("capacity", ctypes.c_uint32), ("max_width", ctypes.c_int32), ("max_height", ctypes.c_int32),
                ("sigma", ctypes.c_float), ("max_depth_diff", ctypes.c_float), ("min_normal_dot", ctypes.c_float)]


class TsdfError(RuntimeError):
    pass


_lib = None
_VP = ctypes.c_void_p
_F16 = ctypes.POINTER(ctypes.c_float)


def lib():
    """Load libtsdf.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        sig = {
            "tf_workspace_bytes": (ctypes.c_size_t, [P(tf_params)]),
            "tf_host_store_bytes": (ctypes.c_size_t, [P(tf_params)]),
            "tf_host_transfer_bytes": (ctypes.c_size_t, [P(tf_params)]),
            "tf_create": (ctypes.c_int, [P(tf_params), _VP, ctypes.c_size_t, _VP, _VP, _VP, P(_VP)]),
            "tf_destroy": (ctypes.c_int, [_VP]),
            "tf_reset": (ctypes.c_int, [_VP, _VP]),
            "tf_alloc_and_visible": (ctypes.c_int, [_VP, _VP, ctypes.c_int, P(tf_intrinsics), _F16, _VP]),
            "tf_integrate": (ctypes.c_int, [_VP, _VP, ctypes.c_int, _F16, _VP]),
            "tf_raycast": (ctypes.c_int, [_VP, _F16, P(tf_intrinsics), _VP, _VP, _VP]),
            "tf_range_image": (ctypes.c_int, [_VP, _F16, P(tf_intrinsics), _VP, _VP, _VP]),
            "tf_swap_out": (ctypes.c_int, [_VP, _VP]),
            "tf_get_stats": (ctypes.c_int, [_VP, P(tf_stats), _VP]),
            "tf_export_entries": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP]),
            "tf_export_visible": (ctypes.c_int, [_VP, _VP, ctypes.c_uint32, P(ctypes.c_uint32), _VP]),
            "tf_export_voxels": (ctypes.c_int, [_VP, _VP, ctypes.c_uint32, _VP, _VP, _VP]),
            "tf_status_string": (ctypes.c_char_p, [ctypes.c_int]),
            "tf_profile_enable": (ctypes.c_int, [_VP, ctypes.c_int]),
            "tf_profile_read": (ctypes.c_int, [_VP, P(tf_profile), ctypes.c_int]),
            "tf_profile_select": (ctypes.c_int, [_VP, ctypes.c_uint32, ctypes.c_uint32]),
            "tf_export_host_voxels": (ctypes.c_int, [_VP, _VP, ctypes.c_uint32, _VP, _VP, _VP]),
            "tf_save": (ctypes.c_int, [_VP, ctypes.c_char_p, _VP]),
            "tf_load": (ctypes.c_int, [_VP, ctypes.c_char_p, _VP]),
            "tf_camera_depth": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int32, _F16, _VP, _VP]),
            "tf_multi_workspace_bytes": (ctypes.c_size_t, [P(tf_params), ctypes.c_uint32, ctypes.c_uint32,
                                                           ctypes.c_uint32, ctypes.c_uint32]),
            "tf_multi_host_bytes": (ctypes.c_size_t, []),
            "tf_multi_create": (ctypes.c_int, [P(tf_params), ctypes.c_uint32, _F16, ctypes.c_uint32,
                                               ctypes.c_uint32, ctypes.c_uint32, _VP, ctypes.c_size_t, _VP,
                                               ctypes.c_size_t, _VP, P(_VP)]),
            "tf_multi_destroy": (ctypes.c_int, [_VP]),
            "tf_multi_submap": (ctypes.c_int, [_VP, ctypes.c_uint32, P(_VP)]),
            "tf_multi_set_config": (ctypes.c_int, [_VP, P(tf_multi_config)]),
            "tf_multi_get_config": (ctypes.c_int, [_VP, P(tf_multi_config)]),
            "tf_multi_integrate": (ctypes.c_int, [_VP, _VP, ctypes.c_int, P(tf_intrinsics), _F16,
                                                  P(ctypes.c_uint32), ctypes.c_uint32, _VP]),
            "tf_multi_raycast": (ctypes.c_int, [_VP, P(tf_view), ctypes.c_uint32, _VP]),
            "tf_multi_frame": (ctypes.c_int, [_VP, _VP, ctypes.c_int, P(tf_intrinsics), _F16,
                                              P(ctypes.c_uint32), ctypes.c_uint32, P(tf_view), ctypes.c_uint32,
                                              ctypes.c_int, _VP]),
            "tf_multi_range_image": (ctypes.c_int, [_VP, P(tf_view), _VP, _VP, _VP]),
            "tf_multi_autotune": (ctypes.c_int, [_VP, _VP, ctypes.c_int, P(tf_intrinsics), _F16,
                                                 P(ctypes.c_uint32), ctypes.c_uint32, P(tf_view), ctypes.c_uint32,
                                                 ctypes.c_int, P(tf_multi_config), P(ctypes.c_float), _VP]),
            "tf_multi_get_stats": (ctypes.c_int, [_VP, P(tf_multi_stats), _VP]),
            "tf_nn_param_count": (ctypes.c_uint32, []),
            "tf_nn_workspace_bytes": (ctypes.c_size_t, [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                                        ctypes.c_int]),
            "tf_nn_create": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int, _VP,
                                            ctypes.c_size_t, P(_VP)]),
            "tf_nn_destroy": (ctypes.c_int, [_VP]),
            "tf_nn_set_params": (ctypes.c_int, [_VP, _VP, _VP]),
            "tf_nn_get_params": (ctypes.c_int, [_VP, _VP, _VP]),
            "tf_nn_forward": (ctypes.c_int, [_VP, _VP, ctypes.c_int, ctypes.c_uint32, _VP, _VP]),
            "tf_nn_backward": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
            "tf_nn_adam_step": (ctypes.c_int, [_VP, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                               ctypes.c_float, _VP]),
            "tf_nn_tensor": (ctypes.c_int, [_VP, ctypes.c_int, P(_VP), P(ctypes.c_int32)]),
            "tf_track_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
            "tf_track": (ctypes.c_int, [_VP, ctypes.c_int, P(tf_intrinsics), _VP, _VP, P(tf_intrinsics), _F16, _F16,
                                        P(tf_track_params), _VP, ctypes.c_size_t, _VP, _VP]),
            "tf_surfel_workspace_bytes": (ctypes.c_size_t, [P(tf_surfel_params)]),
            "tf_surfel_create": (ctypes.c_int, [P(tf_surfel_params), _VP, ctypes.c_size_t, _VP, P(_VP)]),
            "tf_surfel_destroy": (ctypes.c_int, [_VP]),
            "tf_surfel_reset": (ctypes.c_int, [_VP, _VP]),
            "tf_surfel_fuse": (ctypes.c_int, [_VP, _VP, ctypes.c_int, P(tf_intrinsics), _F16, _VP]),
            "tf_surfel_stats": (ctypes.c_int, [_VP, P(ctypes.c_uint32), P(ctypes.c_uint32), P(ctypes.c_uint32), _VP]),
            "tf_surfel_export": (ctypes.c_int, [_VP, ctypes.c_uint32, _VP, _VP, _VP, _VP]),
            "tf_surfel_export_frame": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
            "tf_mesh_workspace_bytes": (ctypes.c_size_t, [P(tf_params)]),
            "tf_mesh": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_uint64, _VP, _VP, ctypes.c_size_t, _VP]),
            "tf_bilateral": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int32, ctypes.c_int32,
                                            P(tf_bilateral_params), _VP, _VP]),
            "tf_track_noalloc": (ctypes.c_int, [_VP, ctypes.c_int, P(tf_intrinsics), _VP, _VP, P(tf_intrinsics),
                                                _F16, _F16, P(tf_track_params), _VP, _VP]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int, what: str = "") -> None:
    if status != TF_OK:
        msg = lib().tf_status_string(status).decode()
        raise TsdfError(f"{what}: {msg} ({status})")


def _pose_arg(pose):
    M = np.ascontiguousarray(np.asarray(pose, np.float32).reshape(16))
    return M, M.ctypes.data_as(_F16)


def make_intrinsics(intr) -> tf_intrinsics:
    """From synth.Intrinsics, a dict, or (fx, fy, cx, cy, W, H)."""
    if hasattr(intr, "fx"):
        return tf_intrinsics(intr.fx, intr.fy, intr.cx, intr.cy, intr.width, intr.height)
    fx, fy, cx, cy, W, H = intr
    return tf_intrinsics(fx, fy, cx, cy, int(W), int(H))


def make_params(vp, max_width, max_height, swap_transfer_blocks=0) -> tf_params:
    return tf_params(vp.voxel_size, vp.mu, vp.max_w, vp.n_buckets, vp.n_excess, vp.n_blocks,
                     max_width, max_height, swap_transfer_blocks)


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


# ---- C-named thin wrappers ---------------------------------------------------------

def tf_workspace_bytes(params: tf_params) -> int:
    return int(lib().tf_workspace_bytes(ctypes.byref(params)))


def tf_create(params, d_workspace_ptr, nbytes, h_store=None, h_transfer=None, stream=None):
    ctx = _VP()
    check(lib().tf_create(ctypes.byref(params), ctypes.c_void_p(d_workspace_ptr), nbytes,
                          h_store, h_transfer, _stream_ptr(stream), ctypes.byref(ctx)), "tf_create")
    return ctx


def tf_alloc_and_visible(ctx, depth, depth_format, intr, pose, stream=None):
    _, Mp = _pose_arg(pose)
    K = make_intrinsics(intr)
    check(lib().tf_alloc_and_visible(ctx, ctypes.c_void_p(depth.data_ptr()), depth_format,
                                     ctypes.byref(K), Mp, _stream_ptr(stream)), "tf_alloc_and_visible")


def tf_integrate(ctx, depth, depth_format, pose, stream=None):
    _, Mp = _pose_arg(pose)
    check(lib().tf_integrate(ctx, ctypes.c_void_p(depth.data_ptr()), depth_format, Mp,
                             _stream_ptr(stream)), "tf_integrate")


def tf_raycast(ctx, pose, intr, points, normals, stream=None):
    _, Mp = _pose_arg(pose)
    K = make_intrinsics(intr)
    check(lib().tf_raycast(ctx, Mp, ctypes.byref(K), ctypes.c_void_p(points.data_ptr()),
                           ctypes.c_void_p(normals.data_ptr()), _stream_ptr(stream)), "tf_raycast")


def tf_range_image(ctx, pose, intr, zmin, zmax, stream=None):
    _, Mp = _pose_arg(pose)
    K = make_intrinsics(intr)
    check(lib().tf_range_image(ctx, Mp, ctypes.byref(K), ctypes.c_void_p(zmin.data_ptr()),
                               ctypes.c_void_p(zmax.data_ptr()), _stream_ptr(stream)), "tf_range_image")


def tf_camera_depth(points, pose, depth, stream=None):
    """camera z of raycast hit points (H, W, 4) under pose into depth (H, W); 0 on a miss"""
    _, Mp = _pose_arg(pose)
    H, W = int(points.shape[0]), int(points.shape[1])
    check(lib().tf_camera_depth(ctypes.c_void_p(points.data_ptr()), W, H, Mp, ctypes.c_void_p(depth.data_ptr()),
                                _stream_ptr(stream)), "tf_camera_depth")


def tf_get_stats(ctx, stream=None) -> dict:
    st = tf_stats()
    check(lib().tf_get_stats(ctx, ctypes.byref(st), _stream_ptr(stream)), "tf_get_stats")
    return st.as_dict()


class Volume:
    """One TSDF volume on the current HIP device."""

    def __init__(self, vp, max_width, max_height, swap_transfer_blocks=0, stream=None):
        import torch
        self.params = make_params(vp, max_width, max_height, swap_transfer_blocks)
        nbytes = tf_workspace_bytes(self.params)
        if nbytes == 0:
            raise TsdfError("invalid volume parameters")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.h_store = None
        self.h_transfer = None
        hs = ht = None
        if swap_transfer_blocks:
            n_store = int(lib().tf_host_store_bytes(ctypes.byref(self.params)))
            n_xfer = int(lib().tf_host_transfer_bytes(ctypes.byref(self.params)))
            self.h_store = np.empty(n_store, np.uint8)
            # touch every page now: a swap-out writes blocks at entry-indexed,
            # scattered places, and first-touch page faults would land there
            self.h_store[::4096] = 0
            self.h_transfer = torch.empty(n_xfer, dtype=torch.uint8, pin_memory=True)
            hs = ctypes.c_void_p(self.h_store.ctypes.data)
            ht = ctypes.c_void_p(self.h_transfer.data_ptr())
        self.ctx = tf_create(self.params, self.workspace.data_ptr(), nbytes, hs, ht, stream)
        self.n_entries = self.params.n_buckets + self.params.n_excess

    @classmethod
    def borrowed(cls, ctx, params, owner):
        """A view of a context the library owns (a submap of a MultiMap)."""
        v = cls.__new__(cls)
        v.params = params
        v.workspace = None
        v.h_store = v.h_transfer = None
        v.ctx = ctx
        v.n_entries = params.n_buckets + params.n_excess
        v._owner = owner
        v._borrowed = True
        return v

    def close(self):
        if getattr(self, "_borrowed", False):
            self.ctx = None
            return
        if getattr(self, "ctx", None):
            lib().tf_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reset(self, stream=None):
        check(lib().tf_reset(self.ctx, _stream_ptr(stream)), "tf_reset")

    def alloc_and_visible(self, depth, intr, pose, stream=None):
        fmt = TF_DEPTH_U16_MM if depth.dtype.itemsize == 2 else TF_DEPTH_F32_M
        tf_alloc_and_visible(self.ctx, depth, fmt, intr, pose, stream)

    def integrate(self, depth, pose, stream=None):
        fmt = TF_DEPTH_U16_MM if depth.dtype.itemsize == 2 else TF_DEPTH_F32_M
        tf_integrate(self.ctx, depth, fmt, pose, stream)

    def raycast(self, pose, intr, points=None, normals=None, stream=None):
        import torch
        K = make_intrinsics(intr)
        if points is None:
            points = torch.empty((K.height, K.width, 4), dtype=torch.float32, device="cuda")
        if normals is None:
            normals = torch.empty((K.height, K.width, 4), dtype=torch.float32, device="cuda")
        tf_raycast(self.ctx, pose, K, points, normals, stream)
        return points, normals

    def range_image(self, pose, intr, stream=None):
        import torch
        K = make_intrinsics(intr)
        zmin = torch.empty((K.height, K.width), dtype=torch.float32, device="cuda")
        zmax = torch.empty((K.height, K.width), dtype=torch.float32, device="cuda")
        tf_range_image(self.ctx, pose, K, zmin, zmax, stream)
        return zmin, zmax

    def swap_out(self, stream=None):
        check(lib().tf_swap_out(self.ctx, _stream_ptr(stream)), "tf_swap_out")

    def stats(self, stream=None) -> dict:
        return tf_get_stats(self.ctx, stream)

    def save(self, path, stream=None):
        """write the whole volume to `path` (synchronising)"""
        check(lib().tf_save(self.ctx, os.fsencode(path), _stream_ptr(stream)), "tf_save")

    def load(self, path, stream=None):
        """replace the volume by the one saved at `path` (same parameters; synchronising)"""
        check(lib().tf_load(self.ctx, os.fsencode(path), _stream_ptr(stream)), "tf_load")

    def profile_enable(self, on=True):
        check(lib().tf_profile_enable(self.ctx, 1 if on else 0), "tf_profile_enable")

    def profile_select(self, classes=None, every=1):
        """time only the named kernel classes (None = all), every n-th launch"""
        mask = 0xffffffff if classes is None else sum(1 << KERNEL_CLASSES.index(c) for c in classes)
        check(lib().tf_profile_select(self.ctx, mask, every), "tf_profile_select")

    def profile_read(self, reset=False) -> dict:
        pr = tf_profile()
        check(lib().tf_profile_read(self.ctx, ctypes.byref(pr), 1 if reset else 0), "tf_profile_read")
        return pr.as_dict()

    def frame(self, depth, intr, pose, points=None, normals=None, stream=None):
        self.alloc_and_visible(depth, intr, pose, stream)
        self.integrate(depth, pose, stream)
        return self.raycast(pose, intr, points, normals, stream)

    # ---- inspection (synchronising) ------------------------------------------------
    def entries(self, stream=None):
        n = self.n_entries
        pos = np.empty((n, 3), np.int16)
        off = np.empty(n, np.int32)
        ptr = np.empty(n, np.int32)
        check(lib().tf_export_entries(self.ctx, pos.ctypes.data_as(_VP), off.ctypes.data_as(_VP),
                                      ptr.ctypes.data_as(_VP), _stream_ptr(stream)), "tf_export_entries")
        return pos, off, ptr

    def visible(self, stream=None) -> np.ndarray:
        cnt = ctypes.c_uint32(0)
        buf = np.empty(self.params.n_blocks, np.int32)
        check(lib().tf_export_visible(self.ctx, buf.ctypes.data_as(_VP), buf.size, ctypes.byref(cnt),
                                      _stream_ptr(stream)), "tf_export_visible")
        return buf[:cnt.value].copy()

    def block_voxels(self, entry_ids, stream=None):
        import torch
        ids = torch.as_tensor(np.ascontiguousarray(entry_ids, np.int32)).cuda()
        n = ids.numel()
        sdf = torch.empty((n, 512), dtype=torch.int16, device="cuda")
        w = torch.empty((n, 512), dtype=torch.uint8, device="cuda")
        if n:
            check(lib().tf_export_voxels(self.ctx, ctypes.c_void_p(ids.data_ptr()), n,
                                         ctypes.c_void_p(sdf.data_ptr()), ctypes.c_void_p(w.data_ptr()),
                                         _stream_ptr(stream)), "tf_export_voxels")
        return sdf.cpu().numpy(), w.cpu().numpy()

    def host_voxels(self, entry_ids):
        """(sdf, w, has) of host-store blocks (swapping volumes only)"""
        ids = np.ascontiguousarray(entry_ids, np.int32)
        sdf = np.empty((ids.size, 512), np.int16)
        w = np.empty((ids.size, 512), np.uint8)
        has = np.empty(ids.size, np.uint8)
        check(lib().tf_export_host_voxels(self.ctx, ids.ctypes.data_as(_VP), ids.size, sdf.ctypes.data_as(_VP),
                                          w.ctypes.data_as(_VP), has.ctypes.data_as(_VP)), "tf_export_host_voxels")
        return sdf, w, has.astype(bool)

    def allocated_positions(self) -> np.ndarray:
        pos, _, ptr = self.entries()
        p = pos[ptr >= 0].astype(np.int32)
        return p[np.lexsort((p[:, 2], p[:, 1], p[:, 0]))] if len(p) else p.reshape(0, 3)

    def mesh(self, stream=None):
        """marching-cubes mesh: (vertices (m, 3, 3) float32 world metres, edge
        keys (m, 3) int64) on the host"""
        import torch
        nbytes = int(lib().tf_mesh_workspace_bytes(ctypes.byref(self.params)))
        ws = torch.empty(max(8, nbytes), dtype=torch.uint8, device="cuda")
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        check(lib().tf_mesh(self.ctx, None, None, 0, ctypes.c_void_p(cnt.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                            nbytes, _stream_ptr(stream)), "tf_mesh")
        n = int(cnt.item())
        verts = torch.empty((max(1, n), 3, 3), dtype=torch.float32, device="cuda")
        keys = torch.empty((max(1, n), 3), dtype=torch.int64, device="cuda")
        check(lib().tf_mesh(self.ctx, ctypes.c_void_p(verts.data_ptr()), ctypes.c_void_p(keys.data_ptr()), n,
                            ctypes.c_void_p(cnt.data_ptr()), ctypes.c_void_p(ws.data_ptr()), nbytes,
                            _stream_ptr(stream)), "tf_mesh")
        return verts[:n].cpu().numpy(), keys[:n].cpu().numpy()

    def voxels_by_position(self):
        pos, _, ptr = self.entries()
        ids = np.flatnonzero(ptr >= 0).astype(np.int32)
        p = pos[ids].astype(np.int32)
        order = np.lexsort((p[:, 2], p[:, 1], p[:, 0]))
        ids = ids[order]
        sdf, w = self.block_voxels(ids)
        return p[order], sdf, w


# ---- rigid submaps, batched ------------------------------------------------------

def make_view(intr, pose, points, normals) -> tf_view:
    v = tf_view()
    v.intr = make_intrinsics(intr)
    M = np.ascontiguousarray(np.asarray(pose, np.float32).reshape(16))
    for i in range(16):
        v.pose_w2c[i] = float(M[i])
    v.d_points = points.data_ptr()
    v.d_normals = normals.data_ptr()
    return v


def _sel_arg(sel):
    a = (ctypes.c_uint32 * len(sel))(*[int(x) for x in sel])
    return a, len(sel)


class MultiMap:
    """Batched rigid submaps (Sec. 7.2) on the current HIP device: n volumes of
    parameters vp with poses P_i (world -> submap, n x 4 x 4)."""

    def __init__(self, vp, poses, frame_w, frame_h, view_w, view_h, bin_capacity, stream=None):
        import torch
        self.params = make_params(vp, frame_w, frame_h, 0)
        self.poses = np.ascontiguousarray(np.asarray(poses, np.float32).reshape(-1, 16))
        self.n = self.poses.shape[0]
        nbytes = int(lib().tf_multi_workspace_bytes(ctypes.byref(self.params), self.n, view_w, view_h,
                                                    bin_capacity))
        if nbytes == 0:
            raise TsdfError("invalid batched-map parameters")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        hb = int(lib().tf_multi_host_bytes())
        self.h_params = torch.empty(hb, dtype=torch.uint8, pin_memory=True)
        h = _VP()
        check(lib().tf_multi_create(ctypes.byref(self.params), self.n, self.poses.ctypes.data_as(_F16), view_w,
                                    view_h, bin_capacity, ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                                    ctypes.c_void_p(self.h_params.data_ptr()), hb, _stream_ptr(stream),
                                    ctypes.byref(h)), "tf_multi_create")
        self.h = h
        self._subs = {}

    def close(self):
        if getattr(self, "h", None):
            lib().tf_multi_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submap(self, i) -> Volume:
        if i not in self._subs:
            c = _VP()
            check(lib().tf_multi_submap(self.h, i, ctypes.byref(c)), "tf_multi_submap")
            self._subs[i] = Volume.borrowed(c, self.params, self)
        return self._subs[i]

    def set_config(self, **kw):
        c = self.get_config()
        for k, v in kw.items():
            setattr(c, k, int(v))
        check(lib().tf_multi_set_config(self.h, ctypes.byref(c)), "tf_multi_set_config")

    def get_config(self) -> tf_multi_config:
        c = tf_multi_config()
        check(lib().tf_multi_get_config(self.h, ctypes.byref(c)), "tf_multi_get_config")
        return c

    def integrate(self, depth, intr, pose, sel, stream=None):
        fmt = TF_DEPTH_U16_MM if depth.dtype.itemsize == 2 else TF_DEPTH_F32_M
        _, Mp = _pose_arg(pose)
        K = make_intrinsics(intr)
        a, n = _sel_arg(sel)
        check(lib().tf_multi_integrate(self.h, ctypes.c_void_p(depth.data_ptr()), fmt, ctypes.byref(K), Mp, a, n,
                                       _stream_ptr(stream)), "tf_multi_integrate")

    @staticmethod
    def _views(views):
        arr = (tf_view * len(views))(*[make_view(*v) for v in views])
        return arr, len(views)

    def raycast(self, views, stream=None):
        """views: list of (intr, pose, points, normals)"""
        arr, n = self._views(views)
        check(lib().tf_multi_raycast(self.h, arr, n, _stream_ptr(stream)), "tf_multi_raycast")

    def frame(self, depth, intr, pose, sel, views, use_graph=True, stream=None):
        fmt = TF_DEPTH_U16_MM if depth.dtype.itemsize == 2 else TF_DEPTH_F32_M
        _, Mp = _pose_arg(pose)
        K = make_intrinsics(intr)
        a, ns = _sel_arg(sel)
        arr, nv = self._views(views)
        check(lib().tf_multi_frame(self.h, ctypes.c_void_p(depth.data_ptr()), fmt, ctypes.byref(K), Mp, a, ns,
                                   arr, nv, 1 if use_graph else 0, _stream_ptr(stream)), "tf_multi_frame")

    def range_image(self, intr, pose, stream=None):
        import torch
        K = make_intrinsics(intr)
        zmin = torch.empty((K.height, K.width), dtype=torch.float32, device="cuda")
        zmax = torch.empty((K.height, K.width), dtype=torch.float32, device="cuda")
        dummy = torch.empty(4, dtype=torch.float32, device="cuda")
        v = make_view(intr, pose, dummy, dummy)
        check(lib().tf_multi_range_image(self.h, ctypes.byref(v), ctypes.c_void_p(zmin.data_ptr()),
                                         ctypes.c_void_p(zmax.data_ptr()), _stream_ptr(stream)),
              "tf_multi_range_image")
        return zmin, zmax

    def autotune(self, depth, intr, pose, sel, views, reps=3, stream=None):
        fmt = TF_DEPTH_U16_MM if depth.dtype.itemsize == 2 else TF_DEPTH_F32_M
        _, Mp = _pose_arg(pose)
        K = make_intrinsics(intr)
        a, ns = _sel_arg(sel)
        arr, nv = self._views(views)
        best = tf_multi_config()
        ms = ctypes.c_float(0.0)
        check(lib().tf_multi_autotune(self.h, ctypes.c_void_p(depth.data_ptr()), fmt, ctypes.byref(K), Mp, a, ns,
                                      arr, nv, reps, ctypes.byref(best), ctypes.byref(ms), _stream_ptr(stream)),
              "tf_multi_autotune")
        return best.as_dict(), float(ms.value)

    def stats(self, stream=None) -> dict:
        st = tf_multi_stats()
        check(lib().tf_multi_get_stats(self.h, ctypes.byref(st), _stream_ptr(stream)), "tf_multi_get_stats")
        return st.as_dict()


# ---- learned depth prefilter ------------------------------------------------------

NN_T = dict(input=0, e1=1, e2=2, e3=3, e4=4, d3=5, d2=6, d1=7, grad_e1=8, grad_e2=9, grad_e3=10, grad_e4=11,
            grad_d3=12, grad_d2=13, grad_d1=14, out=15, ddelta=16, depth=17, grads=18, params=19)
NN_LAYERS = (("e1", 3, 32), ("e2", 32, 64), ("e3", 64, 64), ("e4", 64, 128), ("d3", 128, 64), ("d2", 64, 64),
             ("d1", 64, 32), ("head", 32, 1))


def nn_flatten(P: dict) -> np.ndarray:
    """parameter dict {name.w: (cout, 3, 3, cin), name.b: (cout,)} -> fp32 vector"""
    parts = []
    for name, _, _ in NN_LAYERS:
        parts += [np.asarray(P[name + ".w"], np.float32).reshape(-1), np.asarray(P[name + ".b"], np.float32)]
    return np.concatenate(parts)


def nn_unflatten(v) -> dict:
    v = np.asarray(v, np.float32)
    P, o = {}, 0
    for name, cin, cout in NN_LAYERS:
        n = cout * 9 * cin
        P[name + ".w"] = v[o:o + n].reshape(cout, 3, 3, cin)
        o += n
        P[name + ".b"] = v[o:o + cout]
        o += cout
    assert o == v.size
    return P


class Denoiser:
    """The learned depth prefilter on the current HIP device, for batches of
    up to max_batch frames of height x width (multiples of 8)."""

    def __init__(self, max_batch, height, width, training=False):
        import torch
        self.H, self.W, self.B = height, width, max_batch
        nbytes = int(lib().tf_nn_workspace_bytes(max_batch, height, width, 1 if training else 0))
        if nbytes == 0:
            raise TsdfError("invalid denoiser shape")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        h = _VP()
        check(lib().tf_nn_create(max_batch, height, width, 1 if training else 0,
                                 ctypes.c_void_p(self.workspace.data_ptr()), nbytes, ctypes.byref(h)), "tf_nn_create")
        self.h = h
        self.n_params = int(lib().tf_nn_param_count())
        self.loss = torch.zeros(2, dtype=torch.float32, device="cuda")

    def close(self):
        if getattr(self, "h", None):
            lib().tf_nn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params, stream=None):
        import torch
        p = params if isinstance(params, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(params, np.float32))
        p = p.to(device="cuda", dtype=torch.float32).contiguous()
        assert p.numel() == self.n_params
        check(lib().tf_nn_set_params(self.h, ctypes.c_void_p(p.data_ptr()), _stream_ptr(stream)), "tf_nn_set_params")
        self._params_src = p      # the copy is asynchronous: keep the source alive

    def get_params(self, stream=None):
        import torch
        p = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        check(lib().tf_nn_get_params(self.h, ctypes.c_void_p(p.data_ptr()), _stream_ptr(stream)), "tf_nn_get_params")
        return p

    def forward(self, depth, out=None, stream=None):
        """depth: (N, H, W) uint16 mm or float32 m on the device -> float32 m"""
        import torch
        fmt = TF_DEPTH_U16_MM if depth.dtype.itemsize == 2 else TF_DEPTH_F32_M
        n = depth.shape[0] if depth.dim() == 3 else 1
        if out is None:
            out = torch.empty((n, self.H, self.W), dtype=torch.float32, device="cuda")
        check(lib().tf_nn_forward(self.h, ctypes.c_void_p(depth.data_ptr()), fmt, n, ctypes.c_void_p(out.data_ptr()),
                                  _stream_ptr(stream)), "tf_nn_forward")
        return out

    def backward(self, target, stream=None):
        """loss against target (N, H, W) float32 m; returns the (mean, count) device tensor"""
        check(lib().tf_nn_backward(self.h, ctypes.c_void_p(target.data_ptr()), ctypes.c_void_p(self.loss.data_ptr()),
                                   _stream_ptr(stream)), "tf_nn_backward")
        return self.loss

    def adam_step(self, lr=2e-4, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        check(lib().tf_nn_adam_step(self.h, lr, beta1, beta2, eps, _stream_ptr(stream)), "tf_nn_adam_step")

    def tensor(self, name):
        """a view of an internal tensor: bf16 activations/gradients as int16 bit patterns, else float32"""
        import torch
        ptr = _VP()
        dims = (ctypes.c_int32 * 4)()
        check(lib().tf_nn_tensor(self.h, NN_T[name], ctypes.byref(ptr), dims), "tf_nn_tensor")
        off = ptr.value - self.workspace.data_ptr()
        shape = tuple(int(d) for d in dims)
        bf = NN_T[name] <= 14
        n = int(np.prod(shape)) * (2 if bf else 4)
        return self.workspace[off:off + n].view(torch.int16 if bf else torch.float32).reshape(shape)


def bf16_bits_to_float(t):
    """int16 bf16 bit patterns (torch) -> float32 numpy"""
    a = t.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return a.view(np.float32)


# ---- depth tracker -------------------------------------------------------------------

def make_track_params(iterations=(4, 5, 10), dist_thresh=(0.1, 0.2, 0.3), min_update=0.0) -> tf_track_params:
    """per-level iterations and distance thresholds, index 0 = finest"""
    assert len(iterations) == len(dist_thresh) and 1 <= len(iterations) <= 4
    p = tf_track_params()
    p.n_levels = len(iterations)
    for l, (n, d) in enumerate(zip(iterations, dist_thresh)):
        p.iterations[l] = int(n)
        p.dist_thresh[l] = float(d)
    p.min_update = float(min_update)
    return p


def parse_track_result(raw) -> dict:
    """tf_track_result bytes (numpy uint8) -> dict"""
    r = tf_track_result.from_buffer_copy(np.ascontiguousarray(raw, np.uint8).tobytes())
    return {"pose_w2c": np.array(r.pose_w2c, np.float32).reshape(4, 4),
            "iterations": list(r.iterations), "pairs": list(r.pairs), "status": int(r.status),
            "sums": np.array([list(x) for x in r.sums], np.float64)}


class Tracker:
    """The depth tracker for depth images of width x height on the current
    HIP device: owns its workspace and a device result buffer."""

    def __init__(self, width, height, n_levels=3):
        import torch
        nbytes = int(lib().tf_track_workspace_bytes(width, height, n_levels))
        if nbytes == 0:
            raise TsdfError("invalid tracker size")
        self.W, self.H, self.L = width, height, n_levels
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.result = torch.empty(ctypes.sizeof(tf_track_result), dtype=torch.uint8, device="cuda")

    def track_async(self, depth, intr, ref_points, ref_normals, ref_intr, ref_pose, init_pose, params,
                    stream=None):
        """enqueue one tracking call; the result lands in self.result"""
        fmt = TF_DEPTH_U16_MM if depth.dtype.itemsize == 2 else TF_DEPTH_F32_M
        K, Kr = make_intrinsics(intr), make_intrinsics(ref_intr)
        _, Mr = _pose_arg(ref_pose)
        _, Mi = _pose_arg(init_pose)
        check(lib().tf_track(ctypes.c_void_p(depth.data_ptr()), fmt, ctypes.byref(K),
                             ctypes.c_void_p(ref_points.data_ptr()), ctypes.c_void_p(ref_normals.data_ptr()),
                             ctypes.byref(Kr), Mr, Mi, ctypes.byref(params),
                             ctypes.c_void_p(self.workspace.data_ptr()), self.workspace.numel(),
                             ctypes.c_void_p(self.result.data_ptr()), _stream_ptr(stream)), "tf_track")

    def track(self, depth, intr, ref_points, ref_normals, ref_intr, ref_pose, init_pose, params=None,
              stream=None) -> dict:
        """one tracking call, then the result (synchronises)"""
        params = params or make_track_params()
        self.track_async(depth, intr, ref_points, ref_normals, ref_intr, ref_pose, init_pose, params, stream)
        return parse_track_result(self.result.cpu().numpy())


TF_TRACK_NOALLOC_MAX_BYTES = 8 << 20


def tf_track_noalloc(depth, intr, ref_points, ref_normals, ref_intr, ref_pose, init_pose, params, result,
                     stream=None):
    """tf_track on the library's fixed device workspace (no allocation);
    `result`: device buffer of sizeof(tf_track_result) bytes"""
    fmt = TF_DEPTH_U16_MM if depth.dtype.itemsize == 2 else TF_DEPTH_F32_M
    K, Kr = make_intrinsics(intr), make_intrinsics(ref_intr)
    _, Mr = _pose_arg(ref_pose)
    _, Mi = _pose_arg(init_pose)
    check(lib().tf_track_noalloc(ctypes.c_void_p(depth.data_ptr()), fmt, ctypes.byref(K),
                                 ctypes.c_void_p(ref_points.data_ptr()), ctypes.c_void_p(ref_normals.data_ptr()),
                                 ctypes.byref(Kr), Mr, Mi, ctypes.byref(params), ctypes.c_void_p(result.data_ptr()),
                                 _stream_ptr(stream)), "tf_track_noalloc")


# ---- bilateral depth filter ------------------------------------------------------------

def tf_bilateral(depth, out, radius=2, sigma_space=2.5, sigma_range=0.025, stream=None):
    """bilateral filter of depth (H, W) uint16 mm or float32 m into out (H, W) float32 m"""
    fmt = TF_DEPTH_U16_MM if depth.dtype.itemsize == 2 else TF_DEPTH_F32_M
    H, W = int(depth.shape[-2]), int(depth.shape[-1])
    p = tf_bilateral_params(int(radius), float(sigma_space), float(sigma_range))
    check(lib().tf_bilateral(ctypes.c_void_p(depth.data_ptr()), fmt, W, H, ctypes.byref(p),
                             ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)), "tf_bilateral")
    return out


class Bilateral:
    """The bilateral filter as a depth prefilter with the Denoiser's forward()
    interface: (1, H, W) depth in, (1, H, W) float32 metres out."""

    def __init__(self, height, width, radius=2, sigma_space=2.5, sigma_range=0.025):
        self.H, self.W = height, width
        self.args = (radius, sigma_space, sigma_range)

    def forward(self, depth, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty((1, self.H, self.W), dtype=torch.float32, device="cuda")
        tf_bilateral(depth.reshape(self.H, self.W), out.reshape(self.H, self.W), *self.args, stream=stream)
        return out


# ---- surfel fusion -------------------------------------------------------------------

TF_FLAG_SURFEL_OVERFLOW = 0x20


class SurfelMap:
    """A surfel map on the current HIP device (Sec. 7.3), owning its workspace."""

    def __init__(self, capacity, max_width, max_height, sigma=0.6, max_depth_diff=0.05, min_normal_dot=0.5,
                 stream=None):
        import torch
        self.params = tf_surfel_params(int(capacity), int(max_width), int(max_height), float(sigma),
                                       float(max_depth_diff), float(min_normal_dot))
        nbytes = int(lib().tf_surfel_workspace_bytes(ctypes.byref(self.params)))
        if nbytes == 0:
            raise TsdfError("invalid surfel map parameters")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        h = _VP()
        check(lib().tf_surfel_create(ctypes.byref(self.params), ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                                     _stream_ptr(stream), ctypes.byref(h)), "tf_surfel_create")
        self.h = h
        self.last_shape = None

    def close(self):
        if getattr(self, "h", None):
            lib().tf_surfel_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reset(self, stream=None):
        check(lib().tf_surfel_reset(self.h, _stream_ptr(stream)), "tf_surfel_reset")

    def fuse(self, depth, intr, pose, stream=None):
        fmt = TF_DEPTH_U16_MM if depth.dtype.itemsize == 2 else TF_DEPTH_F32_M
        K = make_intrinsics(intr)
        _, Mp = _pose_arg(pose)
        check(lib().tf_surfel_fuse(self.h, ctypes.c_void_p(depth.data_ptr()), fmt, ctypes.byref(K), Mp,
                                   _stream_ptr(stream)), "tf_surfel_fuse")
        self.last_shape = (K.height, K.width)

    def stats(self, stream=None) -> dict:
        n, f, fr = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
        check(lib().tf_surfel_stats(self.h, ctypes.byref(n), ctypes.byref(f), ctypes.byref(fr), _stream_ptr(stream)),
              "tf_surfel_stats")
        return {"count": int(n.value), "flags": int(f.value), "frames": int(fr.value)}

    def export(self, stream=None):
        """(pos (n, 4), nrm (n, 4), time (n,)) on the host"""
        import torch
        n = self.stats(stream)["count"]
        pos = torch.empty((max(1, n), 4), dtype=torch.float32, device="cuda")
        nrm = torch.empty_like(pos)
        tm = torch.empty(max(1, n), dtype=torch.int32, device="cuda")
        check(lib().tf_surfel_export(self.h, n, ctypes.c_void_p(pos.data_ptr()), ctypes.c_void_p(nrm.data_ptr()),
                                     ctypes.c_void_p(tm.data_ptr()), _stream_ptr(stream)), "tf_surfel_export")
        return pos[:n].cpu().numpy(), nrm[:n].cpu().numpy(), tm[:n].cpu().numpy()

    def export_frame(self, stream=None):
        """(index map, correspondences) of the last fused frame, (H, W) int32 each"""
        import torch
        H, W = self.last_shape
        im = torch.empty((H, W), dtype=torch.int32, device="cuda")
        co = torch.empty((H, W), dtype=torch.int32, device="cuda")
        check(lib().tf_surfel_export_frame(self.h, ctypes.c_void_p(im.data_ptr()), ctypes.c_void_p(co.data_ptr()),
                                           _stream_ptr(stream)), "tf_surfel_export_frame")
        return im.cpu().numpy(), co.cpu().numpy()
