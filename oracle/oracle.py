"""ctypes wrapper around the plain C oracle (tsdf_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the package smoke check and
the benchmark's CPU-baseline leg, never by the product path.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "tsdf_oracle.c")
LIB = os.path.join(_HERE, "liboracle.so")
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
          "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain IEEE float, no contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None

_F = ctypes.POINTER(ctypes.c_float)
_I32 = ctypes.POINTER(ctypes.c_int32)
_I16 = ctypes.POINTER(ctypes.c_int16)
_U8 = ctypes.POINTER(ctypes.c_uint8)
_U16 = ctypes.POINTER(ctypes.c_uint16)
_VP = ctypes.c_void_p


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(LIB)
        sig = {
            "or_set_threads": (None, [ctypes.c_int]),
            "or_get_threads": (ctypes.c_int, []),
            "or_hash": (ctypes.c_uint32, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint32]),
            "or_create": (_VP, [ctypes.c_float, ctypes.c_float, ctypes.c_int, ctypes.c_int,
                                ctypes.c_int, ctypes.c_int]),
            "or_destroy": (None, [_VP]),
            "or_n_entries": (ctypes.c_int, [_VP]),
            "or_flags": (ctypes.c_uint32, [_VP]),
            "or_n_free_blocks": (ctypes.c_int, [_VP]),
            "or_n_free_excess": (ctypes.c_int, [_VP]),
            "or_n_visible": (ctypes.c_int, [_VP]),
            "or_lookup": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
            "or_insert": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
            "or_depth_from_mm": (None, [_U16, _F, ctypes.c_int]),
            "or_segment_blocks": (ctypes.c_int, [ctypes.c_float, ctypes.c_int, ctypes.c_int, _F,
                                                 ctypes.c_int, ctypes.c_int, _F, ctypes.c_float,
                                                 ctypes.c_float, _I32, ctypes.c_int]),
            "or_alloc_and_visible": (None, [_VP, _F, ctypes.c_int, ctypes.c_int, _F, _F]),
            "or_integrate": (None, [_VP, _F, ctypes.c_int, ctypes.c_int, _F, _F]),
            "or_integrate_divide": (None, [_VP, _F, ctypes.c_int, ctypes.c_int, _F, _F]),
            "or_range": (None, [_VP, _I32, ctypes.c_int, ctypes.c_int, ctypes.c_int, _F, _F, _F, _F]),
            "or_raycast": (None, [_VP, ctypes.c_int, ctypes.c_int, _F, _F, _F, _F, _F, _F]),
            "or_trilinear": (ctypes.c_float, [_VP, ctypes.c_float, ctypes.c_float, ctypes.c_float]),
            "or_enable_swap": (ctypes.c_int, [_VP, ctypes.c_int]),
            "or_swap_out": (ctypes.c_int, [_VP]),
            "or_n_swapped_in": (ctypes.c_int, [_VP]),
            "or_get_entries": (None, [_VP, _I16, _I32, _I32]),
            "or_get_visible": (ctypes.c_int, [_VP, _I32]),
            "or_get_block_voxels": (None, [_VP, _I32, ctypes.c_int, _I16, _U8]),
            "or_get_host_block": (ctypes.c_int, [_VP, ctypes.c_int, _I16, _U8]),
            "or_set_block_voxels": (ctypes.c_int, [_VP, ctypes.c_int, _I16, _U8]),
            "or_compose": (None, [_F, _F, _F]),
            "or_multi_range": (None, [_VP, _F, ctypes.c_int, ctypes.c_int, ctypes.c_int, _F, _F, _F, _F]),
            "or_multi_raycast": (None, [_VP, _F, ctypes.c_int, ctypes.c_int, ctypes.c_int, _F, _F, _F, _F,
                                        _F, _F]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t)


def set_threads(n: int) -> None:
    lib().or_set_threads(int(n))


def get_threads() -> int:
    return int(lib().or_get_threads())


def hash_index(x: int, y: int, z: int, mask: int) -> int:
    return int(lib().or_hash(x, y, z, mask))


def depth_from_mm(mm: np.ndarray) -> np.ndarray:
    mm = np.ascontiguousarray(mm, np.uint16)
    out = np.empty(mm.shape, np.float32)
    lib().or_depth_from_mm(_p(mm, _U16), _p(out, _F), mm.size)
    return out


def segment_blocks(d, x, y, intr, W, H, pose, voxel_size, mu, cap=64) -> np.ndarray:
    keys = np.zeros((cap, 3), np.int32)
    intr = np.ascontiguousarray(intr, np.float32)
    pose = np.ascontiguousarray(pose, np.float32).reshape(16)
    n = lib().or_segment_blocks(float(d), int(x), int(y), _p(intr, _F), W, H, _p(pose, _F),
                                float(voxel_size), float(mu), _p(keys, _I32), cap)
    return keys[:n]


class Volume:
    """One voxel-hashed TSDF volume held by the oracle."""

    def __init__(self, voxel_size, mu, max_w, n_buckets, n_excess, n_blocks):
        self.voxel_size = float(voxel_size)
        self.mu = float(mu)
        self.max_w = int(max_w)
        self.n_buckets = int(n_buckets)
        self.n_excess = int(n_excess)
        self.n_blocks = int(n_blocks)
        self._h = lib().or_create(self.voxel_size, self.mu, self.max_w, self.n_buckets,
                                  self.n_excess, self.n_blocks)
        if not self._h:
            raise MemoryError("oracle volume allocation failed")

    @classmethod
    def from_params(cls, p):
        return cls(p.voxel_size, p.mu, p.max_w, p.n_buckets, p.n_excess, p.n_blocks)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.or_destroy(h)
            self._h = None

    # --- state -------------------------------------------------------------
    @property
    def n_entries(self) -> int:
        return lib().or_n_entries(self._h)

    @property
    def flags(self) -> int:
        return int(lib().or_flags(self._h))

    @property
    def n_free_blocks(self) -> int:
        return lib().or_n_free_blocks(self._h)

    @property
    def n_free_excess(self) -> int:
        return lib().or_n_free_excess(self._h)

    def lookup(self, x, y, z) -> int:
        return lib().or_lookup(self._h, x, y, z)

    def insert(self, x, y, z) -> int:
        return lib().or_insert(self._h, x, y, z)

    def entries(self):
        n = self.n_entries
        pos = np.empty((n, 3), np.int16)
        off = np.empty(n, np.int32)
        ptr = np.empty(n, np.int32)
        lib().or_get_entries(self._h, _p(pos, _I16), _p(off, _I32), _p(ptr, _I32))
        return pos, off, ptr

    def visible(self) -> np.ndarray:
        out = np.empty(self.n_entries, np.int32)
        n = lib().or_get_visible(self._h, _p(out, _I32))
        return out[:n].copy()

    def block_voxels(self, entry_ids):
        ids = np.ascontiguousarray(entry_ids, np.int32)
        sdf = np.empty((ids.size, 512), np.int16)
        w = np.empty((ids.size, 512), np.uint8)
        lib().or_get_block_voxels(self._h, _p(ids, _I32), ids.size, _p(sdf, _I16), _p(w, _U8))
        return sdf, w

    def set_block_voxels(self, entry, sdf, w) -> None:
        """overwrite one allocated entry's 512 voxels (in-block order lx + 8 ly + 64 lz)"""
        s = np.ascontiguousarray(sdf, np.int16).reshape(512)
        ww = np.ascontiguousarray(w, np.uint8).reshape(512)
        if not lib().or_set_block_voxels(self._h, int(entry), _p(s, _I16), _p(ww, _U8)):
            raise ValueError(f"entry {entry} has no device block")

    def allocated_positions(self) -> np.ndarray:
        """(N, 3) int block positions of entries with a device block, sorted."""
        pos, _, ptr = self.entries()
        return sort_rows(pos[ptr >= 0].astype(np.int32))

    def voxels_by_position(self):
        """dict-free form: (positions sorted (N,3), sdf (N,512), w (N,512))."""
        pos, _, ptr = self.entries()
        ids = np.flatnonzero(ptr >= 0).astype(np.int32)
        p = pos[ids].astype(np.int32)
        order = np.lexsort((p[:, 2], p[:, 1], p[:, 0]))
        ids = ids[order]
        sdf, w = self.block_voxels(ids)
        return p[order], sdf, w

    # --- pipeline ------------------------------------------------------------
    def alloc_and_visible(self, depth_m, intr, pose):
        d = np.ascontiguousarray(depth_m, np.float32)
        H, W = d.shape
        k = np.ascontiguousarray(intr, np.float32)
        M = np.ascontiguousarray(pose, np.float32).reshape(16)
        lib().or_alloc_and_visible(self._h, _p(d, _F), W, H, _p(k, _F), _p(M, _F))

    def integrate(self, depth_m, intr, pose, divide=False):
        d = np.ascontiguousarray(depth_m, np.float32)
        H, W = d.shape
        k = np.ascontiguousarray(intr, np.float32)
        M = np.ascontiguousarray(pose, np.float32).reshape(16)
        fn = lib().or_integrate_divide if divide else lib().or_integrate
        fn(self._h, _p(d, _F), W, H, _p(k, _F), _p(M, _F))

    def range_image(self, W, H, intr, pose, blocks=None):
        k = np.ascontiguousarray(intr, np.float32)
        M = np.ascontiguousarray(pose, np.float32).reshape(16)
        zmin = np.empty((H, W), np.float32)
        zmax = np.empty((H, W), np.float32)
        if blocks is None:
            blocks = self.visible()
        if isinstance(blocks, str) and blocks == "all":
            b = np.zeros(1, np.int32)
            n = -1
        else:
            b = np.ascontiguousarray(blocks, np.int32)
            n = b.size
        lib().or_range(self._h, _p(b, _I32), n, W, H, _p(k, _F), _p(M, _F), _p(zmin, _F), _p(zmax, _F))
        return zmin, zmax

    def raycast(self, W, H, intr, pose, zmin=None, zmax=None, blocks=None):
        if zmin is None:
            zmin, zmax = self.range_image(W, H, intr, pose, blocks)
        k = np.ascontiguousarray(intr, np.float32)
        M = np.ascontiguousarray(pose, np.float32).reshape(16)
        pts = np.empty((H, W, 4), np.float32)
        nrm = np.empty((H, W, 4), np.float32)
        zmin = np.ascontiguousarray(zmin, np.float32)
        zmax = np.ascontiguousarray(zmax, np.float32)
        lib().or_raycast(self._h, W, H, _p(k, _F), _p(M, _F), _p(zmin, _F), _p(zmax, _F),
                         _p(pts, _F), _p(nrm, _F))
        return pts, nrm

    def trilinear(self, X, Y, Z) -> float:
        return float(lib().or_trilinear(self._h, X, Y, Z))

    # --- swapping --------------------------------------------------------------
    def enable_swap(self, transfer_blocks):
        if lib().or_enable_swap(self._h, int(transfer_blocks)) != 0:
            raise MemoryError("oracle host store allocation failed")

    def swap_out(self) -> int:
        return lib().or_swap_out(self._h)

    @property
    def n_swapped_in(self) -> int:
        return lib().or_n_swapped_in(self._h)

    def host_block(self, entry):
        sdf = np.empty(512, np.int16)
        w = np.empty(512, np.uint8)
        ok = lib().or_get_host_block(self._h, int(entry), _p(sdf, _I16), _p(w, _U8))
        return (sdf, w) if ok else None

    # --- one whole frame ---------------------------------------------------------
    def frame(self, depth_m, intr, pose, W=None, H=None):
        """allocate + visible, integrate, raycast from the same pose."""
        self.alloc_and_visible(depth_m, intr, pose)
        self.integrate(depth_m, intr, pose)
        H0, W0 = np.shape(depth_m)
        return self.raycast(W or W0, H or H0, intr, pose)


def compose(A, P) -> np.ndarray:
    """A * inv(P) (rigid, double, rounded once): the camera matrix of a submap"""
    A = np.ascontiguousarray(A, np.float32).reshape(16)
    P = np.ascontiguousarray(P, np.float32).reshape(16)
    out = np.empty(16, np.float32)
    lib().or_compose(_p(A, _F), _p(P, _F), _p(out, _F))
    return out.reshape(4, 4)


class Multi:
    """Rigid submaps (Sec. 7.2): volumes with poses P_i (world -> submap)."""

    def __init__(self, vols, poses):
        self.vols = list(vols)
        self.poses = np.ascontiguousarray(np.asarray(poses, np.float32).reshape(len(self.vols), 16))
        self._arr = (ctypes.c_void_p * len(self.vols))(*[v._h for v in self.vols])

    def integrate_frame(self, i, depth_m, intr, M_d):
        """allocate + integrate one frame into submap i (camera M_d composed with P_i)"""
        Mi = compose(M_d, self.poses[i])
        self.vols[i].alloc_and_visible(depth_m, intr, Mi)
        self.vols[i].integrate(depth_m, intr, Mi)

    def range_image(self, W, H, intr, V):
        k = np.ascontiguousarray(intr, np.float32)
        Vv = np.ascontiguousarray(V, np.float32).reshape(16)
        zmin = np.empty((H, W), np.float32)
        zmax = np.empty((H, W), np.float32)
        lib().or_multi_range(ctypes.cast(self._arr, _VP), _p(self.poses, _F), len(self.vols), W, H, _p(k, _F),
                             _p(Vv, _F), _p(zmin, _F), _p(zmax, _F))
        return zmin, zmax

    def raycast(self, W, H, intr, V, mask=None):
        """combined-field raycast of a W x H view; with `mask` (H x W bool) only
        those pixels are marched (the range image is still the whole view's;
        the other pixels get an empty range and no hit)"""
        zmin, zmax = self.range_image(W, H, intr, V)
        if mask is not None:
            zmin = np.ascontiguousarray(np.where(mask, zmin, np.float32(np.inf)), np.float32)
            zmax = np.ascontiguousarray(np.where(mask, zmax, np.float32(-np.inf)), np.float32)
        k = np.ascontiguousarray(intr, np.float32)
        Vv = np.ascontiguousarray(V, np.float32).reshape(16)
        pts = np.empty((H, W, 4), np.float32)
        nrm = np.empty((H, W, 4), np.float32)
        lib().or_multi_raycast(ctypes.cast(self._arr, _VP), _p(self.poses, _F), len(self.vols), W, H, _p(k, _F),
                               _p(Vv, _F), _p(zmin, _F), _p(zmax, _F), _p(pts, _F), _p(nrm, _F))
        return pts, nrm


def sort_rows(a: np.ndarray) -> np.ndarray:
    a = np.asarray(a)
    if a.size == 0:
        return a.reshape(0, 3)
    order = np.lexsort((a[:, 2], a[:, 1], a[:, 0]))
    return a[order]
