"""The C ABI library loads on a machine without a GPU and exports every
symbol include/tsdf.h declares; argument validation happens on the host."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    import glob
    src = "".join(open(f).read() for f in sorted(glob.glob(os.path.join(ROOT, "include", "*.h"))))
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tf_[a-z_]+)\s*\(", src)))


def test_header_matches_binding_list():
    import paper_1708_00783_amd as T
    assert sorted(T.EXPORTS) == _declared()


def test_library_exports_every_declared_symbol():
    import paper_1708_00783_amd as T
    L = T.lib()
    for name in _declared():
        assert hasattr(L, name), name


def test_workspace_size_and_validation():
    import paper_1708_00783_amd as T
    from synth import configs
    p = T.make_params(configs.C2_VOLUME, 640, 480)
    n = T.tf_workspace_bytes(p)
    # voxel blocks dominate: 2^18 x 1536 B
    assert (1 << 18) * 1536 < n < (1 << 18) * 1536 + (200 << 20)
    bad = T.make_params(configs.C2_VOLUME, 640, 480)
    bad.n_buckets = 1000          # not a power of two
    assert T.tf_workspace_bytes(bad) == 0
    bad = T.make_params(configs.C2_VOLUME, 640, 480)
    bad.max_w = 256
    assert T.tf_workspace_bytes(bad) == 0
    # tf_create rejects before touching the device
    ctx = ctypes.c_void_p()
    assert T.lib().tf_create(ctypes.byref(bad), None, 0, None, None, None, ctypes.byref(ctx)) == T.TF_E_INVAL
    assert T.lib().tf_create(ctypes.byref(p), ctypes.c_void_p(256), 10, None, None, None,
                             ctypes.byref(ctx)) == T.TF_E_SPACE
    assert T.lib().tf_create(ctypes.byref(p), ctypes.c_void_p(255), n, None, None, None,
                             ctypes.byref(ctx)) == T.TF_E_INVAL
    assert T.lib().tf_integrate(None, None, 0, None, None) == T.TF_E_INVAL
    assert T.lib().tf_status_string(T.TF_E_ORDER) == b"call order violated"


def test_multi_workspace_size_and_validation():
    import paper_1708_00783_amd as T
    from synth import configs
    p = T.make_params(configs.C1_VOLUME, 160, 120)
    L = T.lib()
    one = T.tf_workspace_bytes(p)
    n3 = L.tf_multi_workspace_bytes(ctypes.byref(p), 3, 200, 150, 1 << 16)
    # three submap workspaces, their block lists, the bins and the world-cell
    # submap masks (2^25 cells of 8 bytes)
    base = 3 * one + 3 * 16 * p.n_blocks + (1 << 16) * 32 + (8 << 25)
    assert base <= n3 < base + (8 << 20)
    assert L.tf_multi_workspace_bytes(ctypes.byref(p), 0, 200, 150, 1 << 16) == 0
    assert L.tf_multi_workspace_bytes(ctypes.byref(p), 65, 200, 150, 1 << 16) == 0
    assert L.tf_multi_workspace_bytes(ctypes.byref(p), 3, 200, 150, 0) == 0
    sw = T.make_params(configs.C1_VOLUME, 160, 120, swap_transfer_blocks=64)
    assert L.tf_multi_workspace_bytes(ctypes.byref(sw), 3, 200, 150, 1 << 16) == 0   # submaps never swap
    assert L.tf_multi_host_bytes() >= 2 * 24 * 1024
    poses = (ctypes.c_float * 48)(*([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1] * 3))
    m = ctypes.c_void_p()
    hb = L.tf_multi_host_bytes()
    # rejected on the host before any device work
    assert L.tf_multi_create(ctypes.byref(p), 3, poses, 200, 150, 1 << 16, ctypes.c_void_p(256), 10,
                             ctypes.c_void_p(256), hb, None, ctypes.byref(m)) == T.TF_E_SPACE
    assert L.tf_multi_create(ctypes.byref(p), 3, None, 200, 150, 1 << 16, ctypes.c_void_p(256), n3,
                             ctypes.c_void_p(256), hb, None, ctypes.byref(m)) == T.TF_E_INVAL
    assert L.tf_multi_create(ctypes.byref(p), 3, poses, 200, 150, 1 << 16, ctypes.c_void_p(256), n3,
                             ctypes.c_void_p(256), 16, None, ctypes.byref(m)) == T.TF_E_SPACE
    cfg = T.tf_multi_config(24, 8, 256, 256, 256)
    assert L.tf_multi_set_config(None, ctypes.byref(cfg)) == T.TF_E_INVAL
    assert L.tf_multi_integrate(None, None, 0, None, None, None, 0, None) == T.TF_E_INVAL
    assert L.tf_multi_raycast(None, None, 0, None) == T.TF_E_INVAL


def test_persistence_and_camera_depth_validation():
    """argument errors of tf_save / tf_load / tf_camera_depth, caught on the host"""
    import paper_1708_00783_amd as T
    L = T.lib()
    assert L.tf_save(None, b"/tmp/x", None) == T.TF_E_INVAL
    assert L.tf_load(None, b"/tmp/x", None) == T.TF_E_INVAL
    M = (ctypes.c_float * 16)(*[1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1])
    assert L.tf_camera_depth(None, 4, 4, M, ctypes.c_void_p(256), None) == T.TF_E_INVAL
    assert L.tf_camera_depth(ctypes.c_void_p(256), 0, 4, M, ctypes.c_void_p(256), None) == T.TF_E_INVAL
    assert L.tf_camera_depth(ctypes.c_void_p(264), 4, 4, M, ctypes.c_void_p(256), None) == T.TF_E_INVAL
    assert L.tf_camera_depth(ctypes.c_void_p(256), 4, 4, None, ctypes.c_void_p(256), None) == T.TF_E_INVAL
    assert L.tf_status_string(T.TF_E_IO) == b"file error or not a volume of these parameters"
