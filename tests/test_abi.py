"""The C ABI library loads on a machine without a GPU and exports every
symbol include/tsdf.h declares; argument validation happens on the host."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "tsdf.h")).read()
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
