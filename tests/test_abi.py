"""Host-side checks of the C ABI: the library loads, exports every declared
function, and rejects invalid arguments before touching a device."""

import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hgmm.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hgmm_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1807_02587_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1807_02587_amd import build
        build.build()
    return _lib.load()


def test_header_declares_the_entry_points():
    names = _declared_functions()
    for must in ("hgmm_build", "hgmm_register", "hgmm_estep", "hgmm_normal_equations", "hgmm_tree_export",
                 "hgmm_tree_import", "hgmm_tree_labels", "hgmm_tree_destroy", "hgmm_last_error"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    from paper_1807_02587_amd import _lib
    assert set(_declared_functions()) <= set(_lib.SIGNATURES)


def test_node_counts(lib):
    assert [lib.hgmm_tree_nodes(L) for L in range(1, 7)] == [8, 72, 584, 4680, 37448, 299592]
    assert [lib.hgmm_level_offset(l) for l in range(0, 6)] == [0, 8, 72, 584, 4680, 37448]
    assert lib.hgmm_tree_nodes(0) == -1 and lib.hgmm_tree_nodes(7) == -1


def test_defaults(lib):
    from paper_1807_02587_amd._lib import BuildParams, RegParams
    bp, rp = BuildParams(), RegParams()
    assert lib.hgmm_params_default(C.byref(bp), C.byref(rp)) == 0
    assert (bp.levels, bp.build_iters, bp.reg_eps, bp.min_mass) == (2, 30, 1e-6, 1.0)
    assert (rp.max_iters, rp.lambda_c, rp.tol_rot, rp.tol_trans_rel) == (30, 0.01, 1e-6, 1e-6)


def test_workspace_sizes_monotone(lib):
    a = lib.hgmm_build_workspace_bytes(10_000, 2)
    b = lib.hgmm_build_workspace_bytes(300_000, 5)
    assert 0 < a < b
    assert lib.hgmm_build_workspace_bytes(100, 0) == 0
    assert 0 < lib.hgmm_register_workspace_bytes(10_000, 2) < lib.hgmm_register_workspace_bytes(300_000, 5)


def test_argument_errors_before_device_work(lib):
    from paper_1807_02587_amd._lib import BuildParams
    h = C.c_void_p(None)
    bad_levels = BuildParams(9, 30, 1e-6, 1.0)
    rc = lib.hgmm_build(C.c_void_p(16), 100, C.byref(bad_levels), C.c_void_p(16), 1 << 20, None, C.byref(h))
    assert rc == -1 and "levels" in lib.hgmm_last_error().decode()
    good = BuildParams(2, 30, 1e-6, 1.0)
    rc = lib.hgmm_build(C.c_void_p(16), 5, C.byref(good), C.c_void_p(16), 1 << 20, None, C.byref(h))
    assert rc == -2
    neg_eps = BuildParams(2, 30, -1.0, 1.0)
    assert lib.hgmm_build(C.c_void_p(16), 100, C.byref(neg_eps), C.c_void_p(16), 1 << 20, None, C.byref(h)) == -1
    assert lib.hgmm_build(None, 100, C.byref(good), C.c_void_p(16), 1 << 20, None, C.byref(h)) == -1
    assert h.value is None


def test_odometry_argument_errors_before_device_work(lib):
    import numpy as np
    from paper_1807_02587_amd._lib import BuildParams, RegParams
    bp = BuildParams(2, 30, 1e-6, 1.0)
    rp = RegParams(30, 0, 0.01, 1e-6, 1e-6)
    off = np.array([0, 100, 200, 300], np.int64)
    optr = off.ctypes.data_as(C.c_void_p)
    need = lib.hgmm_odometry_workspace_bytes(optr, 3, 2)
    assert need > 0
    assert lib.hgmm_odometry_workspace_bytes(optr, 1, 2) == 0      # one frame is no sequence
    assert lib.hgmm_odometry_workspace_bytes(optr, 3, 7) == 0      # levels out of range
    out = [np.zeros(64) for _ in range(4)]
    it = np.zeros(4, np.int32)
    h = C.c_void_p(None)
    args = lambda F, ws_bytes: (C.c_void_p(16), optr, F, C.byref(bp), C.byref(rp), None, None, 0, C.c_void_p(16),
                                ws_bytes, None, C.byref(h), *[o.ctypes.data_as(C.c_void_p) for o in out],
                                it.ctypes.data_as(C.c_void_p), None)
    assert lib.hgmm_odometry(*args(1, need)) == -1
    assert lib.hgmm_odometry(*args(3, need - 1)) == -1 and "workspace" in lib.hgmm_last_error().decode()
    bad = np.array([0, 100, 50, 300], np.int64)
    assert lib.hgmm_odometry(C.c_void_p(16), bad.ctypes.data_as(C.c_void_p), 3, C.byref(bp), C.byref(rp), None,
                             None, 0, C.c_void_p(16), need, None, C.byref(h),
                             *[o.ctypes.data_as(C.c_void_p) for o in out], it.ctypes.data_as(C.c_void_p), None) == -1
    assert h.value is None
    short = np.array([0, 100, 200, 203], np.int64)   # last frame of 3 points
    assert lib.hgmm_odometry(C.c_void_p(16), short.ctypes.data_as(C.c_void_p), 3, C.byref(bp), C.byref(rp), None,
                             None, 0, C.c_void_p(16), need, None, C.byref(h),
                             *[o.ctypes.data_as(C.c_void_p) for o in out], it.ctypes.data_as(C.c_void_p), None) == -2
    assert h.value is None


def test_noalloc_entry_point_limits(lib):
    """The allocation-free registration reports its static scratch size and
    rejects null arguments before any device work."""
    from paper_1807_02587_amd._lib import RegParams
    assert lib.hgmm_noalloc_scratch_bytes() == 48 << 20
    rp = RegParams(30, 0, 0.01, 1e-6, 1e-6)
    R = (C.c_double * 9)()
    t = (C.c_double * 3)()
    it = C.c_int(0)
    assert lib.hgmm_register_noalloc(None, C.c_void_p(16), 100, C.byref(rp), None, None, None, R, t,
                                     C.byref(it), None) == -1
    assert lib.hgmm_register_noalloc(C.c_void_p(16), C.c_void_p(16), 0, C.byref(rp), None, None, None, R, t,
                                     C.byref(it), None) == -2
    # the workspace a cloud needs grows with it: 2^19 points on 5 levels fit, 2^21 do not
    assert lib.hgmm_register_workspace_bytes(1 << 19, 5) <= lib.hgmm_noalloc_scratch_bytes()
    assert lib.hgmm_register_workspace_bytes(1 << 21, 5) > lib.hgmm_noalloc_scratch_bytes()
