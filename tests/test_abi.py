"""Host-side checks of the C ABI: the library loads, exports every entry point
the header declares, and rejects bad arguments before touching a device."""

import ctypes
import os
import re

import pytest

from paper_2601_17354_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pocketgs.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(pgs_\w+)\s*\(", text, re.M)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("pgs_project", "pgs_bin_sort", "pgs_render_fwd", "pgs_render_bwd",
                 "pgs_project_bwd", "pgs_sort_pairs", "pgs_loss_l1_dssim", "pgs_adam_step",
                 "pgs_knn", "pgs_pca_seed", "pgs_last_error", "pgs_version"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(_declared()) == set(_lib.SIGNATURES)


def test_version_string():
    assert _lib.load().pgs_version().decode().startswith("pocketgs-gfx950")


def test_invalid_arguments_are_rejected_on_the_host():
    lib = _lib.load()
    cam = _lib.PgsCamera()
    cam.width, cam.height, cam.fx, cam.fy = 64, 48, 50.0, 50.0
    st = lib.pgs_project(None, -1, 0, ctypes.byref(cam), 16, 16, None, None, None, None, None)
    assert st == _lib.PGS_ERR_INVALID_ARG
    assert b"n < 0" in lib.pgs_last_error()
    st = lib.pgs_project(None, 10, 4, ctypes.byref(cam), 16, 16, None, None, None, None, None)
    assert st == _lib.PGS_ERR_INVALID_ARG
    assert lib.pgs_knn(None, 100, 5, None, None, None, 0, None) == _lib.PGS_ERR_INVALID_ARG
    assert lib.pgs_sort_pairs(None, None, None, 10, 70, None, 0, None) == _lib.PGS_ERR_INVALID_ARG
    lr = (ctypes.c_float * 1)(0.1)
    assert lib.pgs_adam_step(None, None, None, None, 65, 10, lr, 1, 0.9, 0.999, 1e-15, None) == \
        _lib.PGS_ERR_INVALID_ARG
    bg = (ctypes.c_float * 3)(0, 0, 0)
    st = lib.pgs_render_fwd(64, 48, 12, 8, None, 0, None, None, 0, bg, None, None, None, None, None, None,
                            None)
    assert st == _lib.PGS_ERR_INVALID_ARG and b"unsupported tile" in lib.pgs_last_error()
    cams = (_lib.PgsCamera * 2)()
    for c in cams:
        c.width, c.height = 64, 48
    vb = _lib.PgsViewBatch(2, ctypes.cast(cams, ctypes.POINTER(_lib.PgsCamera)), 16, 16, 100, 0)
    st = lib.pgs_render_fwd_views(ctypes.byref(vb), None, 0, None, None, bg, None, None, None, None, None, None,
                                  None, None)
    assert st == _lib.PGS_ERR_INVALID_ARG and b"batch 100" in lib.pgs_last_error()
    vb.batch, vb.n_views = 64, 17
    assert lib.pgs_views_layout(ctypes.byref(vb), None, None) == -1
    vb.n_views = 2
    to = (ctypes.c_int32 * 3)()
    po = (ctypes.c_int64 * 3)()
    assert lib.pgs_views_layout(ctypes.byref(vb), to, po) == 24 and list(to) == [0, 12, 24]
    assert list(po) == [0, 64 * 48, 2 * 64 * 48]


def test_workspace_queries_grow_with_size():
    lib = _lib.load()
    assert lib.pgs_bin_sort_workspace(1000, 1 << 20) > lib.pgs_bin_sort_workspace(1000, 1 << 10)
    assert lib.pgs_sort_workspace(1 << 20) >= 12 * (1 << 20)
    assert lib.pgs_loss_workspace(1920, 1440) >= 9 * 4 * 1920 * 1440


def test_missing_library_fails_loudly(tmp_path):
    saved = _lib._lib
    try:
        _lib._lib = None
        with pytest.raises(ImportError):
            _lib.load(str(tmp_path / "nope.so"))
    finally:
        _lib._lib = saved


def test_ba_rejects_bad_problems_before_any_launch():
    import ctypes
    from paper_2601_17354_amd import _lib
    lib = _lib.load()
    pb = _lib.PgsBaProblem()
    pb.n_cams, pb.n_points, pb.n_obs, pb.gauge_axis, pb.huber_delta = 1, 10, 20, 0, 2.0
    st = lib.pgs_ba_cost(ctypes.byref(pb), None, None, None, None, None, 0, None)
    assert st == _lib.PGS_ERR_INVALID_ARG and b"n_cams" in lib.pgs_last_error()
    pb.n_cams = 4
    pb.gauge_axis = 3
    assert lib.pgs_ba_step(ctypes.byref(pb), None, None, None, 1e-3, None, None, None, 0, None) == \
        _lib.PGS_ERR_INVALID_ARG
    pb.gauge_axis, pb.huber_delta = 0, 0.0
    assert lib.pgs_ba_cost(ctypes.byref(pb), None, None, None, None, None, 0, None) == _lib.PGS_ERR_INVALID_ARG
    pb.huber_delta = 2.0
    assert lib.pgs_ba_step(ctypes.byref(pb), None, None, None, -1.0, None, None, None, 0, None) == \
        _lib.PGS_ERR_INVALID_ARG
    assert lib.pgs_ba_workspace(60, 1000, 5000) > 0


def test_mvs_rejects_bad_arguments_before_any_launch():
    lib = _lib.load()
    p = _lib.PgsMvsParams(100, 4, 32, 0.4, 0.5, 0.25, 0.1)
    assert lib.pgs_mvs_cost(None, 64, 48, None, None, 1, None, None, ctypes.byref(p), None,
                            None) == _lib.PGS_ERR_INVALID_ARG
    assert b"n_planes" in lib.pgs_last_error()
    p.n_planes, p.p2 = 64, 5000
    assert lib.pgs_mvs_sgm(None, 64, 48, None, 1, None, ctypes.byref(p), None, None, None, None, 0,
                           None) == _lib.PGS_ERR_INVALID_ARG
    assert b"penalties" in lib.pgs_last_error()
    p.p2 = 32
    assert lib.pgs_mvs_sgm(None, 64, 48, None, 1, None, ctypes.byref(p), None, None, None, None, 0,
                           None) == _lib.PGS_ERR_INVALID_ARG
    assert lib.pgs_mvs_census(None, 1, 64, 48, None, None) == _lib.PGS_ERR_INVALID_ARG
    assert lib.pgs_mvs_depth_range(None, 2, 0, 48, None, 0, None, None, 0, None) == _lib.PGS_ERR_INVALID_ARG
    p.sigma_b = 0.0
    assert lib.pgs_mvs_select_ref(ctypes.c_void_p(8), 3, ctypes.byref(p), ctypes.c_void_p(8),
                                  None) == _lib.PGS_ERR_INVALID_ARG
    assert lib.pgs_mvs_range_workspace(3, 10) >= 3 * 10 * 8 + 12
    assert lib.pgs_mvs_sgm_workspace(2, 8, 4, 64) >= 2 * 8 * 4 * 64 * 2


def test_noalloc_sort_scratch_holds_its_largest_capacity_and_rejects_beyond():
    lib = _lib.load()
    assert lib.pgs_sort_workspace(_lib.SORT_NOALLOC_MAX_PAIRS) <= _lib.SORT_NOALLOC_SCRATCH_BYTES
    st = lib.pgs_sort_pairs_noalloc(None, None, None, _lib.SORT_NOALLOC_MAX_PAIRS + 1, 40, None)
    assert st == _lib.PGS_ERR_INVALID_ARG and b"exceeds" in lib.pgs_last_error()
    assert lib.pgs_sort_pairs_noalloc(None, None, None, 10, 65, None) == _lib.PGS_ERR_INVALID_ARG


def test_runtime_helpers_reject_bad_arguments_on_the_host():
    lib = _lib.load()
    assert lib.pgs_check_flags(None, None, None) == _lib.PGS_ERR_INVALID_ARG
    assert lib.pgs_graph_begin(None) == _lib.PGS_ERR_INVALID_ARG       # the null stream
    assert b"null stream" in lib.pgs_last_error()
    assert lib.pgs_graph_end(None, None) == _lib.PGS_ERR_INVALID_ARG
    assert lib.pgs_graph_launch(None, None) == _lib.PGS_ERR_INVALID_ARG
    lib.pgs_graph_destroy(None)                                         # no-op
