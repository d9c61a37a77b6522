"""ctypes view of libpocketgs.so (declarations in include/pocketgs.h).

Loading fails loudly when the library has not been built: there is no other
implementation of these calls in this package.
"""

from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_float, c_int32, c_size_t, c_uint32, c_uint64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpocketgs.so")

PGS_OK = 0
PGS_ERR_INVALID_ARG = 1
PGS_ERR_HIP = 2
PGS_ERR_CAPACITY = 3
PGS_FLAG_PAIR_OVERFLOW = 1
PGS_FLAG_CACHE_OVERFLOW = 2
SORT_NOALLOC_MAX_PAIRS = 1 << 20
SORT_NOALLOC_SCRATCH_BYTES = 16 << 20
PROJ_FIELDS = 12
PROJ_STRIDE = 16
GRAD2D_FIELDS = 9
GRAD2D_STRIDE = 16


class PgsCamera(ctypes.Structure):
    _fields_ = [("width", c_int32), ("height", c_int32), ("fx", c_float), ("fy", c_float),
                ("cx", c_float), ("cy", c_float), ("viewmat", c_float * 12)]


class PgsReplay(ctypes.Structure):
    _fields_ = [("mask_dev", c_void_p), ("steps_dev", c_void_p), ("base_dev", c_void_p), ("used_dev", c_void_p),
                ("entry_dev", c_void_p), ("count_dev", c_void_p), ("entry_capacity", c_uint64),
                ("pair_capacity", c_uint32), ("entry_words", c_uint32)]


class PgsViewBatch(ctypes.Structure):
    _fields_ = [("n_views", c_int32), ("cams", POINTER(PgsCamera)), ("tile_w", c_int32), ("tile_h", c_int32),
                ("batch", c_int32), ("blocks", c_int32)]


class PgsMvsParams(ctypes.Structure):
    _fields_ = [("n_planes", c_int32), ("p1", c_int32), ("p2", c_int32), ("conf_min", c_double),
                ("b_target", c_double), ("sigma_b", c_double), ("alpha_min", c_double)]


class PgsBaProblem(ctypes.Structure):
    _fields_ = [("n_cams", c_int32), ("n_points", c_int32), ("n_obs", c_int32), ("gauge_axis", c_int32),
                ("fx", c_double), ("fy", c_double), ("cx", c_double), ("cy", c_double), ("huber_delta", c_double),
                ("obs_cam_dev", c_void_p), ("obs_pt_dev", c_void_p), ("obs_uv_dev", c_void_p),
                ("point_start_dev", c_void_p), ("cam_obs_dev", c_void_p), ("cam_start_dev", c_void_p)]


# name -> (restype, argtypes)
SIGNATURES = {
    "pgs_version": (c_char_p, []),
    "pgs_last_error": (c_char_p, []),
    "pgs_check_flags": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "pgs_graph_begin": (c_int32, [c_void_p]),
    "pgs_graph_end": (c_int32, [c_void_p, POINTER(c_void_p)]),
    "pgs_graph_launch": (c_int32, [c_void_p, c_void_p]),
    "pgs_graph_destroy": (None, [c_void_p]),
    "pgs_project": (c_int32, [c_void_p, c_int32, c_int32, POINTER(PgsCamera), c_int32, c_int32,
                              c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "pgs_bin_sort_workspace": (c_size_t, [c_int32, c_uint32]),
    "pgs_bin_sort": (c_int32, [c_int32, c_void_p, c_void_p, c_void_p, c_int32, c_int32, c_int32,
                               c_uint32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                               c_void_p, c_size_t, c_void_p]),
    "pgs_sort_workspace": (c_size_t, [c_uint32]),
    "pgs_sort_pairs": (c_int32, [c_void_p, c_void_p, c_void_p, c_uint32, c_int32, c_void_p,
                                 c_size_t, c_void_p]),
    "pgs_sort_pairs_noalloc": (c_int32, [c_void_p, c_void_p, c_void_p, c_uint32, c_int32, c_void_p]),
    "pgs_trace_entries": (c_size_t, [c_uint32, c_int32, c_int32]),
    "pgs_render_fwd": (c_int32, [c_int32, c_int32, c_int32, c_int32, c_void_p, c_int32, c_void_p,
                                 c_void_p, c_int32, POINTER(c_float), c_void_p, c_void_p, c_void_p,
                                 POINTER(PgsReplay), c_void_p, c_void_p, c_void_p]),
    "pgs_tile_order": (c_int32, [c_void_p, c_int32, c_int32, c_int32, c_void_p, c_void_p]),
    "pgs_render_bwd": (c_int32, [c_int32, c_int32, c_int32, c_int32, c_void_p, c_int32, c_void_p,
                                 c_void_p, c_int32, POINTER(c_float), c_void_p, c_void_p,
                                 POINTER(PgsReplay), c_void_p, c_void_p, c_void_p, c_void_p]),
    "pgs_project_bwd": (c_int32, [c_void_p, c_int32, c_int32, POINTER(PgsCamera), c_void_p,
                                  c_void_p, c_void_p, c_void_p]),
    "pgs_loss_workspace": (c_size_t, [c_int32, c_int32]),
    "pgs_loss_l1_dssim": (c_int32, [c_void_p, c_void_p, c_int32, c_int32, c_float, c_void_p,
                                    c_void_p, c_void_p, c_size_t, c_void_p]),
    "pgs_psnr": (c_int32, [c_void_p, c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_size_t, c_void_p]),
    "pgs_adam_step": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_int32,
                                POINTER(c_float), c_int32, c_float, c_float, c_float, c_void_p]),
    "pgs_knn_workspace": (c_size_t, [c_int32]),
    "pgs_knn": (c_int32, [c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "pgs_pca_seed": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_int32, c_float,
                               c_void_p, c_void_p]),
    "pgs_views_layout": (c_int32, [POINTER(PgsViewBatch), POINTER(c_int32), POINTER(ctypes.c_int64)]),
    "pgs_project_views": (c_int32, [POINTER(PgsViewBatch), c_void_p, c_int32, c_int32, c_void_p, c_void_p,
                                    c_void_p, c_void_p, c_void_p]),
    "pgs_project_bwd_views": (c_int32, [POINTER(PgsViewBatch), c_void_p, c_int32, c_int32, c_void_p, c_void_p,
                                        c_void_p, c_void_p]),
    "pgs_bin_sort_views": (c_int32, [POINTER(PgsViewBatch), c_int32, c_void_p, c_void_p, c_void_p, c_uint32,
                                     c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t,
                                     c_void_p]),
    "pgs_render_fwd_views": (c_int32, [POINTER(PgsViewBatch), c_void_p, c_int32, c_void_p, c_void_p,
                                       POINTER(c_float), c_void_p, c_void_p, c_void_p, POINTER(PgsReplay),
                                       c_void_p, c_void_p, c_void_p, c_void_p]),
    "pgs_render_bwd_views": (c_int32, [POINTER(PgsViewBatch), c_void_p, c_int32, c_void_p, c_void_p,
                                       POINTER(c_float), c_void_p, c_void_p, POINTER(PgsReplay), c_void_p,
                                       c_void_p, c_void_p, c_void_p, c_void_p]),
    "pgs_adam_step_dev": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_int32, POINTER(c_float),
                                    c_void_p, c_float, c_float, c_float, c_void_p]),
    "pgs_mlp_weight_count": (c_int32, []),
    "pgs_mlp_features": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_int32, c_float, c_void_p,
                                   c_void_p, c_void_p]),
    "pgs_mlp_forward": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_void_p]),
    "pgs_mlp_backward_workspace": (c_size_t, [c_int32]),
    "pgs_mlp_backward": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_size_t,
                                   c_void_p]),
    "pgs_seed_targets": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p]),
    "pgs_seed_loss_workspace": (c_size_t, [c_int32]),
    "pgs_seed_loss": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_float, c_void_p, c_void_p,
                                c_void_p, c_size_t, c_void_p]),
    "pgs_seed_apply": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_void_p,
                                 c_void_p]),
    "pgs_stream_copy": (c_int32, [c_void_p, c_void_p, c_size_t, c_void_p]),
    "pgs_atomic_scatter": (c_int32, [c_void_p, c_uint32, c_void_p, c_uint32, c_void_p]),
    "pgs_ba_workspace": (c_size_t, [c_int32, c_int32, c_int32]),
    "pgs_ba_cost": (c_int32, [POINTER(PgsBaProblem), c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t,
                              c_void_p]),
    "pgs_ba_step": (c_int32, [POINTER(PgsBaProblem), c_void_p, c_void_p, c_void_p, c_double, c_void_p, c_void_p,
                              c_void_p, c_size_t, c_void_p]),
    "pgs_ba_apply": (c_int32, [c_int32, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                               c_void_p, c_void_p, c_void_p]),
    "pgs_ba_refine": (c_int32, [POINTER(PgsBaProblem), c_void_p, c_void_p, c_double, c_double, c_void_p, c_void_p,
                                c_void_p, c_void_p]),
    "pgs_ba_compact_workspace": (c_size_t, [c_int32, c_int32]),
    "pgs_ba_compact": (c_int32, [POINTER(PgsBaProblem), c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                 c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "pgs_mvs_census": (c_int32, [c_void_p, c_int32, c_int32, c_int32, c_void_p, c_void_p]),
    "pgs_mvs_range_workspace": (c_size_t, [c_int32, c_int32]),
    "pgs_mvs_depth_range": (c_int32, [c_void_p, c_int32, c_int32, c_int32, c_void_p, c_int32, c_void_p, c_void_p,
                                      c_size_t, c_void_p]),
    "pgs_mvs_select_ref": (c_int32, [c_void_p, c_int32, POINTER(PgsMvsParams), c_void_p, c_void_p]),
    "pgs_mvs_cost": (c_int32, [c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_int32, c_void_p, c_void_p,
                               POINTER(PgsMvsParams), c_void_p, c_void_p]),
    "pgs_mvs_sgm_workspace": (c_size_t, [c_int32, c_int32, c_int32, c_int32]),
    "pgs_mvs_sgm": (c_int32, [c_void_p, c_int32, c_int32, c_void_p, c_int32, c_void_p, POINTER(PgsMvsParams),
                              c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "pgs_mvs_fuse_workspace": (c_size_t, [c_int32, c_int32]),
    "pgs_mvs_fuse": (c_int32, [c_void_p, c_void_p, c_int32, c_int32, c_int32, c_void_p, c_void_p, c_uint32,
                               c_void_p, c_void_p, c_uint32, c_void_p, c_void_p, c_size_t, c_void_p]),
}

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load and type the library once; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run `python -m paper_2601_17354_amd.build`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class PgsError(RuntimeError):
    pass


def check(status: int, what: str) -> None:
    if status != PGS_OK:
        msg = load().pgs_last_error().decode(errors="replace")
        raise PgsError(f"{what} failed with status {status}: {msg}")
