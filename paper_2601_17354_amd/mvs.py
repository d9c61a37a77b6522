"""Single-reference cost-volume multi-view stereo on the GPU (binding and
pipeline).

The paper densifies the refined sparse scaffold into the cloud P that seeds
the Gaussians (subsection "Single-Reference Cost-Volume MVS"): per target
view a depth range from the projected bundle-adjustment points, one
reference view chosen by the score S_ref, a Census plane-sweep cost volume,
SGM aggregation, the confidence filter at 0.4 and fusion.  Every step runs
in libpocketgs (pgs_mvs_*); the functions below have the entry points' names
and only marshal arguments, and `MVS` sequences them and owns the buffers.
"""

from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import PgsCamera, PgsMvsParams, check


@dataclass
class MVSParams:
    """Hypotheses, penalties and reference-score constants (the paper gives
    only the confidence threshold 0.4; the rest are chosen for 8-bit images,
    48-bit Census costs and the ring captures)."""
    n_planes: int = 128
    p1: int = 4
    p2: int = 32
    conf_min: float = 0.4
    b_target: float = 0.5
    sigma_b: float = 0.25
    alpha_min: float = math.radians(5.0)

    def struct(self) -> PgsMvsParams:
        return PgsMvsParams(int(self.n_planes), int(self.p1), int(self.p2), float(self.conf_min),
                            float(self.b_target), float(self.sigma_b), float(self.alpha_min))


def _p(t, dtype=None):
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def cameras_tensor(cams, device="cuda") -> torch.Tensor:
    """The cameras as a device array of pgs_camera structs."""
    arr = (PgsCamera * len(cams))()
    for i, cam in enumerate(cams):
        c = arr[i]
        c.width, c.height = int(cam["width"]), int(cam["height"])
        c.fx, c.fy, c.cx, c.cy = (float(cam[k]) for k in ("fx", "fy", "cx", "cy"))
        vm = np.asarray(cam["viewmat"], np.float32).reshape(12)
        for k in range(12):
            c.viewmat[k] = float(vm[k])
    raw = np.frombuffer(bytes(arr), np.uint8).copy()
    return torch.as_tensor(raw, device=device)


def pgs_mvs_census(grey, census):
    V, H, W = grey.shape
    assert census.shape == (V, H, W)
    check(_lib.load().pgs_mvs_census(_p(grey, torch.uint8), V, W, H, _p(census, torch.int64), _stream()),
          "pgs_mvs_census")


def pgs_mvs_depth_range(cams_dev, n_views, width, height, points, rng, workspace=None):
    M = points.shape[0]
    lib = _lib.load()
    need = lib.pgs_mvs_range_workspace(n_views, M)
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=points.device)
    assert rng.shape == (n_views, 2)
    check(lib.pgs_mvs_depth_range(_p(cams_dev, torch.uint8), n_views, width, height, _p(points, torch.float64), M,
                                  _p(rng, torch.float64), _p(workspace), workspace.numel(), _stream()),
          "pgs_mvs_depth_range")


def pgs_mvs_select_ref(cams_dev, n_views, params: MVSParams, ref):
    assert ref.shape == (n_views,)
    ps = params.struct()
    check(_lib.load().pgs_mvs_select_ref(_p(cams_dev, torch.uint8), n_views, ctypes.byref(ps),
                                         _p(ref, torch.int32), _stream()), "pgs_mvs_select_ref")


def pgs_mvs_cost(cams_dev, width, height, census, targets, ref, rng, params: MVSParams, cost):
    T = targets.numel()
    assert cost.shape == (T, height, width, params.n_planes) and cost.dtype == torch.uint8
    assert census.shape[1:] == (height, width)
    ps = params.struct()
    check(_lib.load().pgs_mvs_cost(_p(cams_dev, torch.uint8), width, height, _p(census, torch.int64),
                                   _p(targets, torch.int32), T, _p(ref, torch.int32), _p(rng, torch.float64),
                                   ctypes.byref(ps), _p(cost), _stream()), "pgs_mvs_cost")


def pgs_mvs_sgm(cost, targets, rng, params: MVSParams, depth, conf, agg_out=None, workspace=None):
    T, H, W, D = cost.shape
    assert D == params.n_planes and depth.shape == (T, H, W) and conf.shape == (T, H, W)
    lib = _lib.load()
    if agg_out is not None:
        assert agg_out.shape == cost.shape and agg_out.dtype == torch.int16
    need = lib.pgs_mvs_sgm_workspace(T, W, H, D)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=cost.device)
    ws, nbytes = _p(workspace), workspace.numel()
    ps = params.struct()
    check(lib.pgs_mvs_sgm(_p(cost, torch.uint8), W, H, _p(targets, torch.int32), T, _p(rng, torch.float64),
                          ctypes.byref(ps), _p(depth, torch.float32), _p(conf, torch.float32),
                          _p(agg_out) if agg_out is not None else ctypes.c_void_p(0), ws, nbytes, _stream()),
          "pgs_mvs_sgm")


def pgs_mvs_fuse(cams_dev, targets, depth, points, count, workspace=None, grey=None, colours=None, stride=1):
    """points (and colours): [3][capacity] float32; count: one int32."""
    T, H, W = depth.shape
    cap = points.shape[1]
    assert points.shape[0] == 3 and (colours is None or colours.shape == points.shape)
    lib = _lib.load()
    need = lib.pgs_mvs_fuse_workspace(T, H)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=depth.device)
    nul = ctypes.c_void_p(0)
    check(lib.pgs_mvs_fuse(_p(cams_dev, torch.uint8), _p(targets, torch.int32), T, W, H, _p(depth, torch.float32),
                           _p(grey, torch.uint8) if grey is not None else nul, int(stride), _p(points, torch.float32),
                           _p(colours, torch.float32) if colours is not None else nul, cap, _p(count, torch.int32),
                           _p(workspace), workspace.numel(), _stream()), "pgs_mvs_fuse")


class MVS:
    """Depth maps and the fused cloud for a set of views sharing one image
    size.  Buffers are sized for `max_targets` target views per call."""

    def __init__(self, cams, width, height, params: MVSParams | None = None, max_targets=8, device="cuda"):
        self.params = params or MVSParams()
        self.cams = list(cams)
        self.V, self.W, self.H = len(self.cams), int(width), int(height)
        self.device = torch.device(device)
        self.cams_dev = cameras_tensor(self.cams, self.device)
        D = self.params.n_planes
        T = int(max_targets)
        self.T = T
        dev = self.device
        self.census = torch.empty((self.V, self.H, self.W), dtype=torch.int64, device=dev)
        self.range = torch.zeros((self.V, 2), dtype=torch.float64, device=dev)
        self.ref = torch.empty(self.V, dtype=torch.int32, device=dev)
        self.cost = torch.empty((T, self.H, self.W, D), dtype=torch.uint8, device=dev)
        self.depth = torch.empty((T, self.H, self.W), dtype=torch.float32, device=dev)
        self.conf = torch.empty((T, self.H, self.W), dtype=torch.float32, device=dev)
        lib = _lib.load()
        self.sgm_ws = torch.empty(lib.pgs_mvs_sgm_workspace(T, self.W, self.H, D), dtype=torch.uint8, device=dev)
        self.fuse_ws = torch.empty(max(lib.pgs_mvs_fuse_workspace(T, self.H), 1), dtype=torch.uint8, device=dev)
        self.count = torch.zeros(1, dtype=torch.int32, device=dev)

    def prepare(self, grey, sparse_points):
        """Census of every view, depth ranges from the sparse points and the
        reference of every view."""
        assert grey.shape == (self.V, self.H, self.W)
        pgs_mvs_census(grey, self.census)
        pgs_mvs_depth_range(self.cams_dev, self.V, self.W, self.H, sparse_points, self.range)
        pgs_mvs_select_ref(self.cams_dev, self.V, self.params, self.ref)

    def depth_maps(self, targets):
        """Cost volume and SGM for up to max_targets target views (a device
        int32 tensor); depth and confidence land in self.depth[:T]."""
        T = targets.numel()
        assert T <= self.T
        pgs_mvs_cost(self.cams_dev, self.W, self.H, self.census, targets, self.ref, self.range, self.params,
                     self.cost[:T])
        pgs_mvs_sgm(self.cost[:T], targets, self.range, self.params, self.depth[:T], self.conf[:T],
                    workspace=self.sgm_ws)
        return self.depth[:T]

    def fuse(self, targets, points, grey=None, colours=None, stride=1):
        """Kept pixels of the last depth maps back-projected into `points`
        ([3][capacity]; every stride-th kept pixel, with its intensity in
        `colours` when given); returns the device count of kept pixels."""
        T = targets.numel()
        pgs_mvs_fuse(self.cams_dev, targets, self.depth[:T], points, self.count, workspace=self.fuse_ws, grey=grey,
                     colours=colours, stride=stride)
        return self.count
