"""Robust bundle adjustment on the GPU (binding and Levenberg-Marquardt loop).

The paper refines the tracking poses and sparse points by a global bundle
adjustment (subsection "GPU-Native Global BA as Mobile MAP Refinement"):
Huber-robustified reprojection error, scale-aware gauge fixing, and the
normal equations solved through the reduced camera system.  Every step runs
in libpocketgs (pgs_ba_cost / pgs_ba_step / pgs_ba_apply); this module
builds the problem's index arrays on the host, holds the device buffers and
runs the damping schedule: lambda / 10 after a step that lowers the cost,
lambda * 10 (state kept) after one that does not.
"""

from __future__ import annotations

import ctypes
import math

import numpy as np
import torch

from . import _lib
from ._lib import PgsBaProblem, check

F64 = torch.float64


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class BAProblem:
    """Observations (ordered by point) and intrinsics, resident on the GPU."""

    def __init__(self, n_cams, obs_cam, obs_pt, obs_uv, fx, fy, cx, cy, gauge_axis, huber_delta=2.0,
                 device="cuda"):
        obs_cam = np.asarray(obs_cam, np.uint32)
        obs_pt = np.asarray(obs_pt, np.uint32)
        if obs_pt.size and np.any(np.diff(obs_pt.astype(np.int64)) < 0):
            raise ValueError("observations must be ordered by point")
        n_points = int(obs_pt.max()) + 1 if obs_pt.size else 0
        point_start = np.searchsorted(obs_pt, np.arange(n_points + 1)).astype(np.uint32)
        cam_obs = np.argsort(obs_cam, kind="stable").astype(np.uint32)
        cam_start = np.searchsorted(obs_cam[cam_obs], np.arange(n_cams + 1)).astype(np.uint32)
        d = torch.device(device)
        u32 = lambda a: torch.as_tensor(a.astype(np.int32), device=d)  # noqa: E731
        arrays = [u32(obs_cam), u32(obs_pt), torch.as_tensor(np.asarray(obs_uv, np.float64), device=d),
                  u32(point_start), u32(cam_obs), u32(cam_start)]
        self._finish(int(n_cams), n_points, int(obs_cam.size), arrays, (fx, fy, cx, cy), gauge_axis, huber_delta, d)

    def _finish(self, n_cams, n_points, n_obs, arrays, intrinsics, gauge_axis, huber_delta, d):
        self.n_cams, self.n_points, self.n_obs = n_cams, n_points, n_obs
        self.intrinsics, self.gauge_axis, self.huber_delta = tuple(float(v) for v in intrinsics), int(gauge_axis), \
            float(huber_delta)
        self._keep = arrays
        k = arrays
        fx, fy, cx, cy = self.intrinsics
        self.struct = PgsBaProblem(n_cams, n_points, n_obs, self.gauge_axis, fx, fy, cx, cy, self.huber_delta,
                                   _p(k[0]), _p(k[1]), _p(k[2]), _p(k[3]), _p(k[4]), _p(k[5]))
        ws = _lib.load().pgs_ba_workspace(n_cams, n_points, n_obs)
        self.workspace = torch.empty(ws, dtype=torch.uint8, device=d)
        self.device = d

    def arrays(self):
        """(obs_cam, obs_pt, obs_uv, point_start, cam_obs, cam_start) on the device."""
        return tuple(self._keep)

    @classmethod
    def from_tracks(cls, tr, huber_delta=2.0, device="cuda"):
        return cls(tr["R0"].shape[0], tr["obs_cam"], tr["obs_pt"], tr["obs_uv"], tr["fx"], tr["fy"], tr["cx"],
                   tr["cy"], tr["gauge_axis"], huber_delta, device)


def state(R, c, P, device="cuda"):
    """Device state (rotations [C][9], centres [C][3], points [M][3]) in float64."""
    d = torch.device(device)
    return (torch.as_tensor(np.ascontiguousarray(R, np.float64).reshape(-1, 9), device=d),
            torch.as_tensor(np.ascontiguousarray(c, np.float64), device=d),
            torch.as_tensor(np.ascontiguousarray(P, np.float64), device=d))


def _check_state(pb, st):
    R, c, P = st
    for t, n, k in ((R, pb.n_cams, 9), (c, pb.n_cams, 3), (P, pb.n_points, 3)):
        if t.dtype != F64 or not t.is_cuda or not t.is_contiguous() or t.numel() != n * k:
            raise ValueError("state arrays must be contiguous float64 on the GPU with the problem's sizes")


def cost(pb: BAProblem, st, out=None):
    _check_state(pb, st)
    out = out if out is not None else torch.empty(1, dtype=F64, device=pb.device)
    check(_lib.load().pgs_ba_cost(ctypes.byref(pb.struct), _p(st[0]), _p(st[1]), _p(st[2]), _p(out),
                                  _p(pb.workspace), pb.workspace.numel(), _stream()), "pgs_ba_cost")
    return out


def step(pb: BAProblem, st, lam, dpose=None, dpoint=None):
    _check_state(pb, st)
    dpose = dpose if dpose is not None else torch.empty((pb.n_cams, 6), dtype=F64, device=pb.device)
    dpoint = dpoint if dpoint is not None else torch.empty((pb.n_points, 3), dtype=F64, device=pb.device)
    check(_lib.load().pgs_ba_step(ctypes.byref(pb.struct), _p(st[0]), _p(st[1]), _p(st[2]), float(lam),
                                  _p(dpose), _p(dpoint), _p(pb.workspace), pb.workspace.numel(), _stream()),
          "pgs_ba_step")
    return dpose, dpoint


def apply(pb: BAProblem, st, dpose, dpoint, out=None):
    _check_state(pb, st)
    out = out if out is not None else tuple(torch.empty_like(t) for t in st)
    check(_lib.load().pgs_ba_apply(pb.n_cams, pb.n_points, _p(st[0]), _p(st[1]), _p(st[2]), _p(dpose),
                                   _p(dpoint), _p(out[0]), _p(out[1]), _p(out[2]), _stream()), "pgs_ba_apply")
    return out


def lm(pb: BAProblem, st, lam=1e-3, iters=10):
    """Levenberg-Marquardt; returns (state, cost history, accept flags)."""
    f = float(cost(pb, st).item())
    hist, acc = [f], []
    for _ in range(iters):
        dpose, dpoint = step(pb, st, lam)
        cand = apply(pb, st, dpose, dpoint)
        f1 = float(cost(pb, cand).item())
        if f1 < hist[-1]:
            st = cand
            hist.append(f1)
            acc.append(True)
            lam /= 10.0
        else:
            hist.append(hist[-1])
            acc.append(False)
            lam *= 10.0
    return st, hist, acc


def refine(pb: BAProblem, st, max_err=4.0, min_angle=math.radians(1.5)):
    """One geometric refinement pass: re-triangulated points and the keep
    masks of points and observations (device tensors)."""
    _check_state(pb, st)
    P = torch.empty((pb.n_points, 3), dtype=F64, device=pb.device)
    kp = torch.empty(pb.n_points, dtype=torch.uint8, device=pb.device)
    ko = torch.empty(pb.n_obs, dtype=torch.uint8, device=pb.device)
    check(_lib.load().pgs_ba_refine(ctypes.byref(pb.struct), _p(st[0]), _p(st[1]), float(max_err),
                                    float(min_angle), _p(P), _p(kp), _p(ko), _stream()), "pgs_ba_refine")
    return P, kp, ko


def compact(pb: BAProblem, keep_pt, keep_obs, points):
    """The problem and points restricted to the kept ones (a new BAProblem
    whose arrays stay on the device; the two new sizes are read back)."""
    d = pb.device
    M, O, C = pb.n_points, pb.n_obs, pb.n_cams
    out = [torch.empty(O, dtype=torch.int32, device=d), torch.empty(O, dtype=torch.int32, device=d),
           torch.empty((O, 2), dtype=F64, device=d), torch.empty(M + 1, dtype=torch.int32, device=d),
           torch.empty(O, dtype=torch.int32, device=d), torch.empty(C + 1, dtype=torch.int32, device=d)]
    pts = torch.empty((M, 3), dtype=F64, device=d)
    counts = torch.zeros(2, dtype=torch.int32, device=d)
    lib = _lib.load()
    ws = torch.empty(lib.pgs_ba_compact_workspace(M, O), dtype=torch.uint8, device=d)
    check(lib.pgs_ba_compact(ctypes.byref(pb.struct), _p(keep_pt), _p(keep_obs), _p(points), *(_p(t) for t in out),
                             _p(pts), _p(counts), _p(ws), ws.numel(), _stream()), "pgs_ba_compact")
    m, o = (int(v) for v in counts.cpu())
    if m < 1 or o < 1:
        raise ValueError("refinement kept no point")
    arrays = [out[0][:o], out[1][:o], out[2][:o], out[3][:m + 1], out[4][:o], out[5]]
    q = BAProblem.__new__(BAProblem)
    q._finish(C, m, o, arrays, pb.intrinsics, pb.gauge_axis, pb.huber_delta, d)
    return q, pts[:m].contiguous()


def refine_loop(pb: BAProblem, st, rounds=3, lm_iters=5, lam=1e-3, max_err=4.0, min_angle=math.radians(1.5)):
    """Bundle adjustment embedded in the refinement loop: per round a few
    Levenberg-Marquardt iterations, then re-triangulation, filtering and
    compaction.  Returns the final problem, state and per-round counts."""
    log = []
    for _ in range(rounds):
        st, hist, _ = lm(pb, st, lam=lam, iters=lm_iters)
        P, kp, ko = refine(pb, st, max_err, min_angle)
        pb2, P2 = compact(pb, kp, ko, P)
        log.append(dict(points=pb.n_points, obs=pb.n_obs, kept_points=pb2.n_points, kept_obs=pb2.n_obs,
                        cost=hist[-1]))
        pb, st = pb2, (st[0], st[1], P2)
    return pb, st, log
