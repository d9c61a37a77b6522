"""Training step of the operator T and PCA seeding of I, through the C ABI.

One step (PocketGS Sec. "Hardware-Aligned Differentiable Splatting
Optimization"): project -> bin/sort -> composite (recording the replay trace)
-> loss -> replay backward -> projection backward (index-mapped into the
canonical gradient buffer) -> Adam on the canonical layout.  Every stage is a
libpocketgs kernel; PyTorch holds the buffers and provides the stream.
"""

from __future__ import annotations

import numpy as np
import torch

from . import binding as B
from .raster import Rasterizer, param_rows

BETA1, BETA2, EPS = 0.9, 0.999, 1e-15
R_NORMAL = 0.1


def learning_rates(sh_degree: int, extent: float = 1.0) -> np.ndarray:
    """Per-row Adam learning rates (3D Gaussian Splatting defaults; PocketGS
    names Adam but gives no rates): mean 1.6e-4 * extent, log-scale 5e-3,
    rotation 1e-3, opacity 2.5e-2, SH DC 2.5e-3, higher SH 2.5e-3 / 20."""
    F = param_rows(sh_degree)
    lr = np.zeros(F, np.float32)
    lr[0:3] = 1.6e-4 * extent
    lr[3:6] = 5e-3
    lr[6:10] = 1e-3
    lr[10] = 2.5e-2
    lr[11:14] = 2.5e-3
    lr[14:] = 2.5e-3 / 20.0
    return lr


def seed_pca(points: torch.Tensor, colours: torch.Tensor, r_normal: float = R_NORMAL) -> torch.Tensor:
    """Disc-like seeding from a point cloud: points/colours are [3][m] float32
    device tensors; returns canonical SH-degree-0 parameters [14][m]."""
    m = points.shape[1]
    k = 16
    nbr = torch.empty((k, m), dtype=torch.int32, device=points.device)
    d2 = torch.empty((k, m), dtype=torch.float64, device=points.device)
    ws = torch.empty(B.pgs_knn_workspace(m), dtype=torch.uint8, device=points.device)
    B.pgs_knn(points, m, k, nbr, d2, ws)
    out = torch.empty((14, m), dtype=torch.float32, device=points.device)
    B.pgs_pca_seed(points, colours, m, nbr, d2, k, r_normal, out)
    return out


class Trainer:
    """Canonical parameters, Adam moments and one rasterizer per resolution."""

    def __init__(self, params: torch.Tensor, sh_degree: int, width: int, height: int,
                 cached: bool = True, lam: float = 0.2, extent: float = 1.0,
                 tile=(16, 16), ordered: bool = True, trace_words: int | None = None,
                 device_step_counter: bool = False):
        self.params = params.contiguous()
        self.sh_degree = sh_degree
        self.F, self.n = self.params.shape
        dev = self.params.device
        self.grads = torch.zeros_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.lr = learning_rates(sh_degree, extent)
        self.lam = lam
        self.W, self.H = width, height
        kw = {} if trace_words is None else {"trace_words": trace_words}
        self.rast = Rasterizer(self.n, sh_degree, width, height, tile=tile, cached=cached, ordered=ordered, **kw)
        self.dl = torch.empty((3, height, width), dtype=torch.float32, device=dev)
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        self.loss_ws = torch.empty(B.pgs_loss_workspace(width, height), dtype=torch.uint8, device=dev)
        self.step_count = 0
        # Adam's step counter on the device (pgs_adam_step_dev), so that a
        # step recorded as a graph advances it on every replay
        self.adam_state = torch.zeros(4, dtype=torch.int32, device=dev) if device_step_counter else None
        self.events = None

    def prepare(self, cam: dict, bg=(0.0, 0.0, 0.0)):
        """Grow the pair capacity and trace depth until a forward fits
        (synchronises; call before timing)."""
        self.rast.forward_checked(self.params, cam, bg)

    def _mark(self, name):
        if self.events is not None:
            ev = torch.cuda.Event(enable_timing=True)
            ev.record()
            self.events.append((name, ev))

    def step(self, cam: dict, target: torch.Tensor, bg=(0.0, 0.0, 0.0), adam: bool = True,
             check: bool = False):
        """One training step.  check=True reads the device flags after the
        forward (one synchronisation) and, on an overflow, grows the buffers
        and redoes the forward before anything is updated."""
        r = self.rast
        n = self.n
        self._mark("start")
        B.pgs_project(self.params, n, self.sh_degree, cam, r.tw, r.th, r.proj, r.radius, r.rect, r.touched)
        self._mark("project")
        r.bin_sort()
        self._mark("bin_sort")
        B.pgs_render_fwd(r.W, r.H, r.tw, r.th, r.proj, n, r.values, r.ranges, 0, bg, r.image, r.t_final,
                         r.n_contrib, r.trace if r.cached else None, r.flags, r.fwd_order)
        self._mark("render_fwd")
        r.log_work("render_fwd")
        if check and r.read_flags():
            r.forward_checked(self.params, cam, bg)
        B.pgs_loss_l1_dssim(r.image, target, r.W, r.H, self.lam, self.loss, self.dl, self.loss_ws)
        self._mark("loss")
        self.grads.zero_()
        r.grad2d.zero_()
        self._mark("zero")
        B.pgs_render_bwd(r.W, r.H, r.tw, r.th, r.proj, n, r.values, r.ranges, 0, bg, r.t_final,
                         r.n_contrib, r.trace if r.cached else None, self.dl, r.grad2d, r.tile_order)
        self._mark("render_bwd")
        r.log_work("render_bwd")
        B.pgs_project_bwd(self.params, n, self.sh_degree, cam, r.radius, r.grad2d, self.grads)
        self._mark("project_bwd")
        if adam:
            if self.adam_state is not None:
                B.pgs_adam_step_dev(self.params, self.grads, self.m, self.v, self.F, n, self.lr, self.adam_state,
                                    BETA1, BETA2, EPS)
            else:
                self.step_count += 1
                B.pgs_adam_step(self.params, self.grads, self.m, self.v, self.F, n, self.lr, self.step_count,
                                BETA1, BETA2, EPS)
            self._mark("adam")
        return self.loss


class Evaluator:
    """PSNR of rendered views against targets (evaluation row of the method's
    experiments), through pgs_render_fwd and pgs_psnr."""

    def __init__(self, n: int, sh_degree: int, width: int, height: int, device="cuda"):
        self.rast = Rasterizer(n, sh_degree, width, height, cached=False, device=device)
        self.out = torch.zeros(2, dtype=torch.float32, device=device)
        self.ws = torch.empty(B.pgs_loss_workspace(width, height), dtype=torch.uint8, device=device)

    def psnr(self, params: torch.Tensor, cam: dict, target: torch.Tensor, bg=(0.0, 0.0, 0.0)) -> float:
        self.rast.forward_checked(params, cam, bg)
        B.pgs_psnr(self.rast.image, target, self.rast.W, self.rast.H, self.out, self.ws)
        return float(self.out[1].item())

    def mean_psnr(self, params, cams, targets, ids, bg=(0.0, 0.0, 0.0)) -> float:
        return float(np.mean([self.psnr(params, cams[i], targets[i], bg) for i in ids]))


def train(trainer: Trainer, cams, targets, order, iters: int, eval_ids=(), eval_at=(),
          bg=(0.0, 0.0, 0.0), log=None):
    """Runs `iters` steps cycling the training views in `order` (checking the
    overflow flags every step) and returns {iteration: mean held-out PSNR}
    for every iteration listed in eval_at (0 = before training)."""
    ev = Evaluator(trainer.n, trainer.sh_degree, trainer.W, trainer.H, device=trainer.params.device)
    hist = {}
    if 0 in eval_at:
        hist[0] = ev.mean_psnr(trainer.params, cams, targets, eval_ids, bg)
    for it in range(1, iters + 1):
        cid = order[(it - 1) % len(order)]
        trainer.step(cams[cid], targets[cid], bg, check=True)
        if it in eval_at:
            hist[it] = ev.mean_psnr(trainer.params, cams, targets, eval_ids, bg)
            if log:
                log(f"iter {it}: held-out PSNR {hist[it]:.3f} dB, loss {float(trainer.loss.item()):.5f}")
    return hist
