"""torch.autograd wrappers over the C ABI.

`rasterize(params, rast, cam, bg)` renders one view with a `Rasterizer` and
returns the image as a differentiable function of the canonical parameters:
forward = projection, binning/sort and compositing (with the replay trace
when the rasterizer is in cached mode); backward = the trace replay (or
recompute-T) backward, the index-mapped scatter and the projection backward
(PocketGS Sec. "Hardware-Aligned Differentiable Splatting Optimization").
`photometric_loss(image, target, lam)` is (1 - lam) L1 + lam (1 - SSIM).

A Rasterizer keeps one view's forward state, so each Rasterizer may have one
forward awaiting its backward at a time.
"""

from __future__ import annotations

import torch

from . import binding as B
from .raster import Rasterizer


class RasterizeFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params: torch.Tensor, rast: Rasterizer, cam: dict, bg=(0.0, 0.0, 0.0)):
        params = params.contiguous()
        rast.forward_checked(params, cam, bg)
        ctx.rast, ctx.cam, ctx.bg = rast, cam, bg
        ctx.save_for_backward(params)
        return rast.image.clone()

    @staticmethod
    def backward(ctx, grad_image: torch.Tensor):
        (params,) = ctx.saved_tensors
        grads = torch.zeros_like(params)
        ctx.rast.backward(params, ctx.cam, grad_image.contiguous(), grads, ctx.bg)
        return grads, None, None, None


def rasterize(params, rast: Rasterizer, cam: dict, bg=(0.0, 0.0, 0.0)) -> torch.Tensor:
    return RasterizeFn.apply(params, rast, cam, bg)


class PhotometricLossFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, image: torch.Tensor, target: torch.Tensor, lam: float = 0.2):
        image = image.contiguous()
        _, H, W = image.shape
        loss = torch.zeros(1, dtype=torch.float32, device=image.device)
        dl = torch.empty_like(image)
        ws = torch.empty(B.pgs_loss_workspace(W, H), dtype=torch.uint8, device=image.device)
        B.pgs_loss_l1_dssim(image, target.contiguous(), W, H, lam, loss, dl, ws)
        ctx.save_for_backward(dl)
        return loss[0]

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        (dl,) = ctx.saved_tensors
        return dl * g, None, None


def photometric_loss(image, target, lam: float = 0.2) -> torch.Tensor:
    return PhotometricLossFn.apply(image, target, lam)
