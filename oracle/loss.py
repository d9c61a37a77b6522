"""Photometric losses and their image gradients (oracle).

PocketGS does not state its loss.  The reading used for the training
workloads is the 3D Gaussian Splatting one: (1 - lambda) L1 + lambda (1 - SSIM)
with lambda = 0.2; the small parity workload uses the plain L1.

  L1     mean over 3HW of |x - y|; dL/dx = sign(x - y) / (3HW), sign(0) = 0
  SSIM   Wang et al. (2004) per channel with an 11x11 Gaussian window
         (sigma 1.5, normalised to sum 1), C1 = 0.01^2, C2 = 0.03^2, zero
         padding ("same" size), averaged over pixels and channels:
           mu_x = w * x, sigma_x^2 = w * x^2 - mu_x^2, sigma_xy = w * xy - mu_x mu_y
           S = (2 mu_x mu_y + C1)(2 sigma_xy + C2) /
               ((mu_x^2 + mu_y^2 + C1)(sigma_x^2 + sigma_y^2 + C2))
The SSIM gradient is reverse-mode automatic differentiation of that float64
definition (torch conv2d on the CPU as the windowed-sum step).
Images are (3, H, W).
"""

from __future__ import annotations

import math

import numpy as np
import torch
import torch.nn.functional as F

SSIM_WIN = 11
SSIM_SIGMA = 1.5
C1 = 0.01 ** 2
C2 = 0.03 ** 2
LAMBDA_DSSIM = 0.2


def l1(x, y):
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    N = x.size
    return float(np.abs(x - y).sum() / N), np.sign(x - y) / N


def gaussian_window():
    i = np.arange(SSIM_WIN) - (SSIM_WIN - 1) / 2.0
    g = np.exp(-(i * i) / (2.0 * SSIM_SIGMA ** 2))
    return g / g.sum()


def _ssim_torch(x, y):
    g = torch.as_tensor(gaussian_window())
    w2 = torch.outer(g, g)[None, None].repeat(3, 1, 1, 1)
    pad = SSIM_WIN // 2

    def blur(t):
        return F.conv2d(t[None], w2, padding=pad, groups=3)[0]

    mx, my = blur(x), blur(y)
    sxx = blur(x * x) - mx * mx
    syy = blur(y * y) - my * my
    sxy = blur(x * y) - mx * my
    S = ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2))
    return S


def ssim_map(x, y) -> np.ndarray:
    with torch.no_grad():
        return _ssim_torch(torch.as_tensor(np.asarray(x, np.float64)),
                           torch.as_tensor(np.asarray(y, np.float64))).numpy()


def ssim(x, y):
    """(SSIM value, dSSIM/dx (3,H,W))."""
    xt = torch.as_tensor(np.asarray(x, np.float64)).clone().requires_grad_(True)
    yt = torch.as_tensor(np.asarray(y, np.float64))
    s = _ssim_torch(xt, yt).mean()
    s.backward()
    return float(s.detach()), xt.grad.numpy()


def l1_dssim(x, y, lam=LAMBDA_DSSIM):
    """(loss, dL/dx) for (1 - lam) L1 + lam (1 - SSIM)."""
    lv, lg = l1(x, y)
    sv, sg = ssim(x, y)
    return (1.0 - lam) * lv + lam * (1.0 - sv), (1.0 - lam) * lg - lam * sg


def psnr(x, y) -> float:
    """10 log10(1 / MSE) over 3HW with both images clamped to [0, 1]."""
    x = np.clip(np.asarray(x, np.float64), 0, 1)
    y = np.clip(np.asarray(y, np.float64), 0, 1)
    mse = float(((x - y) ** 2).mean())
    return math.inf if mse == 0 else 10.0 * math.log10(1.0 / mse)
