"""EWA projection of 3D Gaussians (oracle, torch float64 on the CPU).

PocketGS renders "depth-sorted visible Gaussians" (Sec. "Explicit
Computation Graph") and inherits how they get to the screen from 3D Gaussian
Splatting without restating it.  The reading taken here, with its constants:

  camera point     x_c = R mu + t; visible only if z_c > 0.2 (near plane)
  3D covariance    Sigma = M M^T, M = R(q/|q|) diag(exp(s))
  local affine     J = [[fx/z, 0, -fx tx/z], [0, fy/z, -fy ty/z]] with
                   tx = clamp(x/z, +-1.3 W/(2 fx)), ty likewise (H, fy)
  2D covariance    Sigma2D = (J R) Sigma (J R)^T + 0.3 I  (low-pass dilation,
                   no opacity compensation); det <= 0 culls
  conic            Q = Sigma2D^-1 = (A, B, C) for [[A, B], [B, C]]
  mean             u = fx x/z + cx, v = fy y/z + cy (pixel (i, j) has its
                   centre at (i + 1/2, j + 1/2))
  radius           r = ceil(3 sqrt(lambda_max)),
                   lambda_max = m + sqrt(max(0.1, m^2 - det)), m = (a + c)/2
  tile rectangle   x0 = max(0, floor((u - r)/TW)), x1 = min(TX-1, floor((u + r)/TW)),
                   same for y; empty rectangle culls
  colour           c = max(0, sum_k f_k Y_k(d) + 1/2), d = unit(mu - camera centre)
  opacity          o = sigmoid(logit)

`project` returns the differentiable per-Gaussian outputs (u, v, A, B, C, o,
r, g, b) as torch float64 tensors, plus the integer decisions as numpy
arrays and, for each decision, its distance to the threshold.
"""

from __future__ import annotations

import math

import numpy as np
import torch

from .sh import sh_basis

NEAR = 0.2
DILATION = 0.3
CLAMP = 1.3
RADIUS_SIGMAS = 3.0
EIG_FLOOR = 0.1

OUT_FIELDS = ("u", "v", "A", "B", "C", "o", "r", "g", "b")


def sh_degree_of(F: int) -> int:
    K = (F - 11) // 3
    d = int(round(math.sqrt(K))) - 1
    assert 11 + 3 * (d + 1) ** 2 == F, F
    return d


def quat_to_rot(q: torch.Tensor) -> torch.Tensor:
    """Rotation matrix of unit quaternions (w, x, y, z), (n,4) -> (n,3,3)."""
    w, x, y, z = q.unbind(1)
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], 1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], 1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], 1),
    ], 1)


def camera_tensors(cam: dict):
    vm = torch.as_tensor(np.asarray(cam["viewmat"], np.float64))
    return vm[:, :3], vm[:, 3]


def project_params(params: torch.Tensor, cam: dict):
    """Differentiable part: params (F, n) float64 -> dict of (n,) tensors.

    Also returns the intermediates needed for the decisions: z, Sigma2D
    entries (a, b, c) and the clamp masks.
    """
    F, n = params.shape
    D = sh_degree_of(F)
    K = (D + 1) ** 2
    R_c, t_c = camera_tensors(cam)
    fx, fy, cx, cy = (float(cam[k]) for k in ("fx", "fy", "cx", "cy"))
    W, H = int(cam["width"]), int(cam["height"])

    mu = params[0:3].T
    log_s = params[3:6].T
    q = params[6:10].T
    logit = params[10]
    sh = params[11:].T.reshape(n, K, 3)

    xc = mu @ R_c.T + t_c
    x, y, z = xc.unbind(1)

    qn = q / torch.linalg.norm(q, dim=1, keepdim=True)
    Rg = quat_to_rot(qn)
    M = Rg * torch.exp(log_s)[:, None, :]
    Sigma = M @ M.transpose(1, 2)

    lim_x = CLAMP * W / (2.0 * fx)
    lim_y = CLAMP * H / (2.0 * fy)
    tx = torch.clamp(x / z, -lim_x, lim_x)
    ty = torch.clamp(y / z, -lim_y, lim_y)
    zero = torch.zeros_like(z)
    J = torch.stack([
        torch.stack([fx / z, zero, -fx * tx / z], 1),
        torch.stack([zero, fy / z, -fy * ty / z], 1),
    ], 1)
    T = J @ R_c
    S2 = T @ Sigma @ T.transpose(1, 2)
    a = S2[:, 0, 0] + DILATION
    b = 0.5 * (S2[:, 0, 1] + S2[:, 1, 0])
    c = S2[:, 1, 1] + DILATION
    det = a * c - b * b
    A = c / det
    B = -b / det
    C = a / det

    u = fx * x / z + cx
    v = fy * y / z + cy

    R_np = R_c
    centre = -(R_np.T @ t_c)
    d = mu - centre
    d = d / torch.linalg.norm(d, dim=1, keepdim=True)
    Y = sh_basis(d, D)                                   # (n, K)
    raw = (Y[:, :, None] * sh).sum(1) + 0.5              # (n, 3)
    rgb = torch.clamp(raw, min=0.0)
    o = torch.sigmoid(logit)

    out = dict(u=u, v=v, A=A, B=B, C=C, o=o, r=rgb[:, 0], g=rgb[:, 1], b=rgb[:, 2])
    aux = dict(z=z, a=a, b=b, c=c, det=det, raw_rgb=raw, x_over_z=x / z,
               y_over_z=y / z, lim_x=lim_x, lim_y=lim_y)
    return out, aux


def _frac_margin(v: np.ndarray) -> np.ndarray:
    """Distance of v to the nearest integer, relative to max(1, |v|)."""
    return np.abs(v - np.round(v)) / np.maximum(1.0, np.abs(v))


def project(params, cam: dict, tile_w=16, tile_h=16, with_grad=False):
    """Full projection of one view.

    params: (F, n) array-like (float32 input converts exactly to float64).
    Returns dict with float64 numpy arrays for every OUT_FIELDS entry, `z`,
    `depth32` (float32 depth used in the key), `radius` (int64, 0 if culled),
    `rect` (n,4) = (x0, y0, x1, y1) inclusive tile bounds, `tiles_touched`,
    `visible`, `marginal` (bool: some decision within 1e-9 relative of its
    threshold) and, if with_grad, the torch tensors and params leaf.
    """
    P = torch.as_tensor(np.array(params, np.float64))
    if with_grad:
        P = P.clone().requires_grad_(True)
    out, aux = project_params(P, cam)
    W, H = int(cam["width"]), int(cam["height"])
    TX = (W + tile_w - 1) // tile_w
    TY = (H + tile_h - 1) // tile_h

    z = aux["z"].detach().numpy()
    a = aux["a"].detach().numpy()
    c = aux["c"].detach().numpy()
    det = aux["det"].detach().numpy()
    u = out["u"].detach().numpy()
    v = out["v"].detach().numpy()
    n = z.shape[0]
    eps = 1e-9

    in_front = z > NEAR
    pos_det = det > 0.0
    marginal = (np.abs(z - NEAR) <= eps * max(NEAR, 1.0)) | (np.abs(det) <= eps * np.abs(a * c))

    with np.errstate(invalid="ignore", divide="ignore"):
        mid = 0.5 * (a + c)
        lam = mid + np.sqrt(np.maximum(EIG_FLOOR, mid * mid - det))
        rf = RADIUS_SIGMAS * np.sqrt(lam)
        radius = np.ceil(rf)
        marginal |= (_frac_margin(rf) <= eps)

        lo_x = (u - radius) / tile_w
        hi_x = (u + radius) / tile_w
        lo_y = (v - radius) / tile_h
        hi_y = (v + radius) / tile_h
        for q in (lo_x, hi_x, lo_y, hi_y):
            marginal |= (_frac_margin(q) <= eps)
        x0 = np.clip(np.floor(lo_x), 0, TX)
        x1 = np.clip(np.floor(hi_x), -1, TX - 1)
        y0 = np.clip(np.floor(lo_y), 0, TY)
        y1 = np.clip(np.floor(hi_y), -1, TY - 1)

    ok = in_front & pos_det & np.isfinite(u) & np.isfinite(v)
    ok &= (x0 <= x1) & (y0 <= y1)
    radius = np.where(ok, radius, 0).astype(np.int64)
    rect = np.stack([x0, y0, x1, y1], 1)
    rect = np.where(ok[:, None], rect, 0).astype(np.int64)
    touched = np.where(ok, (rect[:, 2] - rect[:, 0] + 1) * (rect[:, 3] - rect[:, 1] + 1), 0)

    raw = aux["raw_rgb"].detach().numpy()
    xz = aux["x_over_z"].detach().numpy()
    yz = aux["y_over_z"].detach().numpy()
    colour_clamped = raw < 0.0
    clamp_xy = np.stack([np.abs(xz) > aux["lim_x"], np.abs(yz) > aux["lim_y"]], 1)
    marginal |= (np.abs(raw) <= eps).any(1)
    marginal |= np.abs(np.abs(xz) - aux["lim_x"]) <= eps * aux["lim_x"]
    marginal |= np.abs(np.abs(yz) - aux["lim_y"]) <= eps * aux["lim_y"]

    res = {k: out[k].detach().numpy() for k in OUT_FIELDS}
    res.update(z=z, depth32=z.astype(np.float32), radius=radius, rect=rect,
               tiles_touched=touched.astype(np.int64), visible=ok,
               colour_clamped=colour_clamped & ok[:, None], clamp_xy=clamp_xy & ok[:, None],
               marginal=marginal & ok, tiles=(TX, TY), n=n)
    if with_grad:
        res["torch_out"] = out
        res["params_leaf"] = P
        res["aux"] = aux
    return res


def project_vjp(params, cam: dict, grad2d: np.ndarray, visible: np.ndarray) -> np.ndarray:
    """Gradient of sum(grad2d * (u, v, A, B, C, o, r, g, b)) with respect to
    the canonical parameters (F, n), for the visible Gaussians only.

    This is the exact derivative of the projection above with the discrete
    decisions (culling, clamps) frozen, obtained by reverse-mode automatic
    differentiation of the float64 definition.
    """
    P = np.array(params, np.float64)
    idx = np.nonzero(visible)[0]
    G = np.zeros_like(P)
    if idx.size == 0:
        return G
    sub = torch.as_tensor(P[:, idx]).clone().requires_grad_(True)
    out, _ = project_params(sub, cam)
    g = torch.as_tensor(np.asarray(grad2d, np.float64)[:, idx])
    s = sum((out[k] * g[i]).sum() for i, k in enumerate(OUT_FIELDS))
    s.backward()
    G[:, idx] = sub.grad.numpy()
    return G
