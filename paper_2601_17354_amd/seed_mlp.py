"""Learned seeding: the network that corrects the plain disc-like seed
(PocketGS Sec. "Disc-Like Covariance Seeding") from a point's neighbourhood,
its training step, and seeding with the plain seed as the fall back.

Every step runs in libpocketgs kernels (pgs_knn, pgs_mlp_features,
pgs_mlp_forward / pgs_mlp_backward on bfloat16 matrix cores, pgs_seed_loss,
pgs_adam_step, pgs_seed_apply); this module owns buffers and the schedule.
"""

from __future__ import annotations

import math
import os

import numpy as np
import torch

from . import binding as B
from .train import R_NORMAL

N_WEIGHTS = 13000
K_NN = 16
WEIGHTS_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "seed_mlp.npy")
_SHAPES = [(64, 64), (64,), (64, 64), (64,), (64, 64), (64,), (8, 64), (8,)]


def init_weights(seed: int = 0) -> np.ndarray:
    """He-normal hidden layers, zero biases, zero output layer with output
    bias (0,0,0,1,0,0,0,0): the untrained network reproduces the plain seed."""
    rng = np.random.default_rng(seed)
    parts = []
    for s in _SHAPES:
        if len(s) == 2 and s[0] == 64:
            parts.append(rng.normal(size=s) * math.sqrt(2.0 / s[1]))
        else:
            parts.append(np.zeros(s))
    parts[7][3] = 1.0
    w = np.concatenate([p.reshape(-1) for p in parts]).astype(np.float32)
    assert w.size == N_WEIGHTS
    return w


def load_weights(path: str = WEIGHTS_PATH, device="cuda") -> torch.Tensor:
    w = np.load(path, allow_pickle=False).astype(np.float32)
    if w.size != N_WEIGHTS:
        raise ValueError(f"{path}: expected {N_WEIGHTS} weights, found {w.size}")
    return torch.as_tensor(w, device=device)


def neighbourhoods(points: torch.Tensor):
    """Exact 16 nearest neighbours of every point of a [3][m] cloud."""
    m = points.shape[1]
    nbr = torch.empty((K_NN, m), dtype=torch.int32, device=points.device)
    d2 = torch.empty((K_NN, m), dtype=torch.float64, device=points.device)
    ws = torch.empty(B.pgs_knn_workspace(m), dtype=torch.uint8, device=points.device)
    B.pgs_knn(points, m, K_NN, nbr, d2, ws)
    return nbr, d2


def features(points: torch.Tensor, nbr, d2, r_normal: float = R_NORMAL):
    m = points.shape[1]
    x = torch.empty((m, 64), dtype=torch.float32, device=points.device)
    base = torch.empty((m, 16), dtype=torch.float32, device=points.device)
    B.pgs_mlp_features(points, m, nbr, d2, K_NN, r_normal, x, base)
    return x, base


def forward(weights: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
    y = torch.empty((x.shape[0], 8), dtype=torch.float32, device=x.device)
    B.pgs_mlp_forward(weights, x, x.shape[0], y)
    return y


def seed_learned(points: torch.Tensor, colours: torch.Tensor, weights: torch.Tensor,
                 r_normal: float = R_NORMAL):
    """Canonical SH-degree-0 parameters [14][m] from the network, falling
    back to the plain seed per point; returns (params, fallback count)."""
    m = points.shape[1]
    nbr, d2 = neighbourhoods(points)
    pca = torch.empty((14, m), dtype=torch.float32, device=points.device)
    B.pgs_pca_seed(points, colours, m, nbr, d2, K_NN, r_normal, pca)
    x, base = features(points, nbr, d2, r_normal)
    y = forward(weights, x)
    count = torch.zeros(1, dtype=torch.int32, device=points.device)
    B.pgs_seed_apply(y, base, pca, m, pca, None, count)
    return pca, int(count.item())


def seed_constant_offset(points: torch.Tensor, colours: torch.Tensor, weights: torch.Tensor,
                         r_normal: float = R_NORMAL):
    """Control for the learned seed: the plain seed with the network's mean
    output over the cloud applied to every point as one constant offset
    (the same log-scale offsets, local rotation and logit offset for all),
    which is what a network reduced to its output bias could learn; returns
    (params, fallback count, the mean output)."""
    m = points.shape[1]
    nbr, d2 = neighbourhoods(points)
    pca = torch.empty((14, m), dtype=torch.float32, device=points.device)
    B.pgs_pca_seed(points, colours, m, nbr, d2, K_NN, r_normal, pca)
    x, base = features(points, nbr, d2, r_normal)
    y = forward(weights, x)
    ybar = y.mean(0, dtype=torch.float64).to(torch.float32)
    yc = ybar.expand(m, 8).contiguous()
    count = torch.zeros(1, dtype=torch.int32, device=points.device)
    B.pgs_seed_apply(yc, base, pca, m, pca, None, count)
    return pca, int(count.item()), ybar.cpu().numpy().tolist()


class SeedNetTrainer:
    """Adam on the network weights with the seed loss (mean over a batch)."""

    def __init__(self, weights: torch.Tensor, lr: float = 1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                 max_rows: int = 65536):
        self.w = weights.contiguous().clone()
        dev = self.w.device
        self.g = torch.zeros_like(self.w)
        self.m = torch.zeros_like(self.w)
        self.v = torch.zeros_like(self.w)
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.step_count = 0
        self.max_rows = max_rows
        self.y = torch.empty((max_rows, 8), dtype=torch.float32, device=dev)
        self.dy = torch.empty((max_rows, 8), dtype=torch.float32, device=dev)
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        self.ws_b = torch.empty(B.pgs_mlp_backward_workspace(max_rows), dtype=torch.uint8, device=dev)
        self.ws_l = torch.empty(max(8, B.pgs_seed_loss_workspace(max_rows)), dtype=torch.uint8, device=dev)

    def loss_and_grad(self, x, base, target):
        m = x.shape[0]
        if m > self.max_rows:
            raise ValueError(f"batch of {m} rows exceeds {self.max_rows}")
        y, dy = self.y[:m], self.dy[:m]
        B.pgs_mlp_forward(self.w, x, m, y)
        B.pgs_seed_loss(y, base, target, m, 1.0 / m, self.loss, dy, self.ws_l)
        B.pgs_mlp_backward(self.w, x, m, dy, self.g, self.ws_b)
        return self.loss

    def step(self, x, base, target, lr=None):
        loss = self.loss_and_grad(x, base, target)
        self.step_count += 1
        B.pgs_adam_step(self.w.view(1, -1), self.g.view(1, -1), self.m.view(1, -1), self.v.view(1, -1), 1,
                        N_WEIGHTS, [self.lr if lr is None else lr], self.step_count, self.b1, self.b2, self.eps)
        return loss

    def evaluate(self, x, base, target, chunk=65536):
        """Mean seed loss over all rows (no gradient)."""
        total = 0.0
        chunk = min(chunk, self.max_rows)
        for s in range(0, x.shape[0], chunk):
            e = min(x.shape[0], s + chunk)
            y = self.y[:e - s]
            B.pgs_mlp_forward(self.w, x[s:e], e - s, y)
            B.pgs_seed_loss(y, base[s:e], target[s:e], e - s, 1.0, self.loss, None, self.ws_l)
            total += float(self.loss.item())
        return total / x.shape[0]
