"""Synthetic workloads built on the GPU path (inputs from `synth`).

Mobile-budget training workload (300k Gaussians at 1920x1440): a seeded
spheres-and-planes scene; ground truth = 500k flat opaque Gaussians on its
surfaces; targets = the ground truth rendered by this library at 60 ring
cameras (every 8th held out); the trained model is seeded by PCA seeding
from a 300k-point noisy cloud of the same scene (different seed).  These
stand in for the paper's captured scenes, which are not available.
"""

from __future__ import annotations

import numpy as np
import torch

import synth

from .raster import Rasterizer
from .train import seed_pca


def render_targets(params: torch.Tensor, sh_degree: int, cams: list, width: int, height: int,
                   bg=(0.0, 0.0, 0.0)) -> list:
    R = Rasterizer(params.shape[1], sh_degree, width, height, cached=False)
    out = []
    for cam in cams:
        R.forward_checked(params, cam, bg)
        out.append(R.image.clone())
    return out


def training_workload(n_train=300_000, n_gt=500_000, width=1920, height=1440, scene_seed=0,
                      n_cams=60, target_cams=None, device="cuda"):
    """Returns dict(params0 [14][n], cams, train_ids, test_ids, targets{idx: image})."""
    dev = torch.device(device)
    scene = synth.spheres_planes_scene(scene_seed)
    gt = synth.surface_gaussians(scene, n_gt, seed=1000 + scene_seed, sh_degree=0, opacity=0.95)
    cams = synth.ring_cameras(n_cams, width, height)
    test_ids = [i for i in range(n_cams) if i % 8 == 0]
    train_ids = [i for i in range(n_cams) if i % 8 != 0]
    want = target_cams if target_cams is not None else list(range(n_cams))
    gt_t = torch.as_tensor(gt, device=dev)
    imgs = render_targets(gt_t, 0, [cams[i] for i in want], width, height)
    targets = dict(zip(want, imgs))
    del gt_t
    pts, col = synth.noisy_cloud(scene, n_train, seed=2000 + scene_seed)
    P = torch.as_tensor(np.ascontiguousarray(pts.T), device=dev)
    C = torch.as_tensor(np.ascontiguousarray(col.T), device=dev)
    params0 = seed_pca(P, C)
    torch.cuda.synchronize()
    return dict(params0=params0, cams=cams, train_ids=train_ids, test_ids=test_ids,
                targets=targets, scene=scene, width=width, height=height, cloud=(P, C))
