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


def scene_views(scene_seed, n_points, n_gt=500_000, width=1920, height=1440, n_cams=60, target_cams=None,
                device="cuda", gt_opacity=0.95):
    """Seeded spheres-and-planes scene: ground truth = n_gt flat Gaussians of
    opacity gt_opacity on its surfaces (seed 1000 + scene_seed), targets =
    the ground truth rendered at n_cams ring cameras (every 8th held out),
    and a noisy n_points cloud of the same surfaces (seed 2000 + scene_seed)."""
    dev = torch.device(device)
    scene = synth.spheres_planes_scene(scene_seed)
    gt = synth.surface_gaussians(scene, n_gt, seed=1000 + scene_seed, sh_degree=0, opacity=gt_opacity)
    cams = synth.ring_cameras(n_cams, width, height)
    test_ids = [i for i in range(n_cams) if i % 8 == 0]
    train_ids = [i for i in range(n_cams) if i % 8 != 0]
    want = target_cams if target_cams is not None else list(range(n_cams))
    gt_t = torch.as_tensor(gt, device=dev)
    imgs = render_targets(gt_t, 0, [cams[i] for i in want], width, height)
    targets = dict(zip(want, imgs))
    del gt_t
    pts, col = synth.noisy_cloud(scene, n_points, seed=2000 + scene_seed)
    P = torch.as_tensor(np.ascontiguousarray(pts.T), device=dev)
    C = torch.as_tensor(np.ascontiguousarray(col.T), device=dev)
    return dict(cams=cams, train_ids=train_ids, test_ids=test_ids, targets=targets, scene=scene,
                width=width, height=height, cloud=(P, C))


def training_workload(n_train=300_000, n_gt=500_000, width=1920, height=1440, scene_seed=0,
                      n_cams=60, target_cams=None, device="cuda"):
    """Returns dict(params0 [14][n], cams, train_ids, test_ids, targets{idx: image})."""
    wl = scene_views(scene_seed, n_train, n_gt, width, height, n_cams, target_cams, device)
    P, C = wl["cloud"]
    wl["params0"] = seed_pca(P, C)
    torch.cuda.synchronize()
    return wl


def compare_inits(weights, scene_seeds=(200, 201, 202), n_points=200_000, n_gt=400_000, width=1024,
                  height=768, iters=500, eval_at=(0, 100, 500), isotropic=True, log=None,
                  gt_opacity=(0.95, 0.95, 0.95)):
    """Held-out PSNR after training from the plain seed, the learned seed
    (network `weights`, plain-seed fall back), the control that applies the
    network's mean output to every point as a constant offset, and, for
    context, an isotropic seed (r_normal = 1), on fresh scenes whose ground
    truth has opacity gt_opacity[i].  Returns per-scene histories, the mean
    over scenes, the learned seed's fall-back counts and the control's
    constant offsets."""
    from .seed_mlp import seed_constant_offset, seed_learned
    from .train import Trainer, train
    rng = np.random.default_rng(0)
    per_scene, fallbacks, offsets = {}, {}, {}
    for s, op in zip(scene_seeds, gt_opacity):
        wl = scene_views(s, n_points, n_gt, width, height, gt_opacity=op)
        P, C = wl["cloud"]
        order = [int(i) for i in rng.permutation(wl["train_ids"])]
        inits = {"plain_pca": seed_pca(P, C)}
        inits["learned"], fallbacks[str(s)] = seed_learned(P, C, weights)
        inits["constant_offset"], _, offsets[str(s)] = seed_constant_offset(P, C, weights)
        if isotropic:
            inits["isotropic"] = seed_pca(P, C, r_normal=1.0)
        res = {}
        for name, p0 in inits.items():
            tr = Trainer(p0.clone(), 0, width, height, cached=True, lam=0.2, extent=4.5)
            hist = train(tr, wl["cams"], wl["targets"], order, iters, eval_ids=wl["test_ids"], eval_at=eval_at)
            res[name] = {str(k): round(v, 3) for k, v in hist.items()}
            del tr
            if log:
                log(f"scene {s} {name}: {res[name]}")
        per_scene[str(s)] = res
        del wl, inits
        torch.cuda.empty_cache()
    names = list(next(iter(per_scene.values())).keys())
    mean = {n: {str(k): round(float(np.mean([per_scene[sc][n][str(k)] for sc in per_scene])), 3)
                for k in eval_at} for n in names}
    return dict(per_scene=per_scene, mean=mean, fallbacks=fallbacks, constant_offsets=offsets,
                gt_opacity=dict(zip([str(x) for x in scene_seeds], gt_opacity)))


def batched_workload(n=1_000_000, sh_degree=3, n_gt=500_000, scene_seed=0, device="cuda"):
    """Eight ring views of uneven resolution (640x480 .. 1920x1440) of the
    spheres-and-planes scene; the trained set = plain seed of an n-point
    noisy cloud with SH coefficients up to sh_degree (higher ones zero);
    targets = the ground truth rendered at each view."""
    from .batch import mixed_views
    from .raster import param_rows
    dev = torch.device(device)
    scene = synth.spheres_planes_scene(scene_seed)
    cams = mixed_views()
    gt = torch.as_tensor(synth.surface_gaussians(scene, n_gt, seed=1000 + scene_seed, sh_degree=0, opacity=0.95),
                         device=dev)
    targets = [render_targets(gt, 0, [c], c["width"], c["height"])[0] for c in cams]
    del gt
    pts, col = synth.noisy_cloud(scene, n, seed=3000 + scene_seed)
    P = torch.as_tensor(np.ascontiguousarray(pts.T), device=dev)
    C = torch.as_tensor(np.ascontiguousarray(col.T), device=dev)
    p14 = seed_pca(P, C)
    params = torch.zeros((param_rows(sh_degree), n), dtype=torch.float32, device=dev)
    params[:14] = p14
    torch.cuda.synchronize()
    return dict(params0=params, cams=cams, targets=targets, sh_degree=sh_degree)
