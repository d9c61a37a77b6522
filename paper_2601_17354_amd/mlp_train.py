"""Training pairs and training of the seeding network.

    python -m paper_2601_17354_amd.mlp_train --out DIR

Pairs come from the method's own optimisation: for each scene seed
(default 100..119), a 100k-point noisy cloud of a spheres-and-planes scene is
seeded by the plain disc-like seed and trained for 3000 steps (every one of
the 60 ring views at 1024x768, 0.8 L1 + 0.2 D-SSIM, Adam; no densification,
so Gaussian i stays point i in the canonical layout).  A pair is (features of
point i, trained scale / rotation / opacity of Gaussian i); Gaussians that
never received a gradient are dropped.  The network is trained with Adam on
the seed loss (batch 16384, cosine learning-rate decay) on all scenes but
the last two, which measure the validation loss.  Writes DIR/seed_mlp.npy
(the 13000 float32 weights) and DIR/seed_mlp.json (recipe and losses).
Every step runs in libpocketgs kernels.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

from . import binding as B
from .seed_mlp import N_WEIGHTS, SeedNetTrainer, features, init_weights, neighbourhoods
from .train import R_NORMAL, Trainer, train
from .workloads import scene_views


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def scene_pairs(scene_seed, n_points=100_000, n_gt=400_000, width=1024, height=768, iters=3000):
    """(x [m][64], base [m][16], targets [m][8]) of one scene's reached Gaussians."""
    wl = scene_views(scene_seed, n_points, n_gt, width, height)
    P, C = wl["cloud"]
    nbr, d2 = neighbourhoods(P)
    m = P.shape[1]
    params0 = torch.empty((14, m), dtype=torch.float32, device=P.device)
    B.pgs_pca_seed(P, C, m, nbr, d2, 16, R_NORMAL, params0)
    x, base = features(P, nbr, d2)
    tr = Trainer(params0, 0, width, height, cached=True, lam=0.2, extent=4.5)
    order = [int(i) for i in np.random.default_rng(scene_seed).permutation(len(wl["cams"]))]
    train(tr, wl["cams"], wl["targets"], order, iters)
    tgt = torch.empty((m, 8), dtype=torch.float32, device=P.device)
    B.pgs_seed_targets(tr.params, m, tgt)
    reached = tr.v.abs().sum(0) > 0
    keep = torch.nonzero(reached).squeeze(1)
    torch.cuda.synchronize()
    del tr, wl
    return x.index_select(0, keep), base.index_select(0, keep), tgt.index_select(0, keep), m


def fit(X, Bs, T, Xv, Bv, Tv, epochs=40, batch=16384, lr=1e-3, lr_min=1e-5, seed=0):
    trn = SeedNetTrainer(torch.as_tensor(init_weights(seed), device=X.device), lr=lr, max_rows=batch)
    n = X.shape[0]
    per_epoch = n // batch
    total = epochs * per_epoch
    gen = torch.Generator(device=X.device)
    gen.manual_seed(seed)
    hist = {"val_loss_untrained": trn.evaluate(Xv, Bv, Tv), "train_loss_untrained": trn.evaluate(X, Bs, T)}
    log(f"untrained (plain seed): train {hist['train_loss_untrained']:.4f} val {hist['val_loss_untrained']:.4f}")
    hist["epochs"] = []
    step = 0
    for ep in range(epochs):
        perm = torch.randperm(n, device=X.device, generator=gen)
        for b in range(per_epoch):
            idx = perm[b * batch:(b + 1) * batch]
            rate = lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * step / total))
            trn.step(X.index_select(0, idx), Bs.index_select(0, idx), T.index_select(0, idx), lr=rate)
            step += 1
        val = trn.evaluate(Xv, Bv, Tv)
        hist["epochs"].append(round(val, 5))
        log(f"epoch {ep + 1}/{epochs}: val loss {val:.4f}")
    hist["train_loss"] = trn.evaluate(X, Bs, T)
    hist["val_loss"] = hist["epochs"][-1]
    return trn.w, hist


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--scenes", default="100-119")
    ap.add_argument("--points", type=int, default=100_000)
    ap.add_argument("--gt", type=int, default=400_000)
    ap.add_argument("--width", type=int, default=1024)
    ap.add_argument("--height", type=int, default=768)
    ap.add_argument("--iters", type=int, default=3000)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--batch", type=int, default=16384)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--val-scenes", type=int, default=2)
    args = ap.parse_args()
    a, b = (int(v) for v in args.scenes.split("-"))
    seeds = list(range(a, b + 1))
    os.makedirs(args.out, exist_ok=True)
    t0 = time.perf_counter()
    parts, counts = [], {}
    for s in seeds:
        x, base, tgt, m = scene_pairs(s, args.points, args.gt, args.width, args.height, args.iters)
        counts[str(s)] = [int(x.shape[0]), m]
        parts.append((x, base, tgt))
        log(f"scene {s}: {x.shape[0]} of {m} Gaussians reached ({time.perf_counter() - t0:.0f} s)")
    nv = args.val_scenes
    X = torch.cat([p[0] for p in parts[:-nv]])
    Bs = torch.cat([p[1] for p in parts[:-nv]])
    T = torch.cat([p[2] for p in parts[:-nv]])
    Xv = torch.cat([p[0] for p in parts[-nv:]])
    Bv = torch.cat([p[1] for p in parts[-nv:]])
    Tv = torch.cat([p[2] for p in parts[-nv:]])
    del parts
    log(f"{X.shape[0]} training pairs, {Xv.shape[0]} validation pairs")
    w, hist = fit(X, Bs, T, Xv, Bv, Tv, args.epochs, args.batch, args.lr)
    wn = w.cpu().numpy().astype(np.float32)
    assert wn.size == N_WEIGHTS and np.isfinite(wn).all()
    np.save(os.path.join(args.out, "seed_mlp.npy"), wn)
    meta = dict(recipe=vars(args), scenes=seeds, pairs_per_scene=counts, train_pairs=int(X.shape[0]),
                val_pairs=int(Xv.shape[0]), seconds=round(time.perf_counter() - t0, 1), **hist)
    with open(os.path.join(args.out, "seed_mlp.json"), "w") as f:
        json.dump(meta, f, indent=1)
    log(f"done: val loss {hist['val_loss_untrained']:.4f} -> {hist['val_loss']:.4f}")


if __name__ == "__main__":
    main()
