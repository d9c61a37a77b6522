"""GPU tests of the autograd wrapper, the PSNR metric and a short training
run, against the oracle and finite differences."""

import numpy as np
import pytest
import torch

import synth
from gpu_helpers import GRAD_TOL, IMG_TOL, assert_block_close, say
from oracle import loss as o_loss
from oracle import pipeline

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda")


@pytest.mark.parametrize("cached", [True, False])
def test_autograd_matches_oracle(cached):
    from paper_2601_17354_amd.autograd import rasterize
    from paper_2601_17354_amd.raster import Rasterizer
    P, cam, _ = synth.cfg1_inputs(2)
    w = np.random.default_rng(3).normal(size=(3, 128, 128)).astype(np.float32)
    params = torch.as_tensor(P, device=DEV).requires_grad_(True)
    R = Rasterizer(P.shape[1], 0, 128, 128, cached=cached)
    img = rasterize(params, R, cam)
    (img * torch.as_tensor(w, device=DEV)).sum().backward()
    torch.cuda.synchronize()
    proj, bins, fwd = pipeline.forward(P, cam)
    og, _, taint = pipeline.backward(P, cam, proj, bins, fwd, w)
    ok = ~fwd["marginal"]
    for c in range(3):
        assert_block_close(img.detach().cpu().numpy()[c], fwd["image"][c], IMG_TOL, mask=ok)
    g = params.grad.cpu().numpy()
    for r in range(og.shape[0]):
        assert_block_close(g[r], og[r], GRAD_TOL, mask=~taint, what=f"row {r}")


def test_autograd_finite_differences_fp32():
    # Loose float32 central differences of <w, image> through the wrapper
    # (the tight checks are the oracle comparison above and the oracle's own
    # FP64 differences).  Directions move the colour coefficients, on which
    # the image is linear (no branch can flip), and the opacity logits.
    from paper_2601_17354_amd.autograd import rasterize
    from paper_2601_17354_amd.raster import Rasterizer
    P, cam, _ = synth.cfg1_inputs(4, n=200)
    w = torch.as_tensor(np.random.default_rng(5).normal(size=(3, 128, 128)).astype(np.float32), device=DEV)
    R = Rasterizer(P.shape[1], 0, 128, 128, cached=True)
    params = torch.as_tensor(P, device=DEV).requires_grad_(True)
    (rasterize(params, R, cam) * w).sum().backward()
    g = params.grad.detach().clone()
    rng = np.random.default_rng(6)
    # colour channels at least 0.05 away from the clamp at 0 (and from 1)
    colour = P[11:14] / (2 * np.sqrt(np.pi)) + 0.5
    safe = ((colour > 0.05) & (colour < 0.95)).astype(np.float32)
    base = pipeline.decisions(P, cam)
    for rows, h, tol in (([11, 12, 13], 1e-2, 1e-3), ([10], 1e-4, 2e-2)):
        V = torch.zeros_like(params)
        for _ in range(20):
            d = rng.normal(size=(len(rows), P.shape[1])).astype(np.float32)
            if rows[0] == 11:
                d *= safe
                break
            # opacity moves alpha: keep a direction whose FP64 decisions
            # (skips, terminations, clamps) stay the same at +-h
            D = np.zeros_like(P, dtype=np.float64)
            D[rows] = d
            if (pipeline.same_decisions(pipeline.decisions(P + h * D, cam), base) and
                    pipeline.same_decisions(pipeline.decisions(P - h * D, cam), base)):
                break
        V[rows] = torch.as_tensor(d, device=DEV)
        with torch.no_grad():
            fp = (rasterize(params + h * V, R, cam).double() * w.double()).sum().item()
            fm = (rasterize(params - h * V, R, cam).double() * w.double()).sum().item()
        fd = (fp - fm) / (2 * h)
        an = float((g.double() * V.double()).sum())
        say(f"  rows {rows}: fd {fd:.6f} analytic {an:.6f}")
        assert abs(fd - an) <= tol * abs(an) + 1e-3


def test_photometric_loss_autograd():
    from paper_2601_17354_amd.autograd import photometric_loss
    rng = np.random.default_rng(8)
    x = rng.uniform(size=(3, 40, 52)).astype(np.float32)
    y = rng.uniform(size=(3, 40, 52)).astype(np.float32)
    xt = torch.as_tensor(x, device=DEV).requires_grad_(True)
    loss = photometric_loss(xt, torch.as_tensor(y, device=DEV), 0.2)
    (2.0 * loss).backward()
    want, wg = o_loss.l1_dssim(x, y, 0.2)
    assert abs(loss.item() - want) <= 1e-5 * abs(want)
    for c in range(3):
        assert_block_close(xt.grad.cpu().numpy()[c], 2.0 * wg[c], 1e-4)


def test_psnr_matches_oracle():
    from paper_2601_17354_amd import binding as B
    rng = np.random.default_rng(9)
    x = rng.uniform(-0.2, 1.2, size=(3, 33, 47)).astype(np.float32)
    y = rng.uniform(size=(3, 33, 47)).astype(np.float32)
    out = torch.zeros(2, device=DEV)
    ws = torch.empty(4096, dtype=torch.uint8, device=DEV)
    B.pgs_psnr(torch.as_tensor(x, device=DEV), torch.as_tensor(y, device=DEV), 47, 33, out, ws)
    torch.cuda.synchronize()
    assert abs(out[1].item() - o_loss.psnr(x, y)) < 1e-4


def test_short_training_improves_held_out_psnr():
    # A small scene trained for 150 steps: the held-out PSNR must rise.
    from paper_2601_17354_amd.train import Trainer, seed_pca, train
    from paper_2601_17354_amd.workloads import render_targets
    scene = synth.spheres_planes_scene(4)
    gt = torch.as_tensor(synth.surface_gaussians(scene, 60000, seed=41, opacity=0.95), device=DEV)
    cams = synth.ring_cameras(16, 320, 240)
    targets = dict(enumerate(render_targets(gt, 0, cams, 320, 240)))
    pts, col = synth.noisy_cloud(scene, 40000, seed=42)
    P0 = seed_pca(torch.as_tensor(np.ascontiguousarray(pts.T), device=DEV),
                  torch.as_tensor(np.ascontiguousarray(col.T), device=DEV))
    tr = Trainer(P0, 0, 320, 240, cached=True, extent=4.5)
    train_ids = [i for i in range(16) if i % 4]
    hist = train(tr, cams, targets, train_ids, 150, eval_ids=[0, 4, 8, 12], eval_at=(0, 150))
    say(f"  PSNR {hist}")
    assert np.isfinite(tr.params.cpu().numpy()).all()
    assert hist[150] > hist[0] + 1.0


@pytest.mark.parametrize("cached", [True, False])
def test_single_view_step_graphs_replay_like_eager_steps(cached):
    # One graph per training view (the camera is a kernel argument, Adam's
    # step counter lives on the device), replayed cycling the views with
    # unrelated eager work and host synchronisations in between, against the
    # same steps run eagerly from the same start.
    from paper_2601_17354_amd import binding as B
    from paper_2601_17354_amd.train import Trainer
    scene = synth.spheres_planes_scene(4)
    P = synth.surface_gaussians(scene, 20000, seed=61, sh_degree=0, logit_sigma=0.5)
    cams = [synth.ring_cameras(12, 320, 240)[i] for i in (0, 5)]
    rng = np.random.default_rng(14)
    targets = [torch.as_tensor(rng.uniform(size=(3, 240, 320)).astype(np.float32), device=DEV) for _ in cams]
    say(f"[train] single-view step graphs vs eager, cached={cached}")
    ga, eb = (Trainer(torch.as_tensor(P, device=DEV), 0, 320, 240, cached=cached, extent=4.5,
                      device_step_counter=True) for _ in range(2))
    for t in (ga, eb):
        for c in cams:
            t.prepare(c)
        t.rast.reserve(2.0)
        t.rast.flags.zero_()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graphs = []
    with torch.cuda.stream(s):
        for c, tg in zip(cams, targets):
            B.pgs_graph_begin(s)
            try:
                ga.step(c, tg)
            finally:
                graphs.append(B.pgs_graph_end(s))
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    # capture records without running: nothing has moved yet
    assert int(ga.adam_state[0].item()) == 0
    np.testing.assert_array_equal(ga.params.cpu().numpy(), P)
    try:
        for k in range(6):
            v = k % 2
            B.pgs_graph_launch(graphs[v])
            eb.step(cams[v], targets[v])
            scratch = torch.randn(1 << 20, device=DEV)
            scratch.mul_(2.0).sum().item()
            torch.cuda.synchronize()
            assert ga.rast.read_flags() == 0 and eb.rast.read_flags() == 0
            la, lb = float(ga.loss.item()), float(eb.loss.item())
            say(f"  step {k + 1} (view {v}): loss graph {la:.6f} eager {lb:.6f}")
            assert abs(la - lb) <= 1e-4 * abs(lb)
            diff = np.abs(ga.params.cpu().numpy() - eb.params.cpu().numpy())
            # float atomics may order the gradient sums differently; Adam's
            # normalised step bounds what that can move per step
            assert diff.max() <= 2.0 * (k + 1) * 2.5e-2, diff.max()
            assert (diff <= 1e-5).mean() > 0.99
        assert int(ga.adam_state[0].item()) == 6 and int(eb.adam_state[0].item()) == 6
    finally:
        torch.cuda.synchronize()
        for g in graphs:
            B.pgs_graph_destroy(g)
