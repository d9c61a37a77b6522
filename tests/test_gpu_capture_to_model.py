"""From captures to a trained model, every stage on the GPU: ray-cast
greyscale views of the seeded scene -> depth ranges from surface samples
(standing in for the refined sparse points), references by S_ref, Census /
plane-sweep / SGM depth maps, fusion into a coloured cloud -> PCA seeding
-> training against the same views.  Each stage has its own parity tests;
this checks the chain end to end by properties (parity unpinned: the chain
as a whole has no closed form): the fused cloud lies on the scene, and the
held-out PSNR of the seeded model rises with training."""

import numpy as np
import pytest
import torch

import synth
from gpu_helpers import say

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(600)
def test_capture_to_trained_model():
    from paper_2601_17354_amd import mvs, train
    W, H, V = 320, 240, 24
    scene = synth.spheres_planes_scene(0)
    cams = synth.ring_cameras(V, W, H)
    say("[capture] ray casting")
    grey_np, _ = synth.textured_views(scene, cams, seed=5)
    grey = torch.as_tensor(grey_np, device="cuda")
    sparse = torch.as_tensor(synth.sample_surface(scene, 20000, 1)[0], device="cuda")
    m = mvs.MVS(cams, W, H, mvs.MVSParams(), max_targets=V)
    m.prepare(grey, sparse)
    targets = torch.arange(V, dtype=torch.int32, device="cuda")
    m.depth_maps(targets)
    stride = 12
    cap = V * W * H // stride + 1
    P = torch.empty((3, cap), dtype=torch.float32, device="cuda")
    C = torch.empty_like(P)
    kept = int(m.fuse(targets, P, grey=grey, colours=C, stride=stride).item())
    n = (kept + stride - 1) // stride
    P, C = P[:, :n].contiguous(), C[:, :n].contiguous()
    say(f"[capture] kept pixels {kept}, cloud {n} points")
    assert n > 20000
    # the cloud lies on the scene's surfaces
    Pn = P.cpu().numpy().T.astype(np.float64)
    ds = np.abs(np.linalg.norm(Pn[:, None] - scene.centres[None], axis=2) - scene.radii[None]).min(1)
    dp = np.min(np.stack([np.abs((Pn - o) @ nn) for (o, _, _, nn, _, _) in scene.planes], 1), 1)
    dist = np.minimum(ds, dp)
    say(f"[capture] distance to the surfaces: median {np.median(dist):.4f}, 90% {np.percentile(dist, 90):.4f}")
    assert np.median(dist) < 0.02 and np.percentile(dist, 90) < 0.1
    # seed and train against the captures (every 6th view held out)
    params = train.seed_pca(P, C)
    tgt = {i: (grey[i].float() / 255.0).expand(3, H, W).contiguous() for i in range(V)}
    test_ids = [i for i in range(V) if i % 6 == 0]
    order = [i for i in range(V) if i % 6 != 0]
    tr = train.Trainer(params, 0, W, H)
    tr.prepare(cams[order[0]])
    hist = train.train(tr, cams, tgt, order, 400, eval_ids=test_ids, eval_at=(0, 400), log=say)
    say(f"[capture] held-out PSNR {hist}")
    assert np.isfinite(hist[400]) and hist[400] > hist[0] + 1.0
