"""GPU parity of the batched multi-view step at the size it is measured at:
1M Gaussians at SH degree 3, the eight ring views of uneven resolution
(640x480 .. 1920x1440, 38k tiles), in the launch configuration of the
batched benchmark (16x16 tiles, batches of 256, persistent grid), with the
replay trace and with the recompute backward.

All eight views run in one batched step; two of them (the smallest and the
largest) are compared with the oracle, as the single-view full-size tests
do: every sorted pair of those views, compositing, T_final, n_contrib and
count on sampled tiles (the heaviest plus seeded random ones), their 2D
gradients for every Gaussian, and every canonical gradient.  dL/dimage is
non-zero only on the sampled tiles of the two views (zero on the other six),
which makes the oracle's sampled-tile backward the exact gradient.
Inputs: flat Gaussians on the seeded spheres-and-planes scene.
"""

import numpy as np
import pytest
import torch

import synth
from gpu_helpers import GRAD_TOL, IMG_TOL, assert_block_close, say
from oracle.binning import bin_and_sort
from oracle.projection import project, project_vjp
from oracle.render import render_backward, render_forward

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda")


@pytest.mark.parametrize("cached", [True, False], ids=["cached", "recompute"])
def test_views_full_size_two_views_match_oracle(cached):
    from paper_2601_17354_amd.batch import BatchedStep, mixed_views
    tw, th = 16, 16
    scene = synth.spheres_planes_scene(0)
    P = synth.surface_gaussians(scene, 1_000_000, seed=82, sh_degree=3, logit_sigma=0.5)
    cams = mixed_views()
    sizes = [c["width"] * c["height"] for c in cams]
    checked = sorted({int(np.argmin(sizes)), int(np.argmax(sizes))})
    rng = np.random.default_rng(23)
    ref, dls = {}, []
    for v, cam in enumerate(cams):
        W, H = cam["width"], cam["height"]
        dl = np.zeros((3, H, W), np.float32)
        if v in checked:
            say(f"[views-full] view {v} {W}x{H}: oracle projection and sort")
            proj = project(P, cam, tw, th)
            bins = bin_and_sort(proj)
            lens = bins["ranges"][:, 1] - bins["ranges"][:, 0]
            busy = np.nonzero(lens > 0)[0]
            tiles = sorted({int(np.argmax(lens))} | {int(t) for t in rng.choice(busy, 2, replace=False)})
            fwd = render_forward(proj, bins, cam, tw, th, (0.0, 0.0, 0.0), tiles=tiles)
            TX = (W + tw - 1) // tw
            on = np.zeros((H, W), bool)
            for t in tiles:
                ty, tx = divmod(t, TX)
                on[ty * th:(ty + 1) * th, tx * tw:(tx + 1) * tw] = True
            dl[:, on] = rng.normal(size=(3, int(on.sum()))).astype(np.float32)
            g2d, taint = render_backward(proj, bins, fwd, dl, "cached" if cached else "recompute")
            grads = project_vjp(P, cam, g2d, proj["visible"])
            say(f"  pairs {bins['num_pairs']}, sampled tiles {tiles} with {lens[tiles].tolist()} pairs")
            ref[v] = dict(proj=proj, bins=bins, fwd=fwd, on=on, g2d=g2d, taint=taint, grads=grads)
        dls.append(dl)

    say(f"[views-full] batched step, 8 views, {'cached' if cached else 'recompute'} backward")
    targets = [torch.zeros((3, c["height"], c["width"]), device=DEV) for c in cams]
    st = BatchedStep(torch.as_tensor(P, device=DEV), 3, cams, targets, tile=(tw, th), batch=256, cached=cached)
    st.prepare()
    torch.cuda.synchronize()
    for v in range(len(cams)):
        st.view_slice(st.dl, v).copy_(torch.as_tensor(dls[v], device=DEV))
    st.grads.zero_()
    st.backward_from()
    torch.cuda.synchronize()
    assert st.read_flags() == 0
    assert st.nt == sum(((c["width"] + tw - 1) // tw) * ((c["height"] + th - 1) // th) for c in cams)

    npairs = int(st.num_pairs.item())
    keys = st.keys[:npairs].cpu().numpy().view(np.uint64)
    vals = st.values[:npairs].cpu().numpy().astype(np.int64)
    offs = st.views.tile_offsets
    tile_of = (keys >> np.uint64(32)).astype(np.int64)
    say(f"  batched pairs {npairs}, tiles {st.nt}")
    for v, r in ref.items():
        lo, hi = offs[v], offs[v + 1]
        sel = (tile_of >= lo) & (tile_of < hi)
        want_k = r["bins"]["keys"] + (np.uint64(lo) << np.uint64(32))
        want_v = r["bins"]["values"].astype(np.int64)
        marg = r["proj"]["marginal"]
        kg, kw = ~marg[vals[sel]], ~marg[want_v]
        say(f"  view {v}: pairs {int(sel.sum())} (oracle {want_k.size}), marginal Gaussians {int(marg.sum())}")
        np.testing.assert_array_equal(keys[sel][kg], want_k[kw])
        np.testing.assert_array_equal(vals[sel][kg], want_v[kw])

    grads_want = np.zeros_like(P, dtype=np.float64)
    taint_any = np.zeros(P.shape[1], bool)
    for v, r in ref.items():
        on, fwd = r["on"], r["fwd"]
        ok = on & ~fwd["marginal"]
        img = st.view_slice(st.image, v).cpu().numpy()
        for c in range(3):
            assert_block_close(img[c][on], fwd["image"][c][on], IMG_TOL, mask=ok[on], what=f"view {v} image[{c}]")
        tf = st.view_slice(st.t_final, v, channels=1).cpu().numpy()
        assert_block_close(tf[on], fwd["T_final"][on], IMG_TOL, mask=ok[on], what=f"view {v} T_final")
        nc = st.view_slice(st.n_contrib, v, channels=1).cpu().numpy()
        assert (nc[ok] == fwd["n_contrib"][ok]).all()
        if cached:
            cnt = st.view_slice(st.trace["count"], v, channels=1).cpu().numpy()
            assert (cnt[ok] == fwd["count"][ok]).all()
        g2 = st.grad2d[v].cpu().numpy()[:, :9].T
        for f in range(9):
            assert_block_close(g2[f], r["g2d"][f], GRAD_TOL, mask=~r["taint"], what=f"view {v} grad2d[{f}]")
        grads_want += r["grads"]
        taint_any |= r["taint"]
    g = st.grads.cpu().numpy()
    for row in range(g.shape[0]):
        assert_block_close(g[row], grads_want[row], GRAD_TOL, mask=~taint_any, what=f"canonical row {row}")
