"""GPU parity at full size, in the launch configuration of the training step
(16x16 tiles): the benchmark workload (300k Gaussians, SH degree 0, one
1920x1440 view) and the SH degree 3 configuration (100k Gaussians, one
1024x768 view).

The oracle cannot composite every pixel of that view in a test, so:
  * projection, binning and the (tile, depth) sort are compared in full
    (all Gaussians, every pair key and value, every tile range);
  * compositing, count, n_contrib and the replay trace are compared on
    sampled tiles (the heaviest tile plus seeded random ones), which the
    oracle renders one by one;
  * the backward is driven by a dL/dimage that is non-zero only on those
    tiles, so the oracle's gradients over the sampled tiles are the exact
    gradients of every Gaussian and are compared for all of them.
Inputs: flat Gaussians on the seeded spheres-and-planes scene (the shapes and
size mix of the training workload); ring cameras 7 and 0.
"""

import numpy as np
import pytest

import synth
from gpu_helpers import GRAD_TOL, IMG_TOL, assert_block_close, assert_cin_close, run_gpu, say, trace_entries
from oracle.binning import bin_and_sort
from oracle.projection import OUT_FIELDS, project, project_vjp
from oracle.render import render_backward, render_forward, replay_entries

pytestmark = pytest.mark.gpu

TILE = 16
# name: (Gaussians, SH degree, width, height, ring camera, generator keywords)
CONFIGS = {
    "300k-sh0-1920x1440": (300_000, 0, 1920, 1440, 7, dict(size=1.2)),
    "100k-sh3-1024x768": (100_000, 3, 1024, 768, 0, dict(logit_sigma=0.5)),
}


@pytest.fixture(scope="module", params=list(CONFIGS))
def full(request):
    N, deg, W, H, ci, kw = CONFIGS[request.param]
    scene = synth.spheres_planes_scene(0)
    P = synth.surface_gaussians(scene, N, seed=77, sh_degree=deg, **kw)
    cam = synth.ring_cameras(60, W, H)[ci]
    say(f"[fullsize] {request.param}: oracle projection and sort")
    proj = project(P, cam)
    bins = bin_and_sort(proj)
    r = bins["ranges"]
    npairs = r[:, 1] - r[:, 0]
    rng = np.random.default_rng(11)
    nonempty = np.nonzero(npairs > 0)[0]
    tiles = sorted({int(np.argmax(npairs))} | {int(t) for t in rng.choice(nonempty, 5, replace=False)})
    say(f"[fullsize] pairs {bins['num_pairs']}, sampled tiles {tiles} with {npairs[tiles].tolist()} pairs")
    fwd = render_forward(proj, bins, cam, TILE, TILE, (0.0, 0.0, 0.0), tiles=tiles)
    dl = np.zeros((3, H, W), np.float32)
    TX = W // TILE
    on = np.zeros((H, W), bool)
    for t in tiles:
        ty, tx = divmod(t, TX)
        on[ty * TILE:(ty + 1) * TILE, tx * TILE:(tx + 1) * TILE] = True
    dl[:, on] = rng.normal(size=(3, int(on.sum()))).astype(np.float32)
    g2d, tainted = render_backward(proj, bins, fwd, dl, "cached")
    grads = project_vjp(P, cam, g2d, proj["visible"])
    say("[fullsize] HIP path, cached and recompute")
    gc = run_gpu(P, cam, deg, cached=True, dl_dimage=dl)
    gc4 = run_gpu(P, cam, deg, cached=True, dl_dimage=dl, trace_words=4)
    gr = run_gpu(P, cam, deg, cached=False, dl_dimage=dl)
    return dict(P=P, cam=cam, proj=proj, bins=bins, tiles=tiles, on=on, fwd=fwd, g2d=g2d, tainted=tainted,
                grads=grads, gc=gc, gc4=gc4, gr=gr)


def test_full_projection_and_sort(full):
    proj, bins, g = full["proj"], full["bins"], full["gc"]
    assert g["flags"] == 0
    vis, ok = proj["visible"], ~proj["marginal"]
    assert ((g["radius"] > 0) == vis)[ok].all()
    m = vis & ok
    assert (g["touched"][m] == proj["tiles_touched"][m]).all()
    assert (g["proj"][2][m].view(np.uint32) == proj["depth32"][m].view(np.uint32)).all()
    if proj["marginal"].any():
        keep_g = ~proj["marginal"][g["values"].astype(np.int64)]
        keep_o = ~proj["marginal"][bins["values"].astype(np.int64)]
        np.testing.assert_array_equal(g["keys"][keep_g], bins["keys"][keep_o])
        np.testing.assert_array_equal(g["values"][keep_g].astype(np.int64), bins["values"][keep_o])
    else:
        assert g["num_pairs"] == bins["num_pairs"]
        np.testing.assert_array_equal(g["keys"], bins["keys"])
        np.testing.assert_array_equal(g["values"].astype(np.int64), bins["values"])
        np.testing.assert_array_equal(g["ranges"].T.astype(np.int64), bins["ranges"])


def test_full_sampled_tiles_forward(full):
    fwd, g, on = full["fwd"], full["gc"], full["on"]
    ok = on & ~fwd["marginal"]
    say(f"[fullsize] compared pixels {int(ok.sum())}, marginal {int((on & fwd['marginal']).sum())}")
    for c in range(3):
        assert_block_close(g["image"][c][on], fwd["image"][c][on], IMG_TOL, mask=ok[on], what=f"image[{c}]")
    assert_block_close(g["t_final"][on], fwd["T_final"][on], IMG_TOL, mask=ok[on], what="T_final")
    assert (g["n_contrib"][ok] == fwd["n_contrib"][ok]).all()
    assert (g["count"][ok] == fwd["count"][ok]).all()
    np.testing.assert_array_equal(g["image"], full["gr"]["image"])
    np.testing.assert_array_equal(g["image"], full["gc4"]["image"])


@pytest.mark.parametrize("layout", ["gc", "gc4"])
def test_full_sampled_trace_entries(full, layout):
    fwd, g, cam, on = full["fwd"], full[layout], full["cam"], full["on"]
    ys, xs = np.nonzero(on & ~fwd["marginal"])
    rng = np.random.default_rng(3)
    pick = rng.choice(xs.size, 24, replace=False)
    cnt = np.where(on, fwd["count"], -1)
    yb, xb = np.unravel_index(np.argmax(cnt), cnt.shape)
    pix = [(int(xs[i]), int(ys[i])) for i in pick] + [(int(xb), int(yb))]
    worst = 0.0
    for x, y in pix:
        want = replay_entries(fwd, x, y)
        ids, al, cin = trace_entries(g, cam, x, y)
        assert list(ids) == [e[0] for e in want], (x, y)
        if want:
            if al is not None:
                assert_block_close(al, [e[1] for e in want], IMG_TOL, what=f"alpha {(x, y)}")
            w = np.asarray([e[2] for e in want])
            worst = max(worst, assert_cin_close(cin, w, (x, y)))
    say(f"  C_in error / its rounding bound, worst entry: {worst:.3f}")


@pytest.mark.parametrize("variant", ["gc", "gc4", "gr"])
def test_full_gradients(full, variant):
    g, ok = full[variant], ~full["tainted"]
    say(f"[fullsize] {variant}: Gaussians with gradients {int((np.abs(full['g2d']).sum(0) > 0).sum())}")
    for f, name in enumerate(OUT_FIELDS):
        assert_block_close(g["grad2d"][f], full["g2d"][f], GRAD_TOL, mask=ok, what=f"{variant} d{name}")
    for r in range(full["grads"].shape[0]):
        assert_block_close(g["grads"][r], full["grads"][r], GRAD_TOL, mask=ok, what=f"{variant} row {r}")
