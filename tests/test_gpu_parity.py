"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bars: integer and index outputs (culling, radius, rectangles, pair keys and
values, tile ranges, n_contrib, count, trace ids) bit-exact except where the
oracle reports a near-threshold decision; images 1e-5 and gradients 1e-4 by
the block-relative rule of gpu_helpers.
"""

import numpy as np
import pytest

import synth
from gpu_helpers import (GRAD_TOL, IMG_TOL, assert_block_close, assert_cin_close, max_rel, run_gpu, say,
                         trace_entries)
from oracle import pipeline
from oracle.projection import OUT_FIELDS

pytestmark = pytest.mark.gpu

PROJ_ROWS = dict(u=0, v=1, A=3, B=4, C=5, o=6, r=7, g=8, b=9)


def _scene_small(seed=3, n=20000, W=320, H=240, cam_idx=5):
    scene = synth.spheres_planes_scene(seed)
    P = synth.surface_gaussians(scene, n, seed=seed + 50, sh_degree=3, logit_sigma=0.5)
    cam = synth.ring_cameras(60, W, H)[cam_idx]
    return P, cam


def _cases():
    out = []
    for s in (0, 1, 2):
        P, cam, _ = synth.cfg1_inputs(s)
        out.append((f"cfg1-seed{s}", P, cam, 0, (0.0, 0.0, 0.0)))
    P, cam = _scene_small()
    out.append(("scene-sh3-320x240", P, cam, 3, (0.1, 0.2, 0.3)))
    P, _, _ = synth.cfg1_inputs(7, n=400, width=100, height=75, focal=90.0)
    cam = synth.make_camera(100, 75, 90.0, 90.0, 50.0, 37.5, np.eye(3), np.zeros(3))
    out.append(("ragged-100x75", P, cam, 0, (0.5, 0.5, 0.5)))
    # long thin splats (conic correlations up to ~0.995), half of them with
    # opacity within a few times 1/255: alpha contours that graze the row
    # bands of the tiles' waves, for the forward's per-wave reach test
    P, cam, _ = synth.cfg1_inputs(11, n=1500)
    rng = np.random.default_rng(11)
    n = P.shape[1]
    P[3] = rng.uniform(-2.0, -0.5, n)
    P[4:6] = rng.uniform(-7.0, -5.0, (2, n))
    o = rng.uniform(0.5, 4.0, n) / 255.0
    P[10] = np.where(np.arange(n) % 2 == 0, np.log(o / (1.0 - o)), P[10])
    out.append(("needles-128x128", P.astype(np.float32), cam, 0, (0.0, 0.0, 0.0)))
    return out


CASES = _cases()


@pytest.fixture(scope="module", params=range(len(CASES)), ids=[c[0] for c in CASES])
def case(request):
    name, P, cam, deg, bg = CASES[request.param]
    say(f"[parity] case {name}: n={P.shape[1]} {cam['width']}x{cam['height']} sh={deg}")
    rng = np.random.default_rng(99)
    dl = rng.normal(size=(3, cam["height"], cam["width"])).astype(np.float32)
    proj, bins, fwd = pipeline.forward(P, cam, bg=bg)
    o_grads, o_g2d, tainted = pipeline.backward(P, cam, proj, bins, fwd, dl, "cached")
    gpu_c = run_gpu(P, cam, deg, cached=True, bg=bg, dl_dimage=dl)
    gpu_c4 = run_gpu(P, cam, deg, cached=True, bg=bg, dl_dimage=dl, trace_words=4)
    gpu_r = run_gpu(P, cam, deg, cached=False, bg=bg, dl_dimage=dl)
    return dict(name=name, P=P, cam=cam, bg=bg, dl=dl, proj=proj, bins=bins, fwd=fwd,
                o_grads=o_grads, o_g2d=o_g2d, tainted=tainted, gc=gpu_c, gc4=gpu_c4, gr=gpu_r)


def test_projection(case):
    proj, g = case["proj"], case["gc"]
    vis = proj["visible"]
    ok = ~proj["marginal"]
    assert ((g["radius"] > 0) == vis)[ok].all()
    m = vis & ok
    assert (g["radius"][m] == proj["radius"][m]).all()
    rect = g["rect"]
    x0, y0 = rect[0] & 0xFFFF, rect[0] >> 16
    x1, y1 = rect[1] & 0xFFFF, rect[1] >> 16
    want = proj["rect"]
    assert (x0[m] == want[m, 0]).all() and (y0[m] == want[m, 1]).all()
    assert (x1[m] == want[m, 2]).all() and (y1[m] == want[m, 3]).all()
    assert (g["touched"][m] == proj["tiles_touched"][m]).all()
    assert (g["proj"][2][m].view(np.uint32) == proj["depth32"][m].view(np.uint32)).all()
    for k, row in PROJ_ROWS.items():
        np.testing.assert_allclose(g["proj"][row][m], proj[k][m], rtol=2e-7, atol=1e-30, err_msg=k)


def _drop_marginal(keys, vals, marginal):
    keep = ~marginal[vals.astype(np.int64)]
    return keys[keep], vals[keep]


def test_bin_sort_bit_exact(case):
    bins, g, proj = case["bins"], case["gc"], case["proj"]
    assert g["flags"] == 0
    marg = proj["marginal"]
    say(f"  pairs {bins['num_pairs']} marginal gaussians {int(marg.sum())}")
    if not marg.any():
        assert g["num_pairs"] == bins["num_pairs"]
        np.testing.assert_array_equal(g["keys"], bins["keys"])
        np.testing.assert_array_equal(g["values"].astype(np.int64), bins["values"])
        np.testing.assert_array_equal(g["ranges"].T.astype(np.int64), bins["ranges"])
    else:
        gk, gv = _drop_marginal(g["keys"], g["values"], marg)
        ok_, ov = _drop_marginal(bins["keys"], bins["values"].astype(np.int64), marg)
        np.testing.assert_array_equal(gk, ok_)
        np.testing.assert_array_equal(gv, ov)


def test_render_forward(case):
    fwd, g = case["fwd"], case["gc"]
    ok = ~fwd["marginal"]
    say(f"  marginal pixels {int((~ok).sum())}; image max rel {max_rel(g['image'], fwd['image']):.2e}")
    assert (~ok).sum() <= max(2, ok.size // 1000)
    for c in range(3):
        assert_block_close(g["image"][c], fwd["image"][c], IMG_TOL, mask=ok, what=f"image[{c}]")
    assert_block_close(g["t_final"], fwd["T_final"], IMG_TOL, mask=ok, what="T_final")
    assert (g["n_contrib"][ok] == fwd["n_contrib"][ok]).all()
    assert (g["count"][ok] == fwd["count"][ok]).all()
    # the no-trace forward and the 4-word trace layout write the same image bits
    for other in ("gr", "gc4"):
        np.testing.assert_array_equal(g["image"], case[other]["image"])
        np.testing.assert_array_equal(g["n_contrib"], case[other]["n_contrib"])
    np.testing.assert_array_equal(g["count"], case["gc4"]["count"])


@pytest.mark.parametrize("layout", ["gc", "gc4"])
def test_replay_trace_entries(case, layout):
    # ids and C_in in both entry layouts; alpha where the entry stores it
    from oracle.render import replay_entries
    fwd, g, cam = case["fwd"], case[layout], case["cam"]
    H, W = cam["height"], cam["width"]
    rng = np.random.default_rng(5)
    pix = [(int(x), int(y)) for x, y in zip(rng.integers(0, W, 24), rng.integers(0, H, 24))]
    ys, xs = np.nonzero(fwd["count"] == fwd["count"].max())
    pix.append((int(xs[0]), int(ys[0])))
    worst = 0.0
    for x, y in pix:
        if fwd["marginal"][y, x]:
            continue
        want = replay_entries(fwd, x, y)
        ids, al, cin = trace_entries(g, cam, x, y)
        assert list(ids) == [e[0] for e in want], (x, y)
        if want:
            if al is not None:
                assert_block_close(al, [e[1] for e in want], IMG_TOL, what=f"alpha {(x, y)}")
            w = np.asarray([e[2] for e in want])
            worst = max(worst, assert_cin_close(cin, w, (x, y)))
    say(f"  C_in error / its rounding bound, worst entry: {worst:.3f}")


def test_trace_layouts_hold_the_same_colours(case):
    # Every (tile, wave) region of the 12-byte layout against the first three
    # words of the 16-byte one, bit for bit: the same entries in the same
    # order, only the region starts differ between the two launches.  (A
    # store that picked up the next entry's colour registers showed up here
    # as single mismatched words.)
    a, b = case["gc"]["rast"], case["gc4"]["rast"]
    steps_a, steps_b = a.trace["steps"].cpu().numpy(), b.trace["steps"].cpu().numpy()
    np.testing.assert_array_equal(steps_a, steps_b)
    base_a = a.trace["base"].cpu().numpy().astype(np.int64) & 0xFFFFFFFF
    base_b = b.trace["base"].cpu().numpy().astype(np.int64) & 0xFFFFFFFF
    masks = a.trace["mask"].cpu().numpy().view(np.uint64)
    masks_b = b.trace["mask"].cpu().numpy().view(np.uint64)
    ent_a, ent_b = a.trace["entry"].cpu().numpy(), b.trace["entry"].cpu().numpy()
    ranges = case["gc"]["ranges"]
    total = 0
    for t in range(steps_a.shape[0]):
        start = int(ranges[0, t])
        for w in range(steps_a.shape[1]):
            st = int(steps_a[t, w])
            if st == 0:
                continue
            # only the steps the forward recorded hold masks
            m = masks[w, start:start + st]
            np.testing.assert_array_equal(m, masks_b[w, start:start + st])
            cnt = int(np.bitwise_count(m).sum())
            ra = ent_a[base_a[t, w]:base_a[t, w] + cnt]
            rb = ent_b[base_b[t, w]:base_b[t, w] + cnt, :3]
            assert np.array_equal(ra.view(np.uint32), rb.view(np.uint32)), (t, w)
            total += cnt
    assert total == int(case["gc"]["count"].sum())
    say(f"  {total} entries equal in both layouts")


@pytest.mark.parametrize("variant", ["gc", "gc4", "gr"])
def test_render_backward_2d(case, variant):
    g, og, taint = case[variant], case["o_g2d"], case["tainted"]
    ok = ~taint
    say(f"  {variant} tainted {int(taint.sum())}")
    for f, name in enumerate(OUT_FIELDS):
        assert_block_close(g["grad2d"][f], og[f], GRAD_TOL, mask=ok, what=f"{variant} d{name}")


@pytest.mark.parametrize("variant", ["gc", "gc4", "gr"])
def test_canonical_gradients(case, variant):
    g, og, taint = case[variant], case["o_grads"], case["tainted"]
    ok = ~taint
    for r in range(og.shape[0]):
        assert_block_close(g["grads"][r], og[r], GRAD_TOL, mask=ok, what=f"{variant} row {r}")


def test_cached_and_recompute_agree(case):
    a, b = case["gc"]["grads"], case["gr"]["grads"]
    for r in range(a.shape[0]):
        assert_block_close(a[r], b[r], GRAD_TOL, what=f"row {r}")
