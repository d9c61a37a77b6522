"""GPU parity of the batched multi-view path (one bin/sort over every view,
persistent compositing forward and backward over the (view, tile) queue)
against the oracle run view by view, for every tile shape and several LDS
batch sizes; the device-counter Adam against the host-counter one; and
graph replays of the whole step against eager steps."""

import numpy as np
import pytest
import torch

import synth
from gpu_helpers import GRAD_TOL, IMG_TOL, assert_block_close, say
from oracle import pipeline

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda")


def _views():
    # one cloud of 1000 Gaussians (the small parity workload) seen by three
    # cameras of uneven size at the same pose
    P, _, _ = synth.cfg1_inputs(0)
    cams = [synth.make_camera(128, 128, 128.0, 128.0, 64.0, 64.0, np.eye(3), np.zeros(3)),
            synth.make_camera(100, 75, 90.0, 90.0, 50.0, 37.5, np.eye(3), np.zeros(3)),
            synth.make_camera(72, 40, 60.0, 60.0, 36.0, 20.0, np.eye(3), np.zeros(3))]
    return P, cams


def _oracle(P, cams, tile, bg, dls):
    out = []
    for cam, dl in zip(cams, dls):
        proj, bins, fwd = pipeline.forward(P, cam, tile[0], tile[1], bg)
        og, og2d, taint = pipeline.backward(P, cam, proj, bins, fwd, dl, "cached")
        out.append(dict(proj=proj, bins=bins, fwd=fwd, grads=og, g2d=og2d, taint=taint))
    return out


CONFIGS = [((16, 16), 256, True), ((8, 8), 32, True), ((16, 8), 128, True), ((32, 8), 64, True),
           ((8, 32), 256, True), ((16, 16), 32, True), ((16, 16), 128, False), ((8, 8), 64, False)]


def _assert_queue(st, blocks):
    """The persistent launch's queue counter after it ran: every workgroup
    takes items until one lies past the last tile, so the counter ends at
    tiles + workgroups.  With `blocks` workgroups over more tiles than that,
    the workgroups walked several queue items each (one workgroup walked all
    of them when blocks = 1)."""
    q = int(st.queue[0].item())
    if blocks > 0:
        assert q == st.nt + min(blocks, st.nt), (q, st.nt, blocks)
    else:
        assert st.nt < q <= 2 * st.nt, (q, st.nt)


BLOCKS = [0, 1, 3]


@pytest.mark.parametrize("blocks", BLOCKS, ids=[f"grid{b}" for b in BLOCKS])
@pytest.mark.parametrize("tile,batch,cached", CONFIGS, ids=[f"{t[0]}x{t[1]}-b{b}-{'c' if c else 'r'}"
                                                            for t, b, c in CONFIGS])
def test_views_match_oracle_per_view(tile, batch, cached, blocks):
    from paper_2601_17354_amd.batch import BatchedStep
    P, cams = _views()
    bg = (0.1, 0.2, 0.3)
    rng = np.random.default_rng(11)
    dls = [rng.normal(size=(3, c["height"], c["width"])).astype(np.float32) for c in cams]
    say(f"[views] tile {tile} batch {batch} cached {cached} blocks {blocks}")
    targets = [torch.zeros((3, c["height"], c["width"]), device=DEV) for c in cams]
    st = BatchedStep(torch.as_tensor(P, device=DEV), 0, cams, targets, tile=tile, batch=batch, cached=cached,
                     bg=bg, blocks=blocks)
    st.prepare()
    torch.cuda.synchronize()
    _assert_queue(st, blocks)
    for v in range(len(cams)):
        st.view_slice(st.dl, v).copy_(torch.as_tensor(dls[v], device=DEV))
    st.grads.zero_()
    st.backward_from()
    torch.cuda.synchronize()
    assert st.read_flags() == 0
    _assert_queue(st, blocks)
    ref = _oracle(P, cams, tile, bg, dls)

    # one sorted list = the per-view lists one after the other, tiles offset
    npairs = int(st.num_pairs.item())
    keys = st.keys[:npairs].cpu().numpy().view(np.uint64)
    vals = st.values[:npairs].cpu().numpy().astype(np.int64)
    offs = st.views.tile_offsets
    want_k = np.concatenate([r["bins"]["keys"] + (np.uint64(off) << np.uint64(32)) for r, off in zip(ref, offs)])
    want_v = np.concatenate([r["bins"]["values"] for r in ref]).astype(np.int64)
    n_marg = sum(int(r["proj"]["marginal"].sum()) for r in ref)
    say(f"  pairs {npairs}, marginal gaussians {n_marg}")
    if n_marg == 0:
        np.testing.assert_array_equal(keys, want_k)
        np.testing.assert_array_equal(vals, want_v)
        ranges = st.ranges.cpu().numpy().astype(np.int64)
        base = 0
        for r, t0, t1 in zip(ref, offs[:-1], offs[1:]):
            rr = r["bins"]["ranges"]
            want = np.where((rr[:, 1] > rr[:, 0])[:, None], rr + base, 0)   # empty tiles stay (0, 0)
            np.testing.assert_array_equal(ranges[:, t0:t1].T, want)
            base += r["bins"]["num_pairs"]
    else:
        # drop the pairs of Gaussians whose decisions are marginal in the
        # view the pair belongs to (view from the global tile of the key)
        def keep(k, v):
            view = np.searchsorted(np.asarray(offs[1:]), (k >> np.uint64(32)).astype(np.int64), side="right")
            marg = np.stack([r["proj"]["marginal"] for r in ref])
            return ~marg[view, v]
        kg, kw = keep(keys, vals), keep(want_k, want_v)
        np.testing.assert_array_equal(keys[kg], want_k[kw])
        np.testing.assert_array_equal(vals[kg], want_v[kw])

    grads_want = np.zeros_like(P, dtype=np.float64)
    taint_any = np.zeros(P.shape[1], bool)
    for v, r in enumerate(ref):
        ok = ~r["fwd"]["marginal"]
        img = st.view_slice(st.image, v).cpu().numpy()
        for c in range(3):
            assert_block_close(img[c], r["fwd"]["image"][c], IMG_TOL, mask=ok, what=f"view {v} image[{c}]")
        nc = st.view_slice(st.n_contrib, v, channels=1).cpu().numpy()
        assert (nc[ok] == r["fwd"]["n_contrib"][ok]).all()
        if cached:
            cnt = st.view_slice(st.trace["count"], v, channels=1).cpu().numpy()
            assert (cnt[ok] == r["fwd"]["count"][ok]).all()
        g2 = st.grad2d[v].cpu().numpy()[:, :9].T
        for f in range(9):
            assert_block_close(g2[f], r["g2d"][f], GRAD_TOL, mask=~r["taint"], what=f"view {v} grad2d[{f}]")
        grads_want += r["grads"]
        taint_any |= r["taint"]
    g = st.grads.cpu().numpy()
    for row in range(g.shape[0]):
        assert_block_close(g[row], grads_want[row], GRAD_TOL, mask=~taint_any, what=f"canonical row {row}")


# SH degree 3 on the seeded scene seen by three ring cameras of uneven size
# (6,147 tiles of 16x16): tile shape, LDS batch, backward variant and the
# number of persistent workgroups (each walking many queue items).
BIG = [((16, 16), 256, True, 64, 3), ((16, 16), 256, True, 64, 4), ((16, 16), 256, False, 64, 3),
       ((8, 32), 128, True, 3, 3), ((16, 8), 64, False, 3, 3)]


@pytest.mark.parametrize("tile,batch,cached,blocks,words", BIG,
                         ids=[f"{t[0]}x{t[1]}-b{b}-{'c' if c else 'r'}-grid{g}-w{w}" for t, b, c, g, w in BIG])
def test_views_sh3_ring_sampled_tiles_match_oracle(tile, batch, cached, blocks, words):
    """Every sorted pair in full; compositing, counts and T_final on sampled
    tiles of every view (the heaviest plus seeded random ones) that the
    oracle renders one by one; every Gaussian's 2D gradient per view and
    canonical gradient under a dL/dimage that is non-zero only on those
    tiles, which makes the oracle's sampled-tile backward exact."""
    from paper_2601_17354_amd.batch import BatchedStep, mixed_views
    from oracle.binning import bin_and_sort
    from oracle.projection import project, project_vjp
    from oracle.render import render_backward, render_forward
    scene = synth.spheres_planes_scene(0)
    P = synth.surface_gaussians(scene, 100_000, seed=81, sh_degree=3, logit_sigma=0.5)
    cams = mixed_views(3, sizes=((640, 480), (800, 600), (1024, 768)))
    tw, th = tile
    rng = np.random.default_rng(19)
    ref, dls = [], []
    for v, cam in enumerate(cams):
        W, H = cam["width"], cam["height"]
        proj = project(P, cam, tw, th)
        bins = bin_and_sort(proj)
        lens = bins["ranges"][:, 1] - bins["ranges"][:, 0]
        busy = np.nonzero(lens > 0)[0]
        tiles = sorted({int(np.argmax(lens))} | {int(t) for t in rng.choice(busy, 3, replace=False)})
        fwd = render_forward(proj, bins, cam, tw, th, (0.0, 0.0, 0.0), tiles=tiles)
        TX = (W + tw - 1) // tw
        on = np.zeros((H, W), bool)
        for t in tiles:
            ty, tx = divmod(t, TX)
            on[ty * th:(ty + 1) * th, tx * tw:(tx + 1) * tw] = True
        dl = np.zeros((3, H, W), np.float32)
        dl[:, on] = rng.normal(size=(3, int(on.sum()))).astype(np.float32)
        g2d, taint = render_backward(proj, bins, fwd, dl, "cached")
        grads = project_vjp(P, cam, g2d, proj["visible"])
        ref.append(dict(proj=proj, bins=bins, fwd=fwd, on=on, g2d=g2d, taint=taint, grads=grads, tiles=tiles))
        dls.append(dl)
    say(f"[views-sh3] tile {tile} batch {batch} cached {cached} blocks {blocks}: sampled "
        f"{[r['tiles'] for r in ref]}")
    targets = [torch.zeros((3, c["height"], c["width"]), device=DEV) for c in cams]
    st = BatchedStep(torch.as_tensor(P, device=DEV), 3, cams, targets, tile=tile, batch=batch, cached=cached,
                     blocks=blocks, trace_words=words)
    st.prepare()
    torch.cuda.synchronize()
    assert st.nt > 20 * blocks
    _assert_queue(st, blocks)
    for v in range(len(cams)):
        st.view_slice(st.dl, v).copy_(torch.as_tensor(dls[v], device=DEV))
    st.grads.zero_()
    st.backward_from()
    torch.cuda.synchronize()
    assert st.read_flags() == 0
    _assert_queue(st, blocks)

    npairs = int(st.num_pairs.item())
    keys = st.keys[:npairs].cpu().numpy().view(np.uint64)
    vals = st.values[:npairs].cpu().numpy().astype(np.int64)
    offs = st.views.tile_offsets
    want_k = np.concatenate([r["bins"]["keys"] + (np.uint64(off) << np.uint64(32)) for r, off in zip(ref, offs)])
    want_v = np.concatenate([r["bins"]["values"] for r in ref]).astype(np.int64)
    view_g = np.searchsorted(np.asarray(offs[1:]), (keys >> np.uint64(32)).astype(np.int64), side="right")
    view_w = np.searchsorted(np.asarray(offs[1:]), (want_k >> np.uint64(32)).astype(np.int64), side="right")
    marg = np.stack([r["proj"]["marginal"] for r in ref])
    kg, kw = ~marg[view_g, vals], ~marg[view_w, want_v]
    say(f"  pairs {npairs}, marginal Gaussian-views {int(marg.sum())}")
    np.testing.assert_array_equal(keys[kg], want_k[kw])
    np.testing.assert_array_equal(vals[kg], want_v[kw])

    grads_want = np.zeros_like(P, dtype=np.float64)
    taint_any = np.zeros(P.shape[1], bool)
    for v, r in enumerate(ref):
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


@pytest.mark.parametrize("deg", [0, 3])
def test_project_views_match_per_view_calls(deg):
    # The multi-view projection and its backward run the per-view code once
    # per view in view order, so they reproduce pgs_project / pgs_project_bwd
    # enqueued view by view bit for bit (ten views: two launches of at most
    # eight).
    from paper_2601_17354_amd import binding as B
    scene = synth.spheres_planes_scene(2)
    P = synth.surface_gaussians(scene, 5003, seed=31, sh_degree=deg, logit_sigma=0.5)
    sizes = [(320, 240), (256, 192), (160, 120), (200, 150), (96, 64)]
    ring = synth.ring_cameras(10, 320, 240)
    cams = []
    for i in range(10):
        W, H = sizes[i % len(sizes)]
        c = dict(ring[i])
        c.update(width=W, height=H, cx=W / 2.0, cy=H / 2.0)
        cams.append(c)
    n, V, F = P.shape[1], len(cams), P.shape[0]
    say(f"[views] project_views: n={n} views={V} sh={deg}")
    views = B.ViewBatch(cams, (16, 16))
    params = torch.as_tensor(P, device=DEV)
    proj = torch.zeros((V, n, 16), device=DEV)
    radius = torch.zeros((V, n), dtype=torch.int32, device=DEV)
    rect = torch.zeros((V, 2, n), dtype=torch.int32, device=DEV)
    touched = torch.zeros((V, n), dtype=torch.int32, device=DEV)
    proj1, radius1, rect1, touched1 = (torch.zeros_like(t) for t in (proj, radius, rect, touched))
    B.pgs_project_views(views, params, n, deg, proj, radius, rect, touched)
    for v, cam in enumerate(cams):
        B.pgs_project(params, n, deg, cam, 16, 16, proj1[v], radius1[v], rect1[v], touched1[v])
    torch.cuda.synchronize()
    for a, b in ((proj, proj1), (radius, radius1), (rect, rect1), (touched, touched1)):
        np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())
    vis = (radius > 0).sum().item()
    assert 0 < vis < V * n   # some culled, some visible
    rng = np.random.default_rng(deg + 40)
    g2d = torch.as_tensor(rng.normal(size=(V, n, 16)).astype(np.float32), device=DEV)
    g0 = rng.normal(size=(F, n)).astype(np.float32)
    grads = torch.as_tensor(g0, device=DEV)
    grads1 = torch.as_tensor(g0, device=DEV)
    B.pgs_project_bwd_views(views, params, n, deg, radius, g2d, grads)
    for v, cam in enumerate(cams):
        B.pgs_project_bwd(params, n, deg, cam, radius[v], g2d[v], grads1)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(grads.cpu().numpy(), grads1.cpu().numpy())


def test_adam_step_dev_matches_host_counter():
    from paper_2601_17354_amd import binding as B
    rng = np.random.default_rng(12)
    rows, n = 14, 3001
    p0 = rng.normal(size=(rows, n)).astype(np.float32)
    lr = rng.uniform(1e-4, 1e-2, rows)
    a = [torch.as_tensor(p0, device=DEV)] + [torch.zeros((rows, n), device=DEV) for _ in range(2)]
    b = [torch.as_tensor(p0, device=DEV)] + [torch.zeros((rows, n), device=DEV) for _ in range(2)]
    state = torch.zeros(4, dtype=torch.int32, device=DEV)
    for step in (1, 2, 3):
        g = torch.as_tensor(rng.normal(size=(rows, n)).astype(np.float32), device=DEV)
        B.pgs_adam_step(a[0], g, a[1], a[2], rows, n, lr, step, 0.9, 0.999, 1e-15)
        B.pgs_adam_step_dev(b[0], g, b[1], b[2], rows, n, lr, state, 0.9, 0.999, 1e-15)
    torch.cuda.synchronize()
    assert int(state[0].item()) == 3
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x.cpu().numpy(), y.cpu().numpy())


def _scene_views(n=20000):
    scene = synth.spheres_planes_scene(4)
    P = synth.surface_gaussians(scene, n, seed=60, sh_degree=3, logit_sigma=0.5)
    sizes = [(320, 240), (256, 192), (160, 120)]
    cams = [synth.ring_cameras(12, W, H)[i * 4] for i, (W, H) in enumerate(sizes)]
    return P, cams


def test_graph_replay_matches_eager_steps():
    # Replays of the captured step, with unrelated eager work and host
    # synchronisations in between, against the same steps run eagerly.
    from paper_2601_17354_amd.batch import BatchedStep
    P, cams = _scene_views()
    rng = np.random.default_rng(13)
    targets = [torch.as_tensor(rng.uniform(size=(3, c["height"], c["width"])).astype(np.float32), device=DEV)
               for c in cams]
    say("[views] graph replay vs eager")
    ga = BatchedStep(torch.as_tensor(P, device=DEV), 3, cams, targets, tile=(16, 8), batch=128, extent=4.5)
    eb = BatchedStep(torch.as_tensor(P, device=DEV), 3, cams, targets, tile=(16, 8), batch=128, extent=4.5)
    ga.prepare()
    eb.prepare()
    cap = max(ga.capacity, eb.capacity) * 2
    ga._alloc_pairs(cap)
    eb._alloc_pairs(cap)
    ga.capture()          # runs one eager warm-up step, then records one
    eb.step()
    for k in range(4):
        ga.replay()
        eb.step()
        scratch = torch.randn(1 << 20, device=DEV)
        scratch.mul_(2.0).sum().item()
        torch.cuda.synchronize()
        assert ga.read_flags() == 0 and eb.read_flags() == 0
        la, lb = ga.losses.cpu().numpy(), eb.losses.cpu().numpy()
        say(f"  step {k + 2}: losses graph {la} eager {lb}")
        np.testing.assert_allclose(la, lb, rtol=1e-4)
        pa, pb = ga.params.cpu().numpy(), eb.params.cpu().numpy()
        diff = np.abs(pa - pb)
        # float atomics may order the gradient sums differently; Adam's
        # normalised step bounds what that can move per step
        assert diff.max() <= 2.0 * (k + 2) * 2.5e-2, diff.max()
        assert (diff <= 1e-5).mean() > 0.99
    assert int(ga.adam_state[0].item()) == 5 and int(eb.adam_state[0].item()) == 5


def test_tuner_times_candidates_and_caches_the_choice(tmp_path, monkeypatch):
    from paper_2601_17354_amd.autotune import tune
    monkeypatch.setenv("PGS_TUNE_CACHE", str(tmp_path / "tune.json"))
    P, cams = _views()
    targets = [torch.zeros((3, c["height"], c["width"]), device=DEV) for c in cams]
    params = torch.as_tensor(P, device=DEV)
    cands = [((16, 16), 256), ((8, 8), 64)]
    first = tune(params, 0, cams, targets, steps=2, warmup=1, cands=cands)
    say(f"  tuning table {first['table']}")
    assert not first["cached"] and len(first["table"]) == 2 and all(r["ok"] for r in first["table"])
    assert (tuple(first["tile"]), first["batch"]) in cands
    assert first["ms"] == min(r["ms"] for r in first["table"])
    second = tune(params, 0, cams, targets, steps=2, warmup=1, cands=cands)
    assert second["cached"] and second["tile"] == first["tile"] and second["batch"] == first["batch"]


def test_bin_sort_views_past_one_million_items_matches_per_view_calls():
    # Past 2^20 items the depth sort takes its 2048-key workgroups, with the
    # first pass's histogram written by the depth-key kernel and
    # tiles_touched gathered by the last pass: four views of 300k Gaussians
    # bin and sort to the concatenation of the four single-view lists, whose
    # bit-exactness against the oracle the full-size tests establish.
    from paper_2601_17354_amd import binding as B
    scene = synth.spheres_planes_scene(0)
    P = synth.surface_gaussians(scene, 300_000, seed=1001, sh_degree=0)
    sizes = [(1920, 1440), (1280, 960), (960, 720), (640, 480)]
    ring = synth.ring_cameras(4, 1920, 1440)
    cams = []
    for (W, H), c0 in zip(sizes, ring):
        c = dict(c0)
        c.update(width=W, height=H, fx=c0["fx"] * W / 1920.0, fy=c0["fy"] * W / 1920.0, cx=W / 2.0, cy=H / 2.0)
        cams.append(c)
    n, V = P.shape[1], len(cams)
    assert n * V > (1 << 20)
    say(f"[views] bin_sort_views: n={n} views={V} items={n * V}")
    views = B.ViewBatch(cams, (16, 16))
    params = torch.as_tensor(P, device=DEV)
    proj = torch.zeros((V, n, 16), device=DEV)
    radius = torch.zeros((V, n), dtype=torch.int32, device=DEV)
    rect = torch.zeros((V, 2, n), dtype=torch.int32, device=DEV)
    touched = torch.zeros((V, n), dtype=torch.int32, device=DEV)
    B.pgs_project_views(views, params, n, 0, proj, radius, rect, touched)
    per_view = [int(x) for x in touched.sum(dim=1).cpu()]
    cap = sum(per_view) + 1024
    nt = views.n_tiles

    def buffers(items):
        return (torch.empty(cap, dtype=torch.int64, device=DEV), torch.empty(cap, dtype=torch.int32, device=DEV),
                torch.empty((2, nt), dtype=torch.int32, device=DEV), torch.zeros(1, dtype=torch.int32, device=DEV),
                torch.zeros(1, dtype=torch.int32, device=DEV),
                torch.empty(B.pgs_bin_sort_workspace(items, cap), dtype=torch.uint8, device=DEV))

    keys, values, ranges, num, flags, ws = buffers(n * V)
    B.pgs_bin_sort_views(views, n, proj, rect, touched, cap, keys, values, ranges, num, flags, ws)
    torch.cuda.synchronize()
    assert int(flags.item()) == 0 and int(num.item()) == sum(per_view)
    got_k, got_v, got_r = keys.cpu().numpy(), values.cpu().numpy(), ranges.cpu().numpy()
    base = 0
    for v in range(V):
        k1, v1, r1, num1, f1, ws1 = buffers(n)
        tx = (cams[v]["width"] + 15) // 16
        B.pgs_bin_sort(n, proj[v], rect[v], touched[v], tx, nt, views.tile_offsets[v], cap, k1, v1, r1, num1, f1,
                       ws1)
        torch.cuda.synchronize()
        m = int(num1.item())
        assert int(f1.item()) == 0 and m == per_view[v]
        np.testing.assert_array_equal(got_k[base:base + m], k1.cpu().numpy()[:m])
        np.testing.assert_array_equal(got_v[base:base + m], v1.cpu().numpy()[:m])
        t0, t1 = views.tile_offsets[v], views.tile_offsets[v + 1]
        r1n = r1.cpu().numpy()
        nonempty = r1n[1, t0:t1] > r1n[0, t0:t1]
        np.testing.assert_array_equal(got_r[0, t0:t1][nonempty], r1n[0, t0:t1][nonempty] + base)
        np.testing.assert_array_equal(got_r[1, t0:t1][nonempty], r1n[1, t0:t1][nonempty] + base)
        np.testing.assert_array_equal(got_r[1, t0:t1][~nonempty] - got_r[0, t0:t1][~nonempty], 0)
        base += m
