"""GPU parity of the remaining entry points and the trace / index-map
properties the paper states."""


import numpy as np
import pytest
import torch

import synth
from gpu_helpers import GRAD_TOL, IMG_TOL, assert_block_close, run_gpu, say
from oracle import adam as o_adam
from oracle import loss as o_loss
from oracle import seed as o_seed

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda")


def _sort_gpu(keys, vals, key_bits, capacity=None):
    from paper_2601_17354_amd import binding as B
    n = len(keys)
    cap = capacity if capacity is not None else max(n, 1)
    k = torch.zeros(cap, dtype=torch.int64, device=DEV)
    v = torch.zeros(cap, dtype=torch.int32, device=DEV)
    if n:
        k[:n] = torch.as_tensor(keys.view(np.int64), device=DEV)
        v[:n] = torch.as_tensor(vals.astype(np.int32), device=DEV)
    cnt = torch.tensor([n], dtype=torch.int32, device=DEV)
    ws = torch.empty(B.pgs_sort_workspace(cap), dtype=torch.uint8, device=DEV)
    B.pgs_sort_pairs(k, v, cnt, cap, key_bits, ws)
    torch.cuda.synchronize()
    return k[:n].cpu().numpy().view(np.uint64), v[:n].cpu().numpy()


@pytest.mark.parametrize("n,bits,dup", [(0, 40, 0), (1, 40, 0), (4095, 37, 50), (4097, 64, 0),
                                         (50000, 46, 1000), (123457, 33, 7)])
def test_sort_pairs_stable_bit_exact(n, bits, dup):
    say(f"[sort] n={n} bits={bits}")
    rng = np.random.default_rng(n + bits)
    hi = np.uint64((1 << bits) - 1) if bits < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)
    keys = rng.integers(0, 2 ** 63, n, dtype=np.int64).view(np.uint64) & hi
    if dup and n:
        keys = keys[rng.integers(0, dup, n)] if dup < n else keys   # many equal keys
    vals = np.arange(n, dtype=np.uint32)
    gk, gv = _sort_gpu(keys, vals, bits)
    order = np.argsort(keys, kind="stable")
    np.testing.assert_array_equal(gk, keys[order])
    np.testing.assert_array_equal(gv.astype(np.int64), order)


def test_sort_respects_device_count_and_capacity():
    rng = np.random.default_rng(1)
    keys = rng.integers(0, 1 << 40, 10000, dtype=np.int64).view(np.uint64)
    gk, gv = _sort_gpu(keys, np.arange(10000, dtype=np.uint32), 40, capacity=20000)
    np.testing.assert_array_equal(gk, np.sort(keys, kind="stable"))


@pytest.mark.parametrize("n_tiles", [10800, 77, 1])
def test_tile_order_is_a_heavy_first_permutation(n_tiles):
    """The launch order only schedules, so it is checked by what it promises:
    a permutation of the view's tiles, non-increasing in 8-pair buckets of
    list length (lengths past the last bucket share it), read at the view's
    tile offset."""
    from paper_2601_17354_amd import binding as B
    rng = np.random.default_rng(n_tiles)
    lens = rng.integers(0, 600, n_tiles)
    lens[rng.random(n_tiles) < 0.02] = 5000
    off = 3
    total = n_tiles + 2 * off
    start = np.zeros(total, np.int64)
    start[off:off + n_tiles] = np.concatenate([[0], np.cumsum(lens)[:-1]])
    end = start.copy()
    end[off:off + n_tiles] += lens
    ranges = torch.as_tensor(np.stack([start, end]).astype(np.int32), device=DEV)
    order = torch.full((n_tiles,), -1, dtype=torch.int32, device=DEV)
    B.pgs_tile_order(ranges, n_tiles, off, total, order)
    got = order.cpu().numpy().astype(np.int64)
    np.testing.assert_array_equal(np.sort(got), np.arange(n_tiles))
    assert np.all(np.diff(np.minimum(lens[got] >> 3, 255)) <= 0)


@pytest.mark.parametrize("W,H,lam", [(64, 48, 0.0), (70, 45, 0.2), (128, 96, 0.2)])
def test_loss_matches_oracle(W, H, lam):
    from paper_2601_17354_amd import binding as B
    rng = np.random.default_rng(W)
    x = rng.uniform(size=(3, H, W)).astype(np.float32)
    y = np.clip(x + rng.normal(0, 0.2, x.shape), 0, 1).astype(np.float32)
    xt, yt = torch.as_tensor(x, device=DEV), torch.as_tensor(y, device=DEV)
    loss = torch.zeros(1, device=DEV)
    dl = torch.zeros_like(xt)
    ws = torch.empty(B.pgs_loss_workspace(W, H), dtype=torch.uint8, device=DEV)
    B.pgs_loss_l1_dssim(xt, yt, W, H, lam, loss, dl, ws)
    torch.cuda.synchronize()
    if lam == 0.0:
        want, wg = o_loss.l1(x, y)
    else:
        want, wg = o_loss.l1_dssim(x, y, lam)
    assert abs(loss.item() - want) <= 1e-5 * abs(want)
    for c in range(3):
        assert_block_close(dl.cpu().numpy()[c], wg[c], 1e-4, what=f"dL/dx[{c}]")


def test_adam_matches_oracle():
    from paper_2601_17354_amd import binding as B
    rng = np.random.default_rng(3)
    rows, n = 14, 1000
    p = rng.normal(size=(rows, n)).astype(np.float32)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    lr = np.linspace(1e-4, 1e-2, rows)
    pt, mt, vt = (torch.as_tensor(a, device=DEV) for a in (p, m, v))
    op, om, ov = p.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    for step in range(1, 4):
        g = rng.normal(size=(rows, n)).astype(np.float32)
        B.pgs_adam_step(pt, torch.as_tensor(g, device=DEV), mt, vt, rows, n, lr, step, 0.9, 0.999, 1e-15)
        # the ABI takes float32 betas: give the oracle the same values
        op, om, ov = o_adam.adam_step(op, g, om, ov, lr.astype(np.float32), step,
                                      b1=float(np.float32(0.9)), b2=float(np.float32(0.999)))
    torch.cuda.synchronize()
    np.testing.assert_allclose(pt.cpu().numpy(), op, rtol=1e-5, atol=1e-6)
    # first moment: a float32 running mean of gradients of scale 1
    np.testing.assert_allclose(mt.cpu().numpy(), om, rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(vt.cpu().numpy(), ov, rtol=1e-5)


def _knn_gpu(pts, k=16):
    from paper_2601_17354_amd import binding as B
    m = len(pts)
    P = torch.as_tensor(np.ascontiguousarray(pts.T, np.float32), device=DEV)
    nbr = torch.empty((k, m), dtype=torch.int32, device=DEV)
    d2 = torch.empty((k, m), dtype=torch.float64, device=DEV)
    ws = torch.empty(B.pgs_knn_workspace(m), dtype=torch.uint8, device=DEV)
    B.pgs_knn(P, m, k, nbr, d2, ws)
    return P, nbr, d2


def test_knn_bit_exact_with_ties():
    g = np.arange(6, dtype=np.float32) * 0.5
    lattice = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    rnd = np.random.default_rng(0).uniform(-1, 4, (700, 3)).astype(np.float32)
    for pts in (lattice, np.concatenate([lattice, rnd])):
        _, nbr, d2 = _knn_gpu(pts)
        torch.cuda.synchronize()
        q = list(range(0, len(pts), 7))
        ids, dd = o_seed.knn(pts, q)
        np.testing.assert_array_equal(nbr.cpu().numpy()[:, q].T, ids)
        np.testing.assert_array_equal(d2.cpu().numpy()[:, q].T, dd)


def test_pca_seed_matches_oracle():
    from paper_2601_17354_amd import binding as B
    scene = synth.spheres_planes_scene(0)
    pts, col = synth.noisy_cloud(scene, 6000, seed=11)
    P, nbr, d2 = _knn_gpu(pts)
    colt = torch.as_tensor(np.ascontiguousarray(col.T), device=DEV)
    out = torch.empty((14, len(pts)), dtype=torch.float32, device=DEV)
    B.pgs_pca_seed(P, colt, len(pts), nbr, d2, 16, 0.1, out)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    q = list(range(0, len(pts), 37))
    want = o_seed.seed_points(pts, col, q)
    checked = 0
    for i, w in zip(q, want):
        np.testing.assert_array_equal(nbr.cpu().numpy()[:, i], w["nbr"])
        np.testing.assert_allclose(o[0:3, i], pts[i], rtol=0)
        np.testing.assert_allclose(o[3:6, i], w["log_scales"], rtol=1e-6, atol=1e-6)
        np.testing.assert_allclose(o[10, i], w["logit"], rtol=1e-6)
        np.testing.assert_allclose(o[11:14, i], w["dc"], rtol=1e-5, atol=1e-6)
        if w["gap"] < 1e-3:
            continue          # normal direction ill-defined
        S = o_seed.sigma_from_params(o[3:6, i], o[6:10, i])
        np.testing.assert_allclose(S, w["sigma"], rtol=1e-4, atol=1e-5 * np.abs(w["sigma"]).max())
        checked += 1
    assert checked > len(q) * 0.9


def test_isotropic_seed_ablation():
    # The "without the seeding" ablation seeds isotropic Gaussians: normal
    # radius 1 instead of 0.1.  Only the normal log-scale may change, and it
    # then equals the two in-plane ones, bit for bit.
    from paper_2601_17354_amd import binding as B
    scene = synth.spheres_planes_scene(0)
    pts, col = synth.noisy_cloud(scene, 3000, seed=12)
    P, nbr, d2 = _knn_gpu(pts)
    colt = torch.as_tensor(np.ascontiguousarray(col.T), device=DEV)
    outs = []
    for r_normal in (0.1, 1.0):
        out = torch.empty((14, len(pts)), dtype=torch.float32, device=DEV)
        B.pgs_pca_seed(P, colt, len(pts), nbr, d2, 16, r_normal, out)
        outs.append(out.cpu().numpy())
    disc, iso = outs
    keep = [r for r in range(14) if r != 5]
    np.testing.assert_array_equal(iso[keep], disc[keep])
    np.testing.assert_array_equal(iso[5], iso[3])
    np.testing.assert_array_equal(iso[4], iso[3])
    assert np.all(disc[5] < disc[3])
    # against the oracle's isotropic seed (r_normal = 1): Sigma = s_t^2 I, so
    # every sampled point is compared, eigen-gap or not
    q = list(range(0, len(pts), 23))
    want = o_seed.seed_points(pts, col, q, r_normal=1.0)
    for i, w in zip(q, want):
        np.testing.assert_allclose(iso[3:6, i], w["log_scales"], rtol=1e-6, atol=1e-6)
        np.testing.assert_allclose(iso[10, i], w["logit"], rtol=1e-6)
        np.testing.assert_allclose(iso[11:14, i], w["dc"], rtol=1e-5, atol=1e-6)
        S = o_seed.sigma_from_params(iso[3:6, i], iso[6:10, i])
        np.testing.assert_allclose(S, w["sigma"], rtol=1e-5, atol=1e-6 * np.abs(w["sigma"]).max())


def test_trace_poison_counter_reset_is_exact():
    # Trace contents beyond the per-wave step counters are never read
    # (replay-cache subsection): a trace pre-filled with NaN entries and
    # all-ones masks, one pre-filled with zeros, and one left holding a
    # different scene's trace from a previous iteration give the same
    # gradients (up to atomic-order noise) and the same image bits.
    P, cam, _ = synth.cfg1_inputs(0)
    P_other, _, _ = synth.cfg1_inputs(5)
    from paper_2601_17354_amd.raster import Rasterizer
    params = torch.as_tensor(P, device=DEV)
    dl = torch.as_tensor(np.random.default_rng(1).normal(size=(3, 128, 128)).astype(np.float32), device=DEV)
    outs, imgs = [], []
    for mode in ("nan", "zero", "stale"):
        R = Rasterizer(P.shape[1], 0, 128, 128, cached=True, capacity=40000, entries=1 << 20)
        if mode == "stale":
            R.forward_checked(torch.as_tensor(P_other, device=DEV), cam)
        else:
            fill = float("nan") if mode == "nan" else 0.0
            R.trace["entry"].fill_(fill)
            R.trace["mask"].fill_(-1 if mode == "nan" else 0)
        R.forward_checked(params, cam)
        assert R.capacity == 40000 and R.entry_capacity == 1 << 20   # no reallocation wiped the poison
        grads = torch.zeros_like(params)
        R.backward(params, cam, dl, grads)
        torch.cuda.synchronize()
        outs.append(grads.cpu().numpy())
        imgs.append(R.image.cpu().numpy())
    assert np.isfinite(outs[0]).all()
    for o, im in zip(outs[1:], imgs[1:]):
        np.testing.assert_array_equal(im, imgs[0])
        for r in range(outs[0].shape[0]):
            assert_block_close(o[r], outs[0][r], 1e-6, what=f"row {r}")


def test_launch_order_changes_no_result():
    # The traced forward launches tiles in natural order, the backward and
    # the untraced forward heavy-first; the order only schedules.  The same
    # traced forward in both orders gives the same image, transmittance,
    # contributor counts and per-pixel entry counts to the bit, and the
    # backward replaying either trace the same gradients up to float-atomic
    # order.
    from paper_2601_17354_amd import binding as B
    from paper_2601_17354_amd.raster import Rasterizer
    P, cam, _ = synth.cfg1_inputs(4, n=6000, width=256, height=192, focal=220.0)
    params = torch.as_tensor(P, device=DEV)
    dl = torch.as_tensor(np.random.default_rng(3).normal(size=(3, 192, 256)).astype(np.float32), device=DEV)
    R = Rasterizer(P.shape[1], 0, 256, 192, cached=True)
    R.forward_checked(params, cam)
    assert R.fwd_order is None and R.tile_order is not None
    res = []
    for order in (None, R.tile_order):
        R.flags.zero_()
        B.pgs_render_fwd(R.W, R.H, R.tw, R.th, R.proj, R.n, R.values, R.ranges, 0, (0.0, 0.0, 0.0), R.image,
                         R.t_final, R.n_contrib, R.trace, R.flags, order)
        assert R.read_flags() == 0
        snap = [t.cpu().numpy().copy() for t in (R.image, R.t_final, R.n_contrib, R.trace["count"])]
        grads = torch.zeros_like(params)
        R.backward(params, cam, dl, grads)
        torch.cuda.synchronize()
        res.append((snap, grads.cpu().numpy()))
    (a, ga), (b, gb) = res
    assert int(np.count_nonzero(a[3])) > 1000
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)
    for r in range(ga.shape[0]):
        assert_block_close(gb[r], ga[r], 1e-6, what=f"row {r}")


def test_index_map_permutation_equivariance():
    # Permuting the canonical order leaves the image unchanged and permutes
    # the gradients (index-mapping subsection).
    P, cam, _ = synth.cfg1_inputs(3)
    perm = np.random.default_rng(0).permutation(P.shape[1])
    dl = np.random.default_rng(2).normal(size=(3, 128, 128)).astype(np.float32)
    a = run_gpu(P, cam, 0, dl_dimage=dl)
    b = run_gpu(np.ascontiguousarray(P[:, perm]), cam, 0, dl_dimage=dl)
    np.testing.assert_array_equal(a["image"], b["image"])
    for r in range(P.shape[0]):
        assert_block_close(b["grads"][r], a["grads"][r][perm], 1e-6, what=f"row {r}")


def test_overflow_flags_and_recovery():
    P, cam, _ = synth.cfg1_inputs(1)
    from paper_2601_17354_amd._lib import PGS_FLAG_CACHE_OVERFLOW, PGS_FLAG_PAIR_OVERFLOW
    from paper_2601_17354_amd.raster import Rasterizer
    params = torch.as_tensor(P, device=DEV)
    R = Rasterizer(P.shape[1], 0, 128, 128, cached=True, capacity=100)
    R.flags.zero_()
    R.forward(params, cam)
    assert R.read_flags() & PGS_FLAG_PAIR_OVERFLOW
    R.forward_checked(params, cam)
    assert R.read_flags() == 0 and R.capacity >= int(R.num_pairs.item())
    ref = run_gpu(P, cam, 0)
    np.testing.assert_array_equal(R.image.cpu().numpy(), ref["image"])
    # a trace declared for fewer pairs than the list holds: the tiles beyond it
    # are not recorded and the device says so
    R.trace["pair_capacity"] = 1000
    R.flags.zero_()
    R.forward(params, cam)
    assert R.read_flags() == PGS_FLAG_CACHE_OVERFLOW
    # too few trace entries: the waves that do not fit are left unrecorded,
    # the counter reports the demand and a checked forward recovers
    R2 = Rasterizer(P.shape[1], 0, 128, 128, cached=True, capacity=R.capacity, entries=500)
    R2.flags.zero_()
    R2.forward(params, cam)
    assert R2.read_flags() == PGS_FLAG_CACHE_OVERFLOW
    need = int(R2.trace["used"].item())
    assert need > 500
    R2.forward_checked(params, cam)
    assert R2.read_flags() == 0 and R2.entry_capacity >= need
    np.testing.assert_array_equal(R2.image.cpu().numpy(), ref["image"])
    assert int(R2.trace["count"].sum().item()) == need


@pytest.mark.parametrize("kind", ["empty", "all-culled", "single", "huge", "flat-edge-on"])
def test_edge_cases(kind):
    from oracle import pipeline
    cam = synth.make_camera(96, 80, 90.0, 90.0, 48.0, 40.0, np.eye(3), np.zeros(3))
    base = synth.random_gaussians(4, 30)
    if kind == "empty":
        P = base[:, :0]
    elif kind == "all-culled":
        P = base.copy()
        P[2] = -3.0
    elif kind == "single":
        P = base[:, :1].copy()
        P[0:3, 0] = (0.05, -0.02, 3.0)
        P[3:6, 0] = -2.5
    elif kind == "huge":
        P = base[:, :5].copy()
        P[3:6, 0] = 0.5          # covers every tile
        P[2, 0] = 2.0
    else:
        P = base.copy()
        P[5] = P[3] - 6.0        # one scale 400x thinner than the others
    say(f"[edge] {kind} n={P.shape[1]}")
    dl = np.random.default_rng(0).normal(size=(3, 80, 96)).astype(np.float32)
    g = run_gpu(P, cam, 0, dl_dimage=dl) if P.shape[1] else None
    if P.shape[1] == 0:
        from paper_2601_17354_amd.raster import Rasterizer
        R = Rasterizer(0, 0, 96, 80)
        R.forward_checked(torch.zeros((14, 1), device=DEV), cam)
        torch.cuda.synchronize()
        assert (R.image.cpu().numpy() == 0).all() and int(R.num_pairs.item()) == 0
        return
    proj, bins, fwd = pipeline.forward(P, cam)
    og, _, taint = pipeline.backward(P, cam, proj, bins, fwd, dl)
    assert g["num_pairs"] == bins["num_pairs"]
    np.testing.assert_array_equal(g["values"].astype(np.int64), bins["values"])
    ok = ~fwd["marginal"]
    for c in range(3):
        assert_block_close(g["image"][c], fwd["image"][c], IMG_TOL, mask=ok, what=f"image[{c}]")
    floor = GRAD_TOL * 1e-6 * np.abs(og).max()
    for r in range(og.shape[0]):
        assert_block_close(g["grads"][r], og[r], GRAD_TOL, mask=~taint, what=f"row {r}", atol=floor)


def test_atomic_scatter_adds_one_per_target_and_field():
    # the float-atomic reference: every target adds 1 to fields 0..8 of its
    # record, out-of-range targets are skipped, fields 9..15 are untouched
    from paper_2601_17354_amd import binding as B
    rng = np.random.default_rng(21)
    n_rec, n_t = 5000, 70001
    tg = rng.integers(0, n_rec + 10, n_t).astype(np.int32)
    rec = torch.full((n_rec, 16), 0.5, device=DEV)
    B.pgs_atomic_scatter(rec, n_rec, torch.as_tensor(tg, device=DEV), n_t)
    got = rec.cpu().numpy()
    want = 0.5 + np.bincount(tg[tg < n_rec], minlength=n_rec).astype(np.float64)
    for f in range(9):
        np.testing.assert_array_equal(got[:, f], want)
    assert (got[:, 9:] == 0.5).all()


@pytest.mark.parametrize("case", ["plane", "duplicates", "outlier", "tiny", "scene300k"])
def test_knn_grid_search_cases(case):
    # the grid search against the oracle's brute force with its tie rule:
    # a flat box axis, exact duplicates, a far outlier that stretches the grid,
    # the fewest points allowed, and the benchmark cloud's size (sampled
    # queries)
    rng = np.random.default_rng(31)
    k = 16
    if case == "plane":
        pts = np.c_[rng.uniform(size=(3000, 2)), np.full(3000, 0.25)].astype(np.float32)
    elif case == "duplicates":
        pts = np.repeat(rng.uniform(size=(400, 3)).astype(np.float32), 5, axis=0)
    elif case == "outlier":
        pts = np.r_[rng.normal(size=(4000, 3)) * 0.01, [[60.0, -40.0, 25.0]]].astype(np.float32)
    elif case == "tiny":
        pts = (rng.uniform(size=(17, 3)) * 1e-3 + 5.0).astype(np.float32)
    else:
        pts = synth.noisy_cloud(synth.spheres_planes_scene(0), 300_000, seed=2000)[0].astype(np.float32)
    say(f"[knn] {case}: {len(pts)} points")
    _, nbr, d2 = _knn_gpu(pts, k)
    torch.cuda.synchronize()
    q = list(range(0, len(pts), max(1, len(pts) // 150)))
    if case == "outlier":
        q.append(len(pts) - 1)
    ids, dd = o_seed.knn(pts, q, k)
    np.testing.assert_array_equal(nbr.cpu().numpy()[:, q].T, ids)
    np.testing.assert_array_equal(d2.cpu().numpy()[:, q].T, dd)
