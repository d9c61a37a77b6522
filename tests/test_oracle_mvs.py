"""Pins of the multi-view stereo oracle (CPU): brute force on tiny inputs,
closed forms, library routines and the exact geometry of ray-cast views."""

import itertools

import numpy as np

import synth
from oracle import mvs


def _census_brute(g):
    H, W = g.shape
    out = np.zeros((H, W), np.uint64)
    for y in range(H):
        for x in range(W):
            v, b = 0, 0
            for dy in range(-3, 4):
                for dx in range(-3, 4):
                    if dy == 0 and dx == 0:
                        continue
                    qy, qx = min(max(y + dy, 0), H - 1), min(max(x + dx, 0), W - 1)
                    if int(g[qy, qx]) < int(g[y, x]):
                        v |= 1 << b
                    b += 1
            out[y, x] = v
    return out


def test_census_matches_per_pixel_brute_force():
    g = np.random.default_rng(0).integers(0, 256, (9, 11)).astype(np.uint8)
    g[2:5, 3:6] = 77                                   # a flat patch: ties set no bit
    np.testing.assert_array_equal(mvs.census(g), _census_brute(g))
    assert mvs.CENSUS_BITS == 48


def test_popcount_against_python():
    x = np.random.default_rng(1).integers(0, 2 ** 63, 500, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    assert (mvs.popcount64(x) == np.array([bin(int(v)).count("1") for v in x])).all()


def test_planes_uniform_in_inverse_depth():
    inv, h = mvs.plane_inverse_depths(2.0, 10.0, 64)
    assert abs(1.0 / inv[0] - 10.0) < 1e-12 and abs(1.0 / inv[-1] - 2.0) < 1e-12
    np.testing.assert_allclose(np.diff(inv), h, rtol=1e-12)


def test_sweep_to_the_same_camera_is_the_identity():
    cam = synth.ring_cameras(60, 64, 48)[5]
    ys, xs = np.mgrid[0:48, 0:64]
    qx, qy, ok = mvs.sweep_pixels(cam, cam, 1.0, 20.0, 16, xs.ravel(), ys.ravel())
    assert ok.all()
    assert (qx == xs.ravel()[None]).all() and (qy == ys.ravel()[None]).all()


def test_sweep_at_the_true_depth_lands_on_the_true_projection():
    """Pixels of a ray-cast view, swept at a plane through their exact depth,
    land where the scene point projects in the other view (projection written
    here from the look-at construction: camera axes and focal length)."""
    W, H = 160, 120
    cams = synth.ring_cameras(60, W, H)
    _, dep = synth.textured_views(synth.spheres_planes_scene(0), [cams[0]], seed=1)
    rng = np.random.default_rng(2)
    ys, xs = np.nonzero(dep[0] > 0)
    pick = rng.choice(xs.size, 40, replace=False)
    for i in pick:
        x, y, z = int(xs[i]), int(ys[i]), float(dep[0][ys[i], xs[i]])
        # one plane through z: d_min = d_max is degenerate, so take the
        # first plane (the farthest) at z
        qx, qy, ok = mvs.sweep_pixels(cams[0], cams[3], z / 2.0, z, 2, [x], [y])
        c0, c3 = cams[0], cams[3]
        ang0, ang3 = 0.0, 2 * np.pi * 3 / 60
        eye0 = np.array([4.5 * np.sin(ang0), 0.8, 4.5 * np.cos(ang0)])
        eye3 = np.array([4.5 * np.sin(ang3), 0.8, 4.5 * np.cos(ang3)])

        def axes(eye):
            f = np.array([0.0, 0.3, 0.0]) - eye
            f /= np.linalg.norm(f)
            r = np.cross(f, [0.0, 1.0, 0.0])
            r /= np.linalg.norm(r)
            return r, np.cross(f, r), f
        r0, d0, f0 = axes(eye0)
        P = eye0 + z * ((x - c0["cx"]) / c0["fx"] * r0 + (y - c0["cy"]) / c0["fy"] * d0 + f0)
        r3, d3, f3 = axes(eye3)
        q = P - eye3
        u = c3["fx"] * (q @ r3) / (q @ f3) + c3["cx"]
        v = c3["fy"] * (q @ d3) / (q @ f3) + c3["cy"]
        if 1 <= u <= W - 2 and 1 <= v <= H - 2:
            assert ok[0, 0]
            assert abs(qx[0, 0] - u) <= 0.5 + 1e-3 and abs(qy[0, 0] - v) <= 0.5 + 1e-3, (x, y, u, v)


def _line_energy_brute(C, p1, p2):
    """E(s, k): minimum over label sequences ending at step s with label k of
    the data costs plus the smoothness penalties (0, p1 for a step of one
    plane, p2 beyond), by enumeration."""
    S, D = C.shape
    E = np.full((S, D), np.inf)
    for s in range(S):
        for seq in itertools.product(range(D), repeat=s + 1):
            e = sum(C[i, seq[i]] for i in range(s + 1))
            for i in range(1, s + 1):
                j = abs(seq[i] - seq[i - 1])
                e += 0 if j == 0 else (p1 if j == 1 else p2)
            E[s, seq[-1]] = min(E[s, seq[-1]], e)
    return E


def test_sgm_path_is_the_min_cost_labelling_up_to_a_per_step_constant():
    rng = np.random.default_rng(3)
    for p1, p2 in [(4, 32), (1, 3), (5, 5)]:
        C = rng.integers(0, 49, (5, 4))
        L = mvs.sgm_path(C[None], p1, p2)[0]
        E = _line_energy_brute(C, p1, p2)
        np.testing.assert_array_equal(L - L.min(1, keepdims=True), E - E.min(1, keepdims=True))


def test_sgm_without_penalties_is_four_times_the_cost():
    C = np.random.default_rng(4).integers(0, 49, (6, 7, 8)).astype(np.uint8)
    np.testing.assert_array_equal(mvs.sgm(C, 0, 0), 4 * C.astype(np.int64))


def test_sgm_paths_run_in_all_four_directions():
    """A single cheap plane at one pixel spreads along its row and column
    (both ways) and nowhere else."""
    C = np.full((5, 6, 4), 10, np.uint8)
    C[2, 3, 1] = 0
    S = mvs.sgm(C, 1, 100)
    base = mvs.sgm(np.full((5, 6, 4), 10, np.uint8), 1, 100)
    changed = (S != base).any(2)
    want = np.zeros((5, 6), bool)
    want[2, :] = True
    want[:, 3] = True
    np.testing.assert_array_equal(changed, want)


def test_winner_rules_and_parabola():
    D = 8
    S = np.full((1, 6, D), 100, np.int64)
    S[0, 0, 3] = 10                              # clear winner, S2 = 100
    S[0, 1, [2, 5]] = 10                         # tie: the smaller plane wins, ambiguous: rejected
    S[0, 2, 0] = 1                               # winner on the first plane: rejected
    S[0, 3, 3], S[0, 3, 6] = 70, 99              # 1 - 70/99 < 0.4: rejected
    S[0, 4, 3], S[0, 4, 6] = 59, 99              # 1 - 59/99 > 0.4: kept
    S[0, 5, 1:4] = [25, 1, 9]                    # (4k - 13)^2 about k = 2: vertex 2.25
    S[0, 5, 0], S[0, 5, 4:] = 49, 81
    depth, conf, k = mvs.winner(S, 1.0, 8.0)
    assert list(k[0]) == [3, 2, 0, 3, 3, 2]
    assert [bool(v) for v in depth[0] > 0] == [True, False, False, False, True, True]
    inv, h = mvs.plane_inverse_depths(1.0, 8.0, D)
    assert abs(float(depth[0, 5]) - 1.0 / (1.0 / 8.0 + 2.25 * h)) < 1e-6
    assert abs(float(depth[0, 0]) - 1.0 / inv[3]) < 1e-6    # symmetric neighbours: no shift
    assert abs(float(conf[0, 0]) - 0.9) < 1e-7


def test_quantile_matches_numpy_and_range_brackets_the_depths():
    rng = np.random.default_rng(5)
    for n in (1, 2, 7, 1000):
        z = np.sort(rng.uniform(1, 9, n))
        for p in (0.05, 0.5, 0.95):
            assert abs(mvs.quantile_sorted(z, p) - np.quantile(z, p)) <= 1e-12 * 9
    cam = synth.ring_cameras(60, 320, 240)[0]
    pts = synth.sample_surface(synth.spheres_planes_scene(0), 4000, 1)[0]
    lo, hi = mvs.depth_range(cam, pts)
    z, u, v = mvs.point_depths(cam, pts)
    ins = (z > 0) & (u >= -0.5) & (u < 319.5) & (v >= -0.5) & (v < 239.5)
    assert abs(lo - 0.5 * np.quantile(z[ins], 0.05)) < 1e-9 and abs(hi - 1.5 * np.quantile(z[ins], 0.95)) < 1e-9
    assert 0 < lo < z[ins].min() * 1.01 or lo < np.quantile(z[ins], 0.05)
    # points behind the camera or outside the image do not count
    assert mvs.depth_range(cam, np.array([[0.0, 0.8, 20.0]])) == (0.0, 0.0)


def test_reference_choice_on_the_ring():
    cams = synth.ring_cameras(60, 320, 240)
    c = [-np.asarray(k["viewmat"][:, :3], np.float64).T @ np.asarray(k["viewmat"][:, 3], np.float64)
         for k in cams]
    b2 = np.linalg.norm(c[2] - c[0])
    # the baseline term alone (alpha_min above every angle): the second neighbours
    ref, sc = mvs.select_reference(cams, 0, b2, 0.05, np.pi)
    assert ref in (2, 58)
    assert sc[0] == -np.inf
    # angle term: with b_target far from every baseline the Gaussian is flat,
    # so the widest viewing angle (the opposite camera) wins
    ref, _ = mvs.select_reference(cams, 0, 0.0, 1e3, np.radians(1.0))
    assert ref == 30


def test_fused_points_lie_on_the_scene():
    """Back-projected exact depths of a ray-cast view lie on the scene's
    spheres and planes."""
    scene = synth.spheres_planes_scene(0)
    cam = synth.ring_cameras(60, 96, 72)[7]
    _, dep = synth.textured_views(scene, [cam], seed=1)
    P = mvs.fuse(cam, dep[0]).astype(np.float64)
    assert P.shape == (int((dep[0] > 0).sum()), 3)
    ds = np.abs(np.linalg.norm(P[:, None] - scene.centres[None], axis=2) - scene.radii[None]).min(1)
    dp = np.min(np.stack([np.abs((P - o) @ n) for (o, _, _, n, _, _) in scene.planes], 1), 1)
    assert np.percentile(np.minimum(ds, dp), 99) < 2e-5 * 10


def test_depth_maps_of_ray_cast_views_match_the_exact_depth():
    W, H = 320, 240
    scene = synth.spheres_planes_scene(0)
    cams = synth.ring_cameras(60, W, H)
    g, dep = synth.textured_views(scene, [cams[0], cams[1]], seed=5)
    pts = synth.sample_surface(scene, 5000, 1)[0]
    lo, hi = mvs.depth_range(cams[0], pts)
    r = mvs.depth_map(g[0], g[1], cams[0], cams[1], lo, hi, 64, 4, 32)
    keep = (r["depth"] > 0) & (dep[0] > 0)
    rel = np.abs(r["depth"][keep] - dep[0][keep]) / dep[0][keep]
    assert keep.mean() > 0.3
    assert np.median(rel) < 0.01 and (rel < 0.03).mean() > 0.9
    # a wrong reference (its mirror image) gives garbage
    bad = mvs.depth_map(g[0], g[1][:, ::-1].copy(), cams[0], cams[1], lo, hi, 64, 4, 32)
    kb = (bad["depth"] > 0) & (dep[0] > 0)
    relb = np.abs(bad["depth"][kb] - dep[0][kb]) / dep[0][kb]
    assert kb.mean() < 0.1 and np.median(relb) > 0.1


def _sweep_f32(cam_t, cam_r, d_min, d_max, n_planes, xs, ys, reverse):
    """The sweep's formulas evaluated in float32 (numpy), with the 3x3
    transform's sums in one of two orders: a stand-in for any float32
    implementation, to check what the oracle's marginal cells must cover."""
    f32 = np.float32
    fx, fy, cx, cy, _, _ = mvs.cam64(cam_t)
    fxr, fyr, cxr, cyr = (f32(v) for v in mvs.cam64(cam_r)[:4])
    M, m = (a.astype(f32) for a in mvs.relative_pose(cam_t, cam_r))
    inv, _ = mvs.plane_inverse_depths(d_min, d_max, n_planes)
    d = (1.0 / inv).astype(f32)[:, None]
    a = ((np.asarray(xs, np.float64) - cx) / fx).astype(f32)[None, :]
    b = ((np.asarray(ys, np.float64) - cy) / fy).astype(f32)[None, :]
    X, Y, Z = d * a, d * b, np.broadcast_to(d, (d.shape[0], a.shape[1]))

    def row(r):
        if reverse:
            return m[r] + (M[r, 2] * Z + (M[r, 1] * Y + M[r, 0] * X))
        return ((M[r, 0] * X + M[r, 1] * Y) + M[r, 2] * Z) + m[r]
    xr, yr, zr = row(0), row(1), row(2)
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        u = np.floor(fxr * (xr / zr) + cxr + f32(0.5))
        v = np.floor(fyr * (yr / zr) + cyr + f32(0.5))
    Wr, Hr = cam_r["width"], cam_r["height"]
    ok = (zr > 0) & (u >= 0) & (u <= Wr - 1) & (v >= 0) & (v <= Hr - 1)
    return np.where(ok, u, 0).astype(np.int64), np.where(ok, v, 0).astype(np.int64), ok


def test_marginal_cells_cover_every_float32_disagreement():
    """The float64 sweep's marginal cells hold every cell where a float32
    evaluation (two summation orders) lands on another pixel or another
    validity, and they are few."""
    W, H = 320, 240
    cams = synth.ring_cameras(60, W, H)
    ys, xs = np.mgrid[0:H:3, 0:W:3]
    xs, ys = xs.ravel(), ys.ravel()
    total = flagged = 0
    for t, r, lo, hi in [(0, 1, 2.0, 9.0), (7, 9, 1.0, 14.0), (30, 28, 0.5, 30.0), (12, 45, 2.0, 8.0)]:
        qx, qy, ok, marg = mvs.sweep_pixels(cams[t], cams[r], lo, hi, 64, xs, ys, with_margin=True)
        for rev in (False, True):
            fx_, fy_, fok = _sweep_f32(cams[t], cams[r], lo, hi, 64, xs, ys, rev)
            differ = (fok != ok) | (ok & ((fx_ != qx) | (fy_ != qy)))
            assert not (differ & ~marg).any(), (t, r, rev, int((differ & ~marg).sum()))
            flagged += int(differ.sum())
        total += marg.size
        assert marg.mean() < 0.01, marg.mean()
    assert flagged > 0          # the float32 evaluations do disagree somewhere
