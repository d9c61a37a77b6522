"""Pins of the bundle-adjustment oracle (subsection "GPU-Native Global BA as
Mobile MAP Refinement", equation ba_obj, gauge fixing, reduced camera
system) against facts that do not depend on it: finite differences, the
Huber closed forms, scipy's rotation vector map, exact recovery of the
truth on noise-free tracks, the gauge and robustness to outliers."""

import numpy as np
from scipy.spatial.transform import Rotation

import synth
from oracle import _rot, ba


def _prob(seed=0, **kw):
    d = synth.ba_tracks(seed, n_cams=kw.pop("n_cams", 6), n_points=kw.pop("n_points", 120), **kw)
    return d


def test_exp_so3_matches_scipy():
    w = np.random.default_rng(0).normal(size=(20, 3)) * np.r_[1e-9, 1e-4, 0.3, 2.0].repeat(5)[:, None]
    np.testing.assert_allclose(_rot.exp_so3(w), Rotation.from_rotvec(w).as_matrix(), atol=1e-14)


def test_huber_closed_forms():
    delta = 2.0
    s = np.array([0.0, 1.0, 4.0, 9.0, 100.0])
    rho, w = ba.huber(s, delta)
    np.testing.assert_allclose(rho, [0.0, 1.0, 4.0, 2 * 2 * 3 - 4, 2 * 2 * 10 - 4])
    np.testing.assert_allclose(w, [1.0, 1.0, 1.0, 2 / 3, 2 / 10])
    # continuous value and slope at the threshold
    e = 1e-7
    a, wa = ba.huber(np.array([(delta - e) ** 2]), delta)
    b_, wb = ba.huber(np.array([(delta + e) ** 2]), delta)
    assert abs(a[0] - b_[0]) < 1e-6 and abs(wa[0] - wb[0]) < 1e-6


def test_jacobians_match_finite_differences():
    p = _prob(1, noise_px=0.0, outlier_frac=0.0)
    R, c, P = p["R0"], p["c0"], p["P0"]
    Jpose, Jpt = ba.jacobians(p, R, c, P)
    h = 1e-6
    cam, pt = p["obs_cam"], p["obs_pt"]
    for k in range(6):
        d = np.zeros((R.shape[0], 6))
        d[:, k] = h
        Rp, cp, _ = ba.apply_step(R, c, P, d, np.zeros_like(P))
        Rm, cm, _ = ba.apply_step(R, c, P, -d, np.zeros_like(P))
        fd = (ba.residuals(p, Rp, cp, P) - ba.residuals(p, Rm, cm, P)) / (2 * h)
        np.testing.assert_allclose(Jpose[:, :, k], fd, rtol=1e-5, atol=1e-4, err_msg=f"pose {k}")
    for k in range(3):
        d = np.zeros_like(P)
        d[:, k] = h
        fd = (ba.residuals(p, R, c, P + d) - ba.residuals(p, R, c, P - d)) / (2 * h)
        np.testing.assert_allclose(Jpt[:, :, k], fd, rtol=1e-5, atol=1e-4, err_msg=f"point {k}")
    assert cam.size == Jpose.shape[0] and pt.size == Jpt.shape[0]


def test_noise_free_tracks_recover_the_truth():
    # exact measurements and the truth's gauge: the unique optimum is the truth
    p = _prob(2, noise_px=0.0, outlier_frac=0.0)
    (R, c, P), hist, acc = ba.lm(p, p["R0"], p["c0"], p["P0"], delta=2.0, lam=1e-3, iters=12)
    assert hist[-1] < 1e-12 * max(hist[0], 1.0)
    np.testing.assert_allclose(R, p["R_true"], atol=1e-8)
    np.testing.assert_allclose(c, p["c_true"], atol=1e-8)
    np.testing.assert_allclose(P, p["P_true"], atol=1e-8)


def test_step_vanishes_at_the_optimum_and_keeps_the_gauge():
    p = _prob(3, noise_px=0.0, outlier_frac=0.0)
    dpose, dpoint = ba.lm_step(p, p["R_true"], p["c_true"], p["P_true"], 2.0, 1e-3)
    assert np.abs(dpose).max() < 1e-9 and np.abs(dpoint).max() < 1e-9
    dpose, dpoint = ba.lm_step(p, p["R0"], p["c0"], p["P0"], 2.0, 1e-3)
    assert np.abs(dpose[1:]).max() > 1e-6            # the others move
    assert (dpose[0] == 0).all() and dpose[1, 3 + p["gauge_axis"]] == 0


def test_step_solves_the_damped_normal_equations_sparse_assembly():
    p = _prob(4)
    R, c, P = p["R0"], p["c0"], p["P0"]
    H, b = ba.normal_equations(p, R, c, P, 2.0)
    Hs, bs = ba.normal_equations_sparse(p, R, c, P, 2.0)
    np.testing.assert_allclose(Hs.toarray(), H, rtol=1e-12, atol=1e-9 * np.abs(H).max())
    np.testing.assert_allclose(bs, b, rtol=1e-12, atol=1e-9 * np.abs(b).max())
    assert np.allclose(H, H.T)
    # the step zeroes the damped model's gradient on the free parameters
    lam = 1e-2
    dpose, dpoint = ba.lm_step(p, R, c, P, 2.0, lam)
    C = R.shape[0]
    x = np.r_[dpose.ravel(), dpoint.ravel()]
    free = np.r_[ba.free_pose_params(C, p["gauge_axis"]), 6 * C + np.arange(P.size)]
    A = H[np.ix_(free, free)]
    res = (A + lam * np.diag(np.diag(A))) @ x[free] - b[free]
    assert np.abs(res).max() < 1e-8 * np.abs(b).max()


def test_huber_resists_outliers():
    p = _prob(5, n_points=200, noise_px=0.3, outlier_frac=0.05)
    err = {}
    for name, delta in (("huber", 1.0), ("l2", 1e12)):
        (R, c, P), _, _ = ba.lm(p, p["R0"], p["c0"], p["P0"], delta=delta, iters=15)
        err[name] = np.median(np.linalg.norm(P - p["P_true"], axis=1))
    assert err["huber"] < 0.5 * err["l2"], err


def _cam_looking_at(eye, target):
    f = np.asarray(target, float) - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, [0.0, 1.0, 0.0])
    r /= np.linalg.norm(r)
    return np.stack([r, np.cross(f, r), f]), np.asarray(eye, float)


def _problem(cams, points, obs, fx=500.0, cx=320.0):
    R = np.stack([c[0] for c in cams])
    c = np.stack([c[1] for c in cams])
    cam = np.array([o[0] for o in obs])
    pt = np.array([o[1] for o in obs])
    prob = dict(fx=fx, fy=fx, cx=cx, cy=cx, gauge_axis=0, obs_cam=cam, obs_pt=pt,
                obs_uv=np.zeros((len(obs), 2)))
    _, uv = ba.project(R, c, np.asarray(points, float), fx, fx, cx, cx, cam, pt)
    prob["obs_uv"] = uv
    return prob, R, c


def test_retriangulation_recovers_noise_free_points_and_is_the_ray_least_squares():
    p = synth.ba_tracks(3, n_cams=12, n_points=300, noise_px=0.0, outlier_frac=0.0)
    M = p["P_true"].shape[0]
    P, ok = ba.retriangulate(p, p["R_true"], p["c_true"], M)
    assert ok.all()
    np.testing.assert_allclose(P, p["P_true"], atol=1e-9)
    # with noise: the same point as a library least-squares solve of the
    # stacked ray-distance system (I - d d^T)(P - c) = 0
    q = synth.ba_tracks(4, n_cams=12, n_points=50, noise_px=2.0)
    P, ok = ba.retriangulate(q, q["R_true"], q["c_true"], q["P_true"].shape[0])
    d = ba.observation_rays(q, q["R_true"], q["c_true"])
    for j in range(5):
        o = np.nonzero(q["obs_pt"] == j)[0]
        A = np.concatenate([np.eye(3) - np.outer(d[k], d[k]) for k in o])
        b = np.concatenate([(np.eye(3) - np.outer(d[k], d[k])) @ q["c_true"][q["obs_cam"][k]] for k in o])
        np.testing.assert_allclose(P[j], np.linalg.lstsq(A, b, rcond=None)[0], atol=1e-10)


def test_refinement_filters():
    X = np.array([0.0, 0.0, 0.0])
    cams = [_cam_looking_at(np.array([4.0 * np.sin(a), 0.0, 4.0 * np.cos(a)]), X)
            for a in np.radians([0.0, 20.0, 40.0])]
    cams.append(_cam_looking_at(np.array([0.0, 0.0, -4.0]), [0.0, 0.0, -8.0]))  # faces away from X
    cams.append(_cam_looking_at(np.array([4.0 * np.sin(0.01), 0.0, 4.0 * np.cos(0.01)]), X))
    pts = np.array([X, [0.3, 0.2, 0.1], [0.1, -0.2, 0.3], [-0.2, 0.1, 0.0]])
    obs = [(0, 0), (1, 0), (2, 0), (3, 0),          # point 0: three in front, one behind its camera
           (0, 1), (4, 1),                          # point 1: two rays 0.6 degrees apart
           (0, 2), (1, 2), (2, 2),                  # point 2: one measurement moved 40 px
           (0, 3), (1, 3)]                          # point 3: fine
    prob, R, c = _problem(cams, pts, obs)
    prob["obs_uv"][7] += [40.0, 0.0]
    P, kp, ko, st = ba.refine(prob, R, c, 4)
    np.testing.assert_allclose(P[0], X, atol=1e-9)
    assert list(kp) == [True, False, False, True]
    assert list(ko) == [True, True, True, False, False, False, False, False, False, True, True]
    assert st["count"][0] == 3 and st["mean_err"][2] > 4.0 and np.degrees(np.arccos(st["min_cos"][1])) < 1.5


def test_compaction_keeps_order_and_renumbers():
    p = synth.ba_tracks(5, n_cams=8, n_points=80)
    M = p["P_true"].shape[0]
    P, kp, ko, _ = ba.refine(p, p["R0"], p["c0"], M)
    q, Pc = ba.compact(p, P, kp, ko)
    # explicit loop
    new, cams, pts, uvs = {}, [], [], []
    for j in range(M):
        if kp[j]:
            new[j] = len(new)
    for o in range(p["obs_cam"].size):
        if ko[o]:
            cams.append(p["obs_cam"][o])
            pts.append(new[p["obs_pt"][o]])
            uvs.append(p["obs_uv"][o])
    assert list(q["obs_cam"]) == cams and list(q["obs_pt"]) == pts
    np.testing.assert_array_equal(q["obs_uv"], np.array(uvs))
    np.testing.assert_array_equal(Pc, P[kp])
