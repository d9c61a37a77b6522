"""Pins for the oracle's KNN and PCA seeding: a library KD-tree, tie rules on a
lattice, planar closed forms, the paper's stated constants."""

import json
import math
import os

import numpy as np
from scipy.spatial import cKDTree

from oracle import seed

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


def test_constants_match_paper():
    c = json.load(open(GOLDEN))
    assert seed.K_N == c["knn_normal_neighbourhood"]["value"]
    assert seed.K_S == c["knn_scale_neighbourhood"]["value"]
    assert seed.INIT_OPACITY == c["initial_opacity"]["value"]


def test_knn_matches_kdtree():
    pts = np.random.default_rng(0).uniform(size=(600, 3)).astype(np.float32)
    q = [0, 5, 77, 599]
    ids, d2 = seed.knn(pts, q)
    tree = cKDTree(pts.astype(np.float64))
    dd, ii = tree.query(pts[q].astype(np.float64), k=17)
    np.testing.assert_array_equal(ids, ii[:, 1:])          # self is the first hit
    np.testing.assert_allclose(np.sqrt(d2), dd[:, 1:], rtol=1e-12)


def test_knn_ties_break_by_index():
    # Integer lattice: many equal distances; the order must be (d2, index).
    g = np.arange(4, dtype=np.float32)
    pts = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    for i in [0, 21, 42]:
        ids, d2 = seed.knn_one(pts, i)
        d = ((pts.astype(np.float64) - pts[i]) ** 2).sum(1)
        want = sorted((float(d[j]), j) for j in range(len(pts)) if j != i)[:16]
        assert [w[1] for w in want] == ids.tolist()


def test_planar_neighbourhood_normal_and_scale():
    # Noise-free points on a tilted plane: the normal is the plane normal and
    # the seeded covariance is s_t^2 (I - n n^T) + (0.1 s_t)^2 n n^T.
    n = np.array([1.0, 2.0, 2.0]) / 3.0
    t1 = np.array([2.0, -1.0, 0.0]) / math.sqrt(5)
    t2 = np.cross(n, t1)
    g = np.arange(-3, 4) * 0.25
    a, b = np.meshgrid(g, g)
    pts = (a.reshape(-1, 1) * t1 + b.reshape(-1, 1) * t2 + np.array([0.3, -0.2, 0.7])).astype(np.float32)
    i = 24                                   # grid centre
    s = seed.seed_points(pts, np.full((len(pts), 3), 0.5), [i])[0]
    assert abs(abs(s["normal"] @ n) - 1) < 1e-6
    assert abs(s["s_t"] - 0.25) < 1e-6      # four neighbours at spacing 0.25
    want = 0.25 ** 2 * (np.eye(3) - np.outer(n, n)) + 0.025 ** 2 * np.outer(n, n)
    np.testing.assert_allclose(s["sigma"], want, atol=1e-7)
    assert abs(s["logit"] - math.log(0.1 / 0.9)) < 1e-15
    np.testing.assert_allclose(s["dc"], 0.0, atol=1e-15)


def test_eigen_decomposition_is_consistent():
    pts = np.random.default_rng(3).normal(size=(200, 3)).astype(np.float32)
    for s in seed.seed_points(pts, np.zeros((200, 3)), [0, 10]):
        lam = s["eig"]
        assert lam[0] <= lam[1] <= lam[2]
        np.testing.assert_allclose(s["cov"] @ s["normal"], lam[0] * s["normal"], atol=1e-12)


def test_sigma_from_params_matches_seed_form():
    n = np.array([0.0, 0.0, 1.0])
    S = seed.sigma_from_params([math.log(0.2), math.log(0.2), math.log(0.02)], [1, 0, 0, 0])
    np.testing.assert_allclose(S, 0.04 * (np.eye(3) - np.outer(n, n)) + 0.0004 * np.outer(n, n), atol=1e-16)


def test_isotropic_seed_is_a_ball_of_the_tangential_scale():
    # r_normal = 1 (the ablation without the disc prior): on the same planar
    # neighbourhood every axis gets s_t, so Sigma = s_t^2 I whatever the normal,
    # while the default ratio keeps the disc of the test above.
    n = np.array([1.0, 2.0, 2.0]) / 3.0
    t1 = np.array([2.0, -1.0, 0.0]) / math.sqrt(5)
    t2 = np.cross(n, t1)
    g = np.arange(-3, 4) * 0.25
    a, b = np.meshgrid(g, g)
    pts = (a.reshape(-1, 1) * t1 + b.reshape(-1, 1) * t2).astype(np.float32)
    iso = seed.seed_points(pts, np.zeros((len(pts), 3)), [24], r_normal=1.0)[0]
    disc = seed.seed_points(pts, np.zeros((len(pts), 3)), [24])[0]
    np.testing.assert_allclose(iso["sigma"], 0.25 ** 2 * np.eye(3), atol=1e-7)
    np.testing.assert_allclose(iso["log_scales"], [math.log(0.25)] * 3, atol=1e-6)
    assert iso["s_t"] == disc["s_t"] and iso["s_n"] == 10 * disc["s_n"]
