"""Pins for the oracle's compositing and its backward: closed forms, an
untiled brute-force renderer, invariants, and finite differences."""

import math

import numpy as np
import pytest

import synth
from oracle import pipeline
from oracle.binning import bin_and_sort
from oracle.projection import project
from oracle.render import (ALPHA_MAX, ALPHA_MIN, T_MIN, render_backward,
                           render_forward, replay_entries)


def _one(mu, s, logit, colour):
    P = np.zeros((14, 1))
    P[0:3, 0] = mu
    P[3:6, 0] = math.log(s)
    P[6, 0] = 1.0
    P[10, 0] = logit
    P[11:14, 0] = (np.asarray(colour) - 0.5) * 2 * math.sqrt(math.pi)
    return P


def _cam(W=64, H=48, f=64.0):
    return synth.make_camera(W, H, f, f, W / 2, H / 2, np.eye(3), np.zeros(3))


def test_single_isotropic_gaussian_closed_form():
    # One isotropic Gaussian: C(p) = o exp(-|p - m|^2 / (2 var)) c, var = (f s/z)^2 + 0.3,
    # wherever 1/255 <= alpha <= 0.99 inside its tile rectangle; zero elsewhere.
    # On the optical axis; the principal point is off-centre so the mean is
    # not on a pixel corner.
    f, s, z = 64.0, 0.06, 3.0
    u, v = 30.3, 21.7
    cam = synth.make_camera(64, 48, f, f, u, v, np.eye(3), np.zeros(3))
    mu = (0.0, 0.0, z)
    o_logit, col = 0.4, (0.9, 0.5, 0.2)
    P = _one(mu, s, o_logit, col)
    proj, bins, fwd = pipeline.forward(P, cam)
    var = (f * s / z) ** 2 + 0.3
    o = 1 / (1 + math.exp(-o_logit))
    u, v = float(np.float32(u)), float(np.float32(v))
    ys, xs = np.mgrid[0:48, 0:64]
    a = o * np.exp(-((xs + 0.5 - u) ** 2 + (ys + 0.5 - v) ** 2) / (2 * var))
    x0, y0, x1, y1 = proj["rect"][0]
    inrect = (xs // 16 >= x0) & (xs // 16 <= x1) & (ys // 16 >= y0) & (ys // 16 <= y1)
    a = np.where(inrect & (a >= ALPHA_MIN), np.minimum(a, ALPHA_MAX), 0.0)
    want = a[None] * np.asarray(col)[:, None, None]
    np.testing.assert_allclose(fwd["image"], want, atol=1e-14)
    np.testing.assert_allclose(fwd["T_final"], 1 - a, atol=1e-14)


def test_two_gaussians_composite():
    # Nearer splat first: C = a1 c1 + (1 - a1) a2 c2 at the shared centre.
    cam = _cam()
    P = np.concatenate([_one((0, 0, 3.0), 0.05, 0.3, (1, 0, 0)),
                        _one((0, 0, 2.5), 0.05, -0.2, (0, 0, 1))], 1)
    proj, bins, fwd = pipeline.forward(P, cam)
    a1 = 1 / (1 + math.exp(0.2))      # depth 2.5 is in front
    a2 = 1 / (1 + math.exp(-0.3))
    px = fwd["image"][:, 24, 32]
    # pixel (32, 24) has centre (32.5, 24.5); the mean is at (32, 24)
    var1 = (64 * 0.05 / 2.5) ** 2 + 0.3
    var2 = (64 * 0.05 / 3.0) ** 2 + 0.3
    e1 = a1 * math.exp(-(0.25 + 0.25) / (2 * var1))
    e2 = a2 * math.exp(-(0.25 + 0.25) / (2 * var2))
    np.testing.assert_allclose(px, [(1 - e1) * e2, 0, e1], rtol=1e-13, atol=1e-15)


def _brute_force_image(proj, cam, bg=(0, 0, 0)):
    """Untiled renderer: for every pixel, all Gaussians whose rectangle holds
    the pixel's tile, ordered by (float32 depth, id), composited directly."""
    W, H = cam["width"], cam["height"]
    img = np.zeros((3, H, W))
    order = sorted(np.nonzero(proj["visible"])[0], key=lambda g: (proj["depth32"][g], g))
    for y in range(H):
        for x in range(W):
            tx, ty = x // 16, y // 16
            T, C = 1.0, np.zeros(3)
            for g in order:
                x0, y0, x1, y1 = proj["rect"][g]
                if not (x0 <= tx <= x1 and y0 <= ty <= y1):
                    continue
                dx, dy = proj["u"][g] - (x + 0.5), proj["v"][g] - (y + 0.5)
                pw = -0.5 * (proj["A"][g] * dx * dx + proj["C"][g] * dy * dy) - proj["B"][g] * dx * dy
                if pw > 0:
                    continue
                a = min(ALPHA_MAX, proj["o"][g] * math.exp(pw))
                if a < ALPHA_MIN:
                    continue
                if T * (1 - a) < T_MIN:
                    break
                C += T * a * np.array([proj["r"][g], proj["g"][g], proj["b"][g]])
                T *= 1 - a
            img[:, y, x] = C + T * np.asarray(bg)
    return img


def test_tiled_equals_untiled_brute_force():
    P, _, _ = synth.cfg1_inputs(4, n=300, width=40, height=36, focal=40.0)
    cam = synth.make_camera(40, 36, 40.0, 40.0, 20, 18, np.eye(3), np.zeros(3))
    proj, bins, fwd = pipeline.forward(P, cam, bg=(0.1, 0.2, 0.3))
    want = _brute_force_image(proj, cam, bg=(0.1, 0.2, 0.3))
    np.testing.assert_allclose(fwd["image"], want, rtol=1e-13, atol=1e-15)


def test_transmittance_invariants_and_over_recursion():
    P, cam, _ = synth.cfg1_inputs(0)
    proj, bins, fwd = pipeline.forward(P, cam, bg=(0.2, 0.4, 0.6))
    for tr in fwd["traces"][:20]:
        for p in range(tr["gx"].size):
            js = np.nonzero(tr["contrib"][:, p])[0]
            a = tr["alpha"][js, p]
            T = np.concatenate([[1.0], np.cumprod(1 - a)])
            assert (np.diff(T) <= 0).all() and T.min() >= T_MIN * 0.999 and T.max() <= 1
            # weights sum to one: sum_k T_k a_k + T_K = 1
            assert abs((T[:-1] * a).sum() + T[-1] - 1) < 1e-13
            np.testing.assert_allclose(T[-1], tr["T"][p], rtol=1e-13)
            # the paper's over-recursion from the back reproduces the pixel
            acc = np.array([0.2, 0.4, 0.6])
            for j in js[::-1]:
                g = tr["ids"][j]
                c = np.array([proj["r"][g], proj["g"][g], proj["b"][g]])
                np.testing.assert_allclose(tr["C_in"][j, :, p], acc, rtol=1e-13, atol=1e-15)
                acc = acc * (1 - tr["alpha"][j, p]) + tr["alpha"][j, p] * c
            np.testing.assert_allclose(acc, tr["C"][:, p], rtol=1e-12, atol=1e-15)


def test_replay_entries_shape():
    P, cam, _ = synth.cfg1_inputs(0)
    proj, bins, fwd = pipeline.forward(P, cam)
    ent = replay_entries(fwd, 64, 64)
    assert len(ent) == fwd["count"][64, 64] > 0
    ids = [e[0] for e in ent]
    assert ids == sorted(ids)          # front-to-back = increasing sorted index
    assert all(ALPHA_MIN <= e[1] <= ALPHA_MAX for e in ent)


def test_cached_equals_recompute():
    P, cam, _ = synth.cfg1_inputs(5)
    proj, bins, fwd = pipeline.forward(P, cam, bg=(0.3, 0.1, 0.2))
    G = np.random.default_rng(0).normal(size=(3, 128, 128))
    a, _ = render_backward(proj, bins, fwd, G, "cached")
    b, _ = render_backward(proj, bins, fwd, G, "recompute")
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-12 * np.abs(a).max())


def test_per_step_chain_scalar():
    # The per-step closed forms on a three-splat chain, checked against
    # central differences of C = a1 c1 + (1-a1)(a2 c2 + (1-a2)(a3 c3 + (1-a3) bg)).
    a = np.array([0.3, 0.6, 0.2])
    c = np.array([[0.9, 0.1, 0.4], [0.2, 0.8, 0.3], [0.5, 0.5, 0.9]])
    bg = np.array([0.1, 0.2, 0.3])
    G = np.array([0.7, -1.1, 0.4])

    def comp(a, c):
        acc = bg
        for k in range(2, -1, -1):
            acc = acc * (1 - a[k]) + a[k] * c[k]
        return acc

    # C_in_k: colour behind k; T_k: transmittance in front of k
    acc = bg
    ins = []
    for k in range(2, -1, -1):
        ins.append(acc)
        acc = acc * (1 - a[k]) + a[k] * c[k]
    ins = ins[::-1]
    T = np.concatenate([[1.0], np.cumprod(1 - a)])[:3]
    h = 1e-6
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        fd = G @ (comp(a + e, c) - comp(a - e, c)) / (2 * h)
        assert abs(fd - (T[k] * G) @ (c[k] - ins[k])) < 1e-9
        for ch in range(3):
            cc = c.copy()
            cc[k, ch] += h
            cm = c.copy()
            cm[k, ch] -= h
            fd = G @ (comp(a, cc) - comp(a, cm)) / (2 * h)
            assert abs(fd - a[k] * T[k] * G[ch]) < 1e-9


def _fd_check(f_img, grad_dot, shape, decide, rng, n_dirs=4, support=None, h=1e-6, tol=1e-6):
    """Central-difference dot-product test with frozen branches."""
    base = decide(np.zeros(shape))
    done = 0
    for _ in range(40):
        V = rng.normal(size=shape)
        if support is not None:
            V = V * support
        if not (pipeline.same_decisions(decide(h * V), base) and
                pipeline.same_decisions(decide(-h * V), base)):
            continue
        fd = (f_img(h * V) - f_img(-h * V)) / (2 * h)
        an = grad_dot(V)
        assert abs(fd - an) <= tol * abs(an) + 1e-10, (fd, an)
        done += 1
        if done == n_dirs:
            return
    pytest.fail("no branch-free direction found")


def test_render_backward_fd_2d_params():
    # Perturb the 2D parameters (u, v, A, B, C, o, rgb) directly with the sorted
    # order fixed; the image functional <w, C> against both backward forms.
    P, cam, _ = synth.cfg1_inputs(6, n=200, width=48, height=40, focal=48.0)
    cam = synth.make_camera(48, 40, 48.0, 48.0, 24, 20, np.eye(3), np.zeros(3))
    proj0 = project(P, cam)
    bins = bin_and_sort(proj0)
    fields = ("u", "v", "A", "B", "C", "o", "r", "g", "b")
    w = np.random.default_rng(1).normal(size=(3, 40, 48))
    fwd0 = render_forward(proj0, bins, cam, bg=(0.05, 0.1, 0.15))
    gc, _ = render_backward(proj0, bins, fwd0, w, "cached")
    gr, _ = render_backward(proj0, bins, fwd0, w, "recompute")
    n = proj0["n"]
    vis = proj0["visible"].astype(float)

    def pert(D):
        p = dict(proj0)
        for i, k in enumerate(fields):
            p[k] = proj0[k] + D[i]
        return p

    def f_img(D):
        return (w * render_forward(pert(D), bins, cam, bg=(0.05, 0.1, 0.15))["image"]).sum()

    def decide(D):
        fw = render_forward(pert(D), bins, cam, bg=(0.05, 0.1, 0.15))
        return [np.asarray(t["contrib"]) for t in fw["traces"]] + \
               [np.asarray(t["clamped"] & t["contrib"]) for t in fw["traces"]]

    rng = np.random.default_rng(2)
    scale = np.array([1, 1, 0.01, 0.01, 0.01, 0.1, 0.1, 0.1, 0.1])[:, None]
    _fd_check(f_img, lambda V: (gc * V).sum(), (9, n), decide, rng, support=scale * vis)
    _fd_check(f_img, lambda V: (gr * V).sum(), (9, n), decide, rng, support=scale * vis)


@pytest.mark.parametrize("seed", [0, 1])
def test_full_chain_fd_canonical_params(seed):
    # Image functional through projection, sort and compositing vs the oracle's
    # canonical gradient (render backward + index map + projection VJP).
    P, cam, _ = synth.cfg1_inputs(seed, n=120, width=64, height=64, focal=64.0)
    cam = synth.make_camera(64, 64, 64.0, 64.0, 32, 32, np.eye(3), np.zeros(3))
    P = P.astype(np.float64)
    w = np.random.default_rng(seed + 10).normal(size=(3, 64, 64))
    proj, bins, fwd = pipeline.forward(P, cam)
    grads, _, _ = pipeline.backward(P, cam, proj, bins, fwd, w, "cached")
    grads_r, _, _ = pipeline.backward(P, cam, proj, bins, fwd, w, "recompute")
    np.testing.assert_allclose(grads, grads_r, rtol=1e-11, atol=1e-11 * np.abs(grads).max())
    rng = np.random.default_rng(seed + 20)
    support = np.zeros(P.shape)
    pick = rng.choice(P.shape[1], 15, replace=False)
    support[:, pick] = 1.0

    def f_img(D):
        return (w * pipeline.image(P + D, cam)).sum()

    def decide(D):
        return pipeline.decisions(P + D, cam)

    _fd_check(f_img, lambda V: (grads * V).sum(), P.shape, decide, rng, n_dirs=3, support=support)
