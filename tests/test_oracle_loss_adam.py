"""Pins for the oracle's losses and Adam: direct windowed sums, identities,
finite differences and closed-form steps."""

import math

import numpy as np

from oracle import adam, loss


def test_l1_closed_form():
    x = np.array([[[0.2, 0.5], [0.9, 0.1]]] * 3)
    y = np.array([[[0.1, 0.5], [1.0, 0.4]]] * 3)
    v, g = loss.l1(x, y)
    assert abs(v - (0.1 + 0 + 0.1 + 0.3) / 4) < 1e-15
    np.testing.assert_array_equal(g[0], np.array([[1, 0], [-1, -1]]) / 12.0)


def test_ssim_of_identical_images_is_one_with_zero_gradient():
    x = np.random.default_rng(0).uniform(size=(3, 20, 23))
    v, g = loss.ssim(x, x)
    assert abs(v - 1.0) < 1e-14
    assert np.abs(g).max() < 1e-13


def test_ssim_map_matches_direct_window_sums():
    # Interior and border pixels by explicit loops over the 11x11 window with
    # zero padding, written from the definition.
    rng = np.random.default_rng(1)
    x = rng.uniform(size=(3, 18, 21))
    y = np.clip(x + rng.normal(0, 0.1, x.shape), 0, 1)
    S = loss.ssim_map(x, y)
    g1 = loss.gaussian_window()
    w = np.outer(g1, g1)
    assert abs(w.sum() - 1) < 1e-15
    for ch, r, c in [(0, 9, 10), (1, 0, 0), (2, 17, 5), (0, 3, 20)]:
        sx = sy = sxx = syy = sxy = 0.0
        for i in range(11):
            for j in range(11):
                rr, cc = r + i - 5, c + j - 5
                if 0 <= rr < 18 and 0 <= cc < 21:
                    a, b = x[ch, rr, cc], y[ch, rr, cc]
                    sx += w[i, j] * a
                    sy += w[i, j] * b
                    sxx += w[i, j] * a * a
                    syy += w[i, j] * b * b
                    sxy += w[i, j] * a * b
        vx, vy, cxy = sxx - sx * sx, syy - sy * sy, sxy - sx * sy
        want = ((2 * sx * sy + 1e-4) * (2 * cxy + 9e-4)) / ((sx * sx + sy * sy + 1e-4) * (vx + vy + 9e-4))
        assert abs(S[ch, r, c] - want) < 1e-13


def test_ssim_gradient_fd():
    rng = np.random.default_rng(2)
    x = rng.uniform(size=(3, 14, 15))
    y = rng.uniform(size=(3, 14, 15))
    _, g = loss.ssim(x, y)
    for _ in range(3):
        V = rng.normal(size=x.shape)
        h = 1e-6
        fd = (loss.ssim(x + h * V, y)[0] - loss.ssim(x - h * V, y)[0]) / (2 * h)
        an = (g * V).sum()
        assert abs(fd - an) <= 1e-6 * abs(an) + 1e-12


def test_l1_dssim_combination():
    rng = np.random.default_rng(3)
    x, y = rng.uniform(size=(2, 3, 12, 12))
    v, g = loss.l1_dssim(x, y)
    l1v, l1g = loss.l1(x, y)
    sv, sg = loss.ssim(x, y)
    assert abs(v - (0.8 * l1v + 0.2 * (1 - sv))) < 1e-15
    np.testing.assert_allclose(g, 0.8 * l1g - 0.2 * sg, atol=1e-16)


def test_psnr_constant_images():
    x = np.full((3, 4, 4), 0.5)
    y = np.full((3, 4, 4), 0.6)
    assert abs(loss.psnr(x, y) - 10 * math.log10(1 / 0.01)) < 1e-12


def test_adam_first_step_closed_form():
    # After one step m_hat = g and v_hat = g^2, so the update is -lr g / (|g| + eps).
    rng = np.random.default_rng(4)
    p = rng.normal(size=(3, 5))
    g = rng.normal(size=(3, 5))
    lr = np.array([0.1, 0.01, 0.001])
    p1, m1, v1 = adam.adam_step(p, g, np.zeros_like(p), np.zeros_like(p), lr, 1)
    np.testing.assert_allclose(p1, p - lr[:, None] * g / (np.abs(g) + 1e-15), rtol=1e-14)
    np.testing.assert_allclose(m1, 0.1 * g, rtol=1e-14)
    np.testing.assert_allclose(v1, 0.001 * g * g, rtol=1e-14)


def test_adam_constant_gradient_moves_lr_per_step():
    # With a constant gradient the bias-corrected ratio is exactly sign(g)
    # (up to eps), so each step moves every parameter by lr.
    p = np.zeros((1, 3))
    g = np.array([[2.0, -0.5, 3.0]])
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    for t in range(1, 6):
        p, m, v = adam.adam_step(p, g, m, v, np.array([0.01]), t)
    np.testing.assert_allclose(p, -0.05 * np.sign(g), rtol=1e-12)
