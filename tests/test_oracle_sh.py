"""Pins for the oracle's real SH basis: a library routine and orthonormality."""

import math

import numpy as np
import torch
from scipy.special import lpmv

from oracle.sh import sh_basis


def _dirs(n, seed):
    d = np.random.default_rng(seed).normal(size=(n, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def test_matches_associated_legendre_library():
    # scipy's lpmv includes the Condon-Shortley phase; build the real basis
    # from it in spherical coordinates and compare.
    d = _dirs(200, 0)
    Y = sh_basis(torch.as_tensor(d), 3).numpy()
    x, y, z = d.T
    phi = np.arctan2(y, x)
    k = 0
    for l in range(4):
        for m in range(-l, l + 1):
            am = abs(m)
            K = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
            P = lpmv(am, l, z)
            if m == 0:
                ref = K * P
            elif m > 0:
                ref = math.sqrt(2) * K * P * np.cos(am * phi)
            else:
                ref = math.sqrt(2) * K * P * np.sin(am * phi)
            np.testing.assert_allclose(Y[:, k], ref, atol=1e-13)
            k += 1


def test_orthonormal_by_quadrature():
    # Gauss-Legendre in z (exact to degree 39) x uniform phi (exact for
    # trigonometric degree < 16): products of degree-3 harmonics integrate exactly.
    zn, wz = np.polynomial.legendre.leggauss(20)
    nphi = 16
    phi = 2 * np.pi * np.arange(nphi) / nphi
    Z, PHI = np.meshgrid(zn, phi, indexing="ij")
    Wt = (wz[:, None] * (2 * np.pi / nphi)) * np.ones_like(PHI)
    s = np.sqrt(1 - Z ** 2)
    d = np.stack([s * np.cos(PHI), s * np.sin(PHI), Z], -1).reshape(-1, 3)
    Y = sh_basis(torch.as_tensor(d), 3).numpy()
    G = (Y * Wt.reshape(-1, 1)).T @ Y
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_degree_one_is_condon_shortley_signed():
    # Y_1,-1 = -c y, Y_1,0 = c z, Y_1,1 = -c x with c = sqrt(3/(4 pi))
    d = _dirs(10, 3)
    Y = sh_basis(torch.as_tensor(d), 1).numpy()
    c = math.sqrt(3 / (4 * math.pi))
    np.testing.assert_allclose(Y[:, 0], 1 / (2 * math.sqrt(math.pi)), rtol=1e-15)
    np.testing.assert_allclose(Y[:, 1:], c * np.stack([-d[:, 1], d[:, 2], -d[:, 0]], 1), atol=1e-15)
