"""Rotation helpers for the bundle-adjustment oracle (test infrastructure).

skew(v) is the cross-product matrix [v]x (so [v]x u = v x u); exp_so3 is
the Rodrigues formula exp([w]x) = I + sin(t)/t [w]x + (1 - cos t)/t^2 [w]x^2,
t = |w|, with the series limit at t = 0.
"""

from __future__ import annotations

import numpy as np


def skew(v):
    v = np.asarray(v, np.float64)
    K = np.zeros(v.shape[:-1] + (3, 3))
    K[..., 0, 1], K[..., 0, 2], K[..., 1, 2] = -v[..., 2], v[..., 1], -v[..., 0]
    K[..., 1, 0], K[..., 2, 0], K[..., 2, 1] = v[..., 2], -v[..., 1], v[..., 0]
    return K


def exp_so3(w):
    w = np.asarray(w, np.float64)
    t = np.linalg.norm(w, axis=-1)[..., None, None]
    K = skew(w)
    small = t < 1e-8
    ts = np.where(small, 1.0, t)
    a = np.where(small, 1.0 - t * t / 6.0, np.sin(ts) / ts)
    b = np.where(small, 0.5 - t * t / 24.0, (1.0 - np.cos(ts)) / (ts * ts))
    return np.eye(3) + a * K + b * (K @ K)
