"""KNN local surface statistics and disc-like covariance seeding (oracle).

PocketGS Sec. "Prior-Conditioned Gaussian Parameterization":
  * two neighbourhoods per point p_i: K_n = 16 for the normal, K_s = 3 for
    the tangential scale;
  * local covariance C_i = (1/K_n) sum_k (p_ik - pbar_i)(p_ik - pbar_i)^T with
    pbar_i the neighbourhood centroid (equation for C_i);
  * normal n_i = eigenvector of the smallest eigenvalue of C_i;
  * s_t = mean distance to the K_s nearest neighbours (equation for s_t),
    s_n = r_normal s_t, scales stored as logs;
  * rotation puts the Gaussian's local z on n_i; opacity = logit(0.1).

Readings (the paper is silent): neighbours exclude the point itself, use the
Euclidean distance, and break ties by the smaller index; the K_s = 3
neighbours are the first three of the sixteen; r_normal = 0.1.  The in-plane
rotation is free because both tangential scales equal s_t, so the seeded
covariance is compared as Sigma = s_t^2 (I - n n^T) + s_n^2 n n^T, which does
not depend on the tangent basis or the sign of n.  Colour: degree-0
coefficient (rgb - 1/2) / Y_00 from the point's colour.

Squared distances are formed in float64 from the float32 coordinates as
((dx*dx) + (dy*dy)) + (dz*dz), which fixes every rounding, so a float64
implementation with the same operation order reproduces the neighbour sets
bit for bit.
"""

from __future__ import annotations

import math

import numpy as np

K_N = 16
K_S = 3
R_NORMAL = 0.1
INIT_OPACITY = 0.1


def sq_dists(points, i):
    P = np.asarray(points, np.float32).astype(np.float64)
    d = P - P[i]
    return (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]


def knn_one(points, i, k=K_N):
    """Indices and squared distances of the k nearest other points of point i."""
    d2 = sq_dists(points, i)
    idx = np.arange(d2.size)
    keep = idx != i
    order = np.lexsort((idx[keep], d2[keep]))[:k]
    return idx[keep][order], d2[keep][order]


def knn(points, queries=None, k=K_N):
    """Brute force over all points for each query index (default: all)."""
    M = len(points)
    if queries is None:
        queries = range(M)
    ids, d2s = [], []
    for i in queries:
        a, b = knn_one(points, int(i), k)
        ids.append(a)
        d2s.append(b)
    return np.asarray(ids, np.int64), np.asarray(d2s)


def seed_from_neighbours(points, i, nbr_idx, nbr_d2, r_normal=R_NORMAL):
    """Local statistics and the seeded Gaussian of point i.  r_normal is the
    normal-to-tangential scale ratio; r_normal = 1 gives the isotropic seed of
    the ablation without the disc prior (Table 3, "w/o I")."""
    P = np.asarray(points, np.float32).astype(np.float64)
    nb = P[nbr_idx[:K_N]]
    pbar = nb.mean(0)
    D = nb - pbar
    Cov = (D.T @ D) / K_N
    lam, vec = np.linalg.eigh(Cov)                       # ascending
    n = vec[:, 0]
    s_t = float(np.sqrt(nbr_d2[:K_S]).mean())
    s_n = r_normal * s_t
    Sigma = s_t ** 2 * (np.eye(3) - np.outer(n, n)) + s_n ** 2 * np.outer(n, n)
    gap = (lam[1] - lam[0]) / max(lam[2], 1e-300)
    return dict(cov=Cov, eig=lam, normal=n, s_t=s_t, s_n=s_n, sigma=Sigma,
                log_scales=np.array([math.log(s_t), math.log(s_t), math.log(s_n)]),
                logit=math.log(INIT_OPACITY / (1.0 - INIT_OPACITY)), gap=gap)


def seed_points(points, colours, queries, r_normal=R_NORMAL):
    """Seeds for the query indices; returns a list of dicts (see above) with
    `dc` (3,) added."""
    out = []
    y00 = 1.0 / (2.0 * math.sqrt(math.pi))
    for i in queries:
        a, b = knn_one(points, int(i))
        s = seed_from_neighbours(points, int(i), a, b, r_normal)
        s["nbr"] = a
        s["d2"] = b
        s["dc"] = (np.asarray(colours[int(i)], np.float64) - 0.5) / y00
        out.append(s)
    return out


def sigma_from_params(log_scales, quat):
    """Covariance R diag(exp(2 s)) R^T of one Gaussian (w, x, y, z quaternion)."""
    q = np.asarray(quat, np.float64)
    w, x, y, z = q / np.linalg.norm(q)
    R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                  [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                  [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
    s = np.exp(2.0 * np.asarray(log_scales, np.float64))
    return (R * s) @ R.T
