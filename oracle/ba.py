"""Robust bundle adjustment (oracle; test infrastructure, not the product path).

PocketGS refines the mobile tracking poses and sparse points by a global
bundle adjustment (subsection "GPU-Native Global BA as Mobile MAP
Refinement"): the robustified reprojection objective (equation ba_obj)
sum over observations (i, j) of rho(|pi(T_i, P_j) - p_ij|^2_W), rho the
Huber loss, W_ij the information weighting; scale-aware gauge fixing (the
first keyframe's 6-DoF pose fixed, the second keyframe's translation
constrained along the dominant baseline axis); and the normal equation
H Delta = b with H = J^T J solved through the reduced camera system
(Schur complement over the block-diagonal point blocks).

Readings where the paper is silent:
  * camera i: rotation R_i (world to camera) and centre c_i, x = R_i (P - c_i),
    pinhole pi(x) = (fx x0/x2 + cx, fy x1/x2 + cy) with shared intrinsics;
  * increments: rotation R_i <- R_i exp([dphi]x) (right perturbation),
    centre c_i <- c_i + dc, point P_j <- P_j + dP; pose parameters ordered
    (dphi, dc);
  * W_ij = I (unit information, pixel units);
  * Huber on the residual norm: rho(s) = s for sqrt(s) <= delta, else
    2 delta sqrt(s) - delta^2; the normal equations are the iteratively
    reweighted Gauss-Newton ones, weight w = rho'(s) = min(1, delta/sqrt(s));
  * gauge: camera 0's six parameters and camera 1's centre coordinate along
    the axis of its largest baseline component to camera 0 are held fixed
    (their increments are zero; their rows and columns leave H);
  * Levenberg-Marquardt damping H + lambda diag(H) on the free parameters,
    lambda divided by 10 after an accepted step and multiplied by 10 after
    a rejected one (a step is accepted when it lowers the robust cost).
The step is the plain definition: the damped normal equations over all free
parameters, assembled and solved directly (a library linear solve as one
step); the Schur complement is the method's way of reaching the same
solution and is checked against this.
"""

from __future__ import annotations

import numpy as np

from . import _rot


def project(R, c, P, fx, fy, cx, cy, cam, pt):
    """Camera-space points x (n_obs, 3) and pixels (n_obs, 2) of observations."""
    x = np.einsum("oij,oj->oi", R[cam], P[pt] - c[cam])
    uv = np.stack([fx * x[:, 0] / x[:, 2] + cx, fy * x[:, 1] / x[:, 2] + cy], 1)
    return x, uv


def residuals(prob, R, c, P):
    """r = pi(T_i, P_j) - p_ij for every observation (equation ba_obj)."""
    _, uv = project(R, c, P, prob["fx"], prob["fy"], prob["cx"], prob["cy"], prob["obs_cam"],
                    prob["obs_pt"])
    return uv - prob["obs_uv"]


def huber(s, delta):
    """rho(s) and its derivative w = rho'(s) for squared norms s."""
    n = np.sqrt(s)
    inlier = n <= delta
    rho = np.where(inlier, s, 2.0 * delta * n - delta * delta)
    w = np.where(inlier, 1.0, delta / np.where(inlier, 1.0, n))
    return rho, w


def cost(prob, R, c, P, delta):
    r = residuals(prob, R, c, P)
    return float(huber((r * r).sum(1), delta)[0].sum())


def jacobians(prob, R, c, P):
    """Per observation: d r / d(dphi, dc) (n_obs, 2, 6) and d r / dP (n_obs, 2, 3)."""
    fx, fy = prob["fx"], prob["fy"]
    cam, pt = prob["obs_cam"], prob["obs_pt"]
    d = P[pt] - c[cam]
    Ri = R[cam]
    x = np.einsum("oij,oj->oi", Ri, d)
    z = x[:, 2]
    Jx = np.zeros((x.shape[0], 2, 3))       # d pi / d x
    Jx[:, 0, 0] = fx / z
    Jx[:, 0, 2] = -fx * x[:, 0] / (z * z)
    Jx[:, 1, 1] = fy / z
    Jx[:, 1, 2] = -fy * x[:, 1] / (z * z)
    # x = R exp([dphi]x) d  ->  dx/ddphi = -R [d]x ;  dx/dc = -R ;  dx/dP = R
    Jphi = -np.einsum("oij,ojk->oik", Ri, _rot.skew(d))
    Jpose = np.concatenate([np.einsum("oab,obc->oac", Jx, Jphi), -np.einsum("oab,obc->oac", Jx, Ri)], 2)
    Jpt = np.einsum("oab,obc->oac", Jx, Ri)
    return Jpose, Jpt


def free_pose_params(n_cams, gauge_axis):
    """Indices (into 6 * n_cams) of the pose parameters that move."""
    fixed = set(range(6)) | {6 + 3 + gauge_axis}
    return np.array([k for k in range(6 * n_cams) if k not in fixed], np.int64)


def normal_equations(prob, R, c, P, delta):
    """Dense H = sum w J^T J and b = -sum w J^T r over all parameters
    (poses 6 n_cams, then points 3 n_points)."""
    C, M = R.shape[0], P.shape[0]
    r = residuals(prob, R, c, P)
    _, w = huber((r * r).sum(1), delta)
    Jpose, Jpt = jacobians(prob, R, c, P)
    n = 6 * C + 3 * M
    H = np.zeros((n, n))
    b = np.zeros(n)
    for o in range(r.shape[0]):
        i, j = int(prob["obs_cam"][o]), int(prob["obs_pt"][o])
        J = np.zeros((2, n))
        J[:, 6 * i:6 * i + 6] = Jpose[o]
        J[:, 6 * C + 3 * j:6 * C + 3 * j + 3] = Jpt[o]
        cols = np.r_[6 * i:6 * i + 6, 6 * C + 3 * j:6 * C + 3 * j + 3]
        Jc = J[:, cols]
        H[np.ix_(cols, cols)] += w[o] * Jc.T @ Jc
        b[cols] -= w[o] * Jc.T @ r[o]
    return H, b


def lm_step(prob, R, c, P, delta, lam):
    """The damped step: (H + lam diag(H)) Delta = b over the free parameters,
    zero for the fixed ones.  Returns (dpose (n_cams, 6), dpoint (n_points, 3))."""
    C, M = R.shape[0], P.shape[0]
    H, b = normal_equations(prob, R, c, P, delta)
    free = np.r_[free_pose_params(C, prob["gauge_axis"]), 6 * C + np.arange(3 * M)]
    A = H[np.ix_(free, free)]
    A = A + lam * np.diag(np.diag(A))
    delta_free = np.linalg.solve(A, b[free])
    full = np.zeros(6 * C + 3 * M)
    full[free] = delta_free
    return full[:6 * C].reshape(C, 6), full[6 * C:].reshape(M, 3)


def apply_step(R, c, P, dpose, dpoint):
    """R_i exp([dphi_i]x), c_i + dc_i, P_j + dP_j."""
    return R @ _rot.exp_so3(dpose[:, :3]), c + dpose[:, 3:], P + dpoint


def lm(prob, R, c, P, delta, lam=1e-3, iters=10):
    """Levenberg-Marquardt iterations; returns the final state, the cost
    history and the accept flags."""
    hist, acc = [cost(prob, R, c, P, delta)], []
    for _ in range(iters):
        dpose, dpoint = lm_step(prob, R, c, P, delta, lam)
        R1, c1, P1 = apply_step(R, c, P, dpose, dpoint)
        f1 = cost(prob, R1, c1, P1, delta)
        if f1 < hist[-1]:
            R, c, P = R1, c1, P1
            hist.append(f1)
            acc.append(True)
            lam /= 10.0
        else:
            hist.append(hist[-1])
            acc.append(False)
            lam *= 10.0
    return (R, c, P), hist, acc


def normal_equations_sparse(prob, R, c, P, delta):
    """H (scipy CSR) and b, as normal_equations but assembled sparsely (for
    full-size problems)."""
    import scipy.sparse as sp
    C, M = R.shape[0], P.shape[0]
    r = residuals(prob, R, c, P)
    _, w = huber((r * r).sum(1), delta)
    Jpose, Jpt = jacobians(prob, R, c, P)
    cam = prob["obs_cam"].astype(np.int64)
    pt = prob["obs_pt"].astype(np.int64)
    cols = np.concatenate([6 * cam[:, None] + np.arange(6), 6 * C + 3 * pt[:, None] + np.arange(3)], 1)  # (o, 9)
    J = np.concatenate([Jpose, Jpt], 2)                                   # (o, 2, 9)
    blk = np.einsum("o,oai,oaj->oij", w, J, J)                           # (o, 9, 9)
    rows = np.repeat(cols[:, :, None], 9, 2)
    colz = np.repeat(cols[:, None, :], 9, 1)
    n = 6 * C + 3 * M
    H = sp.coo_matrix((blk.ravel(), (rows.ravel(), colz.ravel())), shape=(n, n)).tocsr()
    b = np.zeros(n)
    np.add.at(b, cols.ravel(), -np.einsum("o,oai,oa->oi", w, J, r).ravel())
    return H, b


# Iterative geometric refinement (subsection "GPU-Native Global BA", the
# refinement loop): after a global update every point is re-triangulated
# from its observations with the updated poses, points with a high
# reprojection error or an insufficient triangulation angle are dropped and
# observations behind their camera are discarded.  Readings: the
# re-triangulated point is the least-squares intersection of the
# observation rays (the point minimising the summed squared distances to
# the rays, sum (I - d d^T) P = sum (I - d d^T) c, d the unit world ray of
# the measured pixel); a point is kept when it has at least two
# observations in front of their cameras (z > 0), the mean reprojection
# error over those is at most max_err pixels and the largest angle between
# two of their camera-to-point rays is at least min_angle (tested as the
# smallest cosine <= cos(min_angle)); an observation is kept when its point
# is kept and it lies in front of its camera.  A point whose normal matrix
# has a determinant of at most 1e-12 times the cube of its trace is dropped.

def observation_rays(prob, R, c):
    """Unit world directions of the measured pixels, (n_obs, 3)."""
    cam = prob["obs_cam"]
    uv = prob["obs_uv"]
    dc = np.stack([(uv[:, 0] - prob["cx"]) / prob["fx"], (uv[:, 1] - prob["cy"]) / prob["fy"],
                   np.ones(uv.shape[0])], 1)
    d = np.einsum("oji,oj->oi", R[cam], dc)          # R^T dc
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def retriangulate(prob, R, c, n_points):
    """Least-squares ray intersection per point; (points, solvable mask)."""
    d = observation_rays(prob, R, c)
    cam, pt = prob["obs_cam"], prob["obs_pt"]
    A = np.zeros((n_points, 3, 3))
    b = np.zeros((n_points, 3))
    Pm = np.eye(3)[None] - d[:, :, None] * d[:, None, :]
    np.add.at(A, pt, Pm)
    np.add.at(b, pt, np.einsum("oij,oj->oi", Pm, c[cam]))
    tr = np.trace(A, axis1=1, axis2=2)
    det = np.linalg.det(A)
    ok = det > 1e-12 * tr ** 3
    P = np.zeros((n_points, 3))
    P[ok] = np.linalg.solve(A[ok], b[ok][:, :, None])[:, :, 0]
    return P, ok


def refine(prob, R, c, n_points, max_err=4.0, min_angle=np.radians(1.5)):
    """Re-triangulated points, point keep mask, observation keep mask and
    the per-point statistics (mean error, smallest ray cosine, count)."""
    P, ok = retriangulate(prob, R, c, n_points)
    cam, pt = prob["obs_cam"], prob["obs_pt"]
    x, uv = project(R, c, P, prob["fx"], prob["fy"], prob["cx"], prob["cy"], cam, pt)
    front = x[:, 2] > 0
    err = np.linalg.norm(uv - prob["obs_uv"], axis=1)
    cnt = np.bincount(pt, weights=front, minlength=n_points)
    esum = np.bincount(pt, weights=np.where(front, err, 0.0), minlength=n_points)
    mean_err = np.where(cnt > 0, esum / np.maximum(cnt, 1), np.inf)
    ray = P[pt] - c[cam]
    ray /= np.linalg.norm(ray, axis=1, keepdims=True)
    min_cos = np.full(n_points, np.inf)
    starts = np.searchsorted(pt, np.arange(n_points + 1))
    for j in range(n_points):
        o = np.arange(starts[j], starts[j + 1])
        o = o[front[o]]
        if o.size >= 2:
            g = ray[o] @ ray[o].T
            min_cos[j] = g[np.triu_indices(o.size, 1)].min()
    keep_pt = ok & (cnt >= 2) & (mean_err <= max_err) & (min_cos <= np.cos(min_angle))
    keep_obs = keep_pt[pt] & front
    return P, keep_pt, keep_obs, dict(mean_err=mean_err, min_cos=min_cos, count=cnt, solvable=ok)


def compact(prob, P, keep_pt, keep_obs):
    """The problem and points restricted to the kept points and
    observations (order preserved, points renumbered)."""
    new_id = np.cumsum(keep_pt) - 1
    out = {k: prob[k] for k in ("fx", "fy", "cx", "cy", "gauge_axis")}
    out["obs_cam"] = prob["obs_cam"][keep_obs]
    out["obs_pt"] = new_id[prob["obs_pt"][keep_obs]]
    out["obs_uv"] = prob["obs_uv"][keep_obs]
    return out, P[keep_pt]
