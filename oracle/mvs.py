"""Single-reference cost-volume multi-view stereo (oracle; test
infrastructure, not the product path).

PocketGS densifies the refined sparse scaffold with a plane-sweep stereo
stage (subsection "Single-Reference Cost-Volume MVS"): per target view a
depth search range from the projected bundle-adjustment points
([0.5 q_.05, 1.5 q_.95] of their depths), ONE reference view chosen by the
score S_ref = exp(-(b - b_target)^2 / (2 sigma_b^2)) * max(alpha / alpha_min, 1)
(equation S_ref; b the baseline, alpha the viewing angle), a Census-transform
matching cost over plane-sweep depth hypotheses, SGM aggregation, a
confidence filter at 0.4 and fusion of the surviving depths into the dense
cloud P.

Readings where the paper is silent (the paper gives no window, hypothesis
count, penalties, path set or confidence measure):
  * images are 8-bit greyscale; Census over a 7 x 7 window, 48 bits: bit b
    (row-major over the window, the centre skipped) is set when the
    neighbour is darker than the centre, I(q) < I(p); neighbours outside the
    image take the nearest border pixel;
  * hypotheses: n_planes fronto-parallel planes of the target camera,
    uniform in inverse depth, plane 0 the farthest:
    1/d_k = 1/d_max + k h,  h = (1/d_min - 1/d_max) / (n_planes - 1);
  * the plane sweep maps target pixel (x, y) (integer pixel centres) at
    depth d_k to X = d_k ((x - cx)/fx, (y - cy)/fy, 1), then to the
    reference camera X_r = M X + m with M = R_r R_t^T, m = t_r - M t_t, and
    samples the reference Census at the nearest pixel
    (floor(fx_r x_r / z_r + cx_r + 0.5), likewise y); the cost is the
    Hamming distance of the two Census strings, 48 where z_r <= 0 or the
    pixel falls outside the reference image.  The sweep is defined in
    float64 (the paper fixes no precision).  An implementation that
    evaluates it in a shorter precision may take a nearest-pixel or
    in-front decision the other way where the exact coordinate lies within
    its rounding error of a rounding step or an image edge; such cells are
    reported as marginal (see sweep_pixels) and either outcome is accepted
    for them, as for the marginal binning decisions of the splatting path;
  * SGM over 4 paths (left to right, right to left, top to bottom, bottom
    to top) with constant penalties P1, P2:
    L_r(p, k) = C(p, k) + min(L_r(p-r, k), L_r(p-r, k-1) + P1,
                L_r(p-r, k+1) + P1, min_i L_r(p-r, i) + P2) - min_i L_r(p-r, i),
    L_r = C at a path's first pixel; S = sum_r L_r;
  * winner k* = argmin_k S (smallest k on ties); confidence
    1 - S(k*) / S2 with S2 = min of S over |k - k*| >= 2; a pixel is kept
    when 0 < k* < n_planes - 1, S2 > 0 and S(k*) <= (1 - 0.4) S2;
  * its depth: the parabola through (k* - 1, k*, k* + 1) refines k* to
    k* + delta, delta = (S(k*-1) - S(k*+1)) / (2 (S(k*-1) - 2 S(k*) + S(k*+1)))
    (0 when the denominator is 0), 1/d = 1/d_max + (k* + delta) h;
  * depth range: the BA points with camera depth z > 0 that project inside
    the target image (pixel coordinate in [-0.5, W - 0.5) x [-0.5, H - 0.5));
    quantile q(p) of their sorted depths z_(0..n-1): h = (n - 1) p,
    i = floor(h), q = z_i + (z_{i+1} - z_i)(h - i);
  * reference score: b = |c_ref - c_target| (camera centres), alpha = the
    angle between the two optical axes; candidates are all other views;
    the formula is taken as printed (the max factor raises the score of
    wider angles, the baseline term keeps the choice near b_target);
    argmax, smallest index on ties;
  * fusion: the union, view by view in row-major pixel order, of the kept
    pixels back-projected to the world, R_t^T (X - t_t), each with its
    image intensity as colour (greyscale captures); every stride-th point
    of that sequence is kept when the cloud is thinned for seeding.
Cameras are the float32-stored intrinsics and [R|t] taken as float64.  The
decisions that turn floating point into integers (nearest reference pixel,
inside tests, range membership) are written as explicit float64 operations
in a fixed order without fused multiply-adds, so that they are
reproducible.
"""

from __future__ import annotations

import math

import numpy as np

CENSUS_R = 3                     # 7 x 7 window
CENSUS_BITS = (2 * CENSUS_R + 1) ** 2 - 1
COST_OUT = CENSUS_BITS
CONF_MIN = 0.4


def cam64(cam):
    """(fx, fy, cx, cy, R (3, 3), t (3,)) in float64 from the float32 camera."""
    vm = np.asarray(cam["viewmat"], np.float32).astype(np.float64)
    f = lambda v: float(np.float32(v))
    return f(cam["fx"]), f(cam["fy"]), f(cam["cx"]), f(cam["cy"]), vm[:, :3], vm[:, 3]


def census(grey):
    """48-bit Census strings (uint64, (H, W)) of an 8-bit image."""
    g = np.asarray(grey).astype(np.int32)
    H, W = g.shape
    pad = np.pad(g, CENSUS_R, mode="edge")
    out = np.zeros((H, W), np.uint64)
    b = 0
    for dy in range(-CENSUS_R, CENSUS_R + 1):
        for dx in range(-CENSUS_R, CENSUS_R + 1):
            if dy == 0 and dx == 0:
                continue
            q = pad[CENSUS_R + dy:CENSUS_R + dy + H, CENSUS_R + dx:CENSUS_R + dx + W]
            out |= (q < g).astype(np.uint64) << np.uint64(b)
            b += 1
    return out


def popcount64(x):
    x = np.asarray(x, np.uint64)
    n = np.zeros(x.shape, np.int64)
    for s in range(0, 64, 8):
        n += _POP8[((x >> np.uint64(s)) & np.uint64(255)).astype(np.int64)]
    return n


_POP8 = np.array([bin(i).count("1") for i in range(256)], np.int64)


def plane_inverse_depths(d_min, d_max, n_planes):
    """1/d_k for k = 0..n_planes-1 (plane 0 the farthest) and the step h."""
    inv_far = 1.0 / d_max
    h = (1.0 / d_min - inv_far) / (n_planes - 1)
    return np.array([inv_far + k * h for k in range(n_planes)]), h


def relative_pose(cam_t, cam_r):
    """M = R_r R_t^T and m = t_r - M t_t, each entry a left-to-right sum."""
    _, _, _, _, Rt, tt = cam64(cam_t)
    _, _, _, _, Rr, tr = cam64(cam_r)
    M = np.zeros((3, 3))
    for i in range(3):
        for j in range(3):
            M[i, j] = Rr[i, 0] * Rt[j, 0] + Rr[i, 1] * Rt[j, 1] + Rr[i, 2] * Rt[j, 2]
    m = np.array([tr[i] - (M[i, 0] * tt[0] + M[i, 1] * tt[1] + M[i, 2] * tt[2]) for i in range(3)])
    return M, m


# unit roundoff of float32, for the marginal-decision bound of the sweep
U32 = 2.0 ** -24


def sweep_pixels(cam_t, cam_r, d_min, d_max, n_planes, xs, ys, with_margin=False):
    """Nearest reference pixel (qx, qy) and validity for target pixels
    (xs, ys) (1-D arrays) at every plane: arrays (n_planes, n), in float64.

    with_margin=True also returns `marginal` (n_planes, n): the cells whose
    outcome (validity and pixel) an evaluation of the same formulas in
    float32 could change.  For the reference coordinate
    t = fx_r x_r / z_r + cx_r + 1/2 a first-order bound of that evaluation's
    error is
      e_q = 8u (S_x + |q| S_z) / |z_r| + u |q|,   q = x_r / z_r,
      e_t = 2 (|fx_r| e_q + 4u (|fx_r q| + |cx_r| + 1)),
    with S_x = |M_00 X| + |M_01 Y| + |M_02 Z| + |m_0| (S_z likewise), u = 2^-24:
    every input (M, m, d, ray) is rounded once and every product, sum and
    quotient once more.  A cell is marginal when floor(t - e_t) and
    floor(t + e_t) differ and at least one of them lies on the image, for
    x or y, or when |z_r| <= 16u S_z (the in-front test)."""
    fx, fy, cx, cy, _, _ = cam64(cam_t)
    fxr, fyr, cxr, cyr, _, _ = cam64(cam_r)
    Wr, Hr = cam_r["width"], cam_r["height"]
    M, m = relative_pose(cam_t, cam_r)
    inv, _ = plane_inverse_depths(d_min, d_max, n_planes)
    d = (1.0 / inv)[:, None]
    a = ((np.asarray(xs, np.float64) - cx) / fx)[None, :]
    b = ((np.asarray(ys, np.float64) - cy) / fy)[None, :]
    X, Y, Z = d * a, d * b, np.broadcast_to(d, (d.shape[0], a.shape[1]))
    rows = [((M[r, 0] * X + M[r, 1] * Y) + M[r, 2] * Z) + m[r] for r in range(3)]
    xr, yr, zr = rows
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        qx_, qy_ = xr / zr, yr / zr
        tx = fxr * qx_ + cxr + 0.5
        ty = fyr * qy_ + cyr + 0.5
        u, v = np.floor(tx), np.floor(ty)
    front = zr > 0
    ok = front & (u >= 0) & (u <= Wr - 1) & (v >= 0) & (v <= Hr - 1)
    qx = np.where(ok, u, 0).astype(np.int64)
    qy = np.where(ok, v, 0).astype(np.int64)
    if not with_margin:
        return qx, qy, ok
    S = [np.abs(M[r, 0] * X) + np.abs(M[r, 1] * Y) + np.abs(M[r, 2] * Z) + abs(m[r]) for r in range(3)]
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        az = np.abs(zr)

        def step_marginal(t, q, Sq, f, c, n_pix):
            e_q = 8 * U32 * (Sq + np.abs(q) * S[2]) / az + U32 * np.abs(q)
            e_t = 2.0 * (abs(f) * e_q + 4 * U32 * (np.abs(f * q) + abs(c) + 1.0))
            lo, hi = np.floor(t - e_t), np.floor(t + e_t)
            on_image = ((lo >= 0) & (lo <= n_pix - 1)) | ((hi >= 0) & (hi <= n_pix - 1))
            return (lo != hi) & on_image

        mx = step_marginal(tx, qx_, S[0], fxr, cxr, Wr)
        my = step_marginal(ty, qy_, S[1], fyr, cyr, Hr)
    mz = az <= 16 * U32 * S[2]
    marginal = mz | (front & (mx | my))
    return qx, qy, ok, marginal


def cost_volume(cen_t, cen_r, cam_t, cam_r, d_min, d_max, n_planes, rows=None, with_margin=False):
    """C[y][x][k] (uint8): Hamming distance of the target Census and the
    reference Census at the swept pixel, COST_OUT where invalid.  `rows`
    restricts to those target rows (the result then has len(rows) rows).
    with_margin=True also returns the marginal cells of the sweep (same
    shape, bool; see sweep_pixels)."""
    H, W = cen_t.shape
    rows = np.arange(H) if rows is None else np.asarray(rows)
    ys, xs = np.meshgrid(rows, np.arange(W), indexing="ij")
    sw = sweep_pixels(cam_t, cam_r, d_min, d_max, n_planes, xs.ravel(), ys.ravel(), with_margin)
    qx, qy, ok = sw[:3]
    ham = popcount64(cen_t[ys.ravel(), xs.ravel()][None, :] ^ cen_r[qy, qx])
    C = np.where(ok, ham, COST_OUT).astype(np.uint8)            # (n_planes, n)
    C = C.T.reshape(len(rows), W, n_planes)
    if not with_margin:
        return C
    return C, sw[3].T.reshape(len(rows), W, n_planes)


def sgm_path(C, p1, p2):
    """L_r along axis 1 of C (lines, steps, planes), first step to last."""
    C = C.astype(np.int64)
    L = np.empty_like(C)
    L[:, 0] = C[:, 0]
    big = np.iinfo(np.int64).max // 4
    for s in range(1, C.shape[1]):
        prev = L[:, s - 1]
        mn = prev.min(1, keepdims=True)
        km1 = np.concatenate([np.full((prev.shape[0], 1), big), prev[:, :-1]], 1)
        kp1 = np.concatenate([prev[:, 1:], np.full((prev.shape[0], 1), big)], 1)
        best = np.minimum(np.minimum(prev, km1 + p1), np.minimum(kp1 + p1, mn + p2))
        L[:, s] = C[:, s] + best - mn
    return L


def sgm(C, p1, p2):
    """S = sum of the four path costs (int64, (H, W, n_planes))."""
    S = sgm_path(C, p1, p2)                                       # left to right
    S = S + sgm_path(C[:, ::-1], p1, p2)[:, ::-1]                 # right to left
    Ct = C.transpose(1, 0, 2)
    S = S + sgm_path(Ct, p1, p2).transpose(1, 0, 2)               # top to bottom
    S = S + sgm_path(Ct[:, ::-1], p1, p2)[:, ::-1].transpose(1, 0, 2)  # bottom to top
    return S


def winner(S, d_min, d_max, conf_min=CONF_MIN):
    """Depth (float32, 0 where rejected), confidence (float32) and the
    winning plane per pixel from the aggregated costs S (H, W, n_planes)."""
    H, W, D = S.shape
    k = S.argmin(2)
    s1 = np.take_along_axis(S, k[..., None], 2)[..., 0]
    kk = np.arange(D)[None, None, :]
    far = np.abs(kk - k[..., None]) >= 2
    s2 = np.where(far, S, np.iinfo(np.int64).max).min(2)
    keep = (k > 0) & (k < D - 1) & (s2 > 0) & (s1 <= (1.0 - conf_min) * s2)
    km = np.take_along_axis(S, np.clip(k - 1, 0, D - 1)[..., None], 2)[..., 0]
    kp = np.take_along_axis(S, np.clip(k + 1, 0, D - 1)[..., None], 2)[..., 0]
    den = km - 2 * s1 + kp
    with np.errstate(divide="ignore", invalid="ignore"):
        delta = np.where(den > 0, (km - kp) / (2.0 * np.where(den > 0, den, 1)), 0.0)
    _, h = plane_inverse_depths(d_min, d_max, D)
    inv = 1.0 / d_max + (k + delta) * h
    depth = np.where(keep, 1.0 / inv, 0.0).astype(np.float32)
    with np.errstate(divide="ignore", invalid="ignore"):
        conf = np.where(s2 > 0, 1.0 - s1 / np.where(s2 > 0, s2, 1), 0.0).astype(np.float32)
    return depth, conf, k


def point_depths(cam, points):
    """Camera depth z and pixel (u, v) of world points, each coordinate a
    left-to-right float64 sum (the range estimate's projection)."""
    fx, fy, cx, cy, R, t = cam64(cam)
    P = np.asarray(points, np.float64)
    x = R[0, 0] * P[:, 0] + R[0, 1] * P[:, 1] + R[0, 2] * P[:, 2] + t[0]
    y = R[1, 0] * P[:, 0] + R[1, 1] * P[:, 1] + R[1, 2] * P[:, 2] + t[1]
    z = R[2, 0] * P[:, 0] + R[2, 1] * P[:, 1] + R[2, 2] * P[:, 2] + t[2]
    with np.errstate(divide="ignore", invalid="ignore"):
        u = fx * (x / z) + cx
        v = fy * (y / z) + cy
    return z, u, v


def quantile_sorted(z, p):
    """q(p) of ascending z: z_i + (z_{i+1} - z_i)(h - i), h = (n - 1) p."""
    n = len(z)
    h = (n - 1) * p
    i = int(math.floor(h))
    if i + 1 >= n:
        return float(z[n - 1])
    return float(z[i] + (z[i + 1] - z[i]) * (h - i))


def depth_range(cam, points):
    """[0.5 q_.05, 1.5 q_.95] of the depths of the points that project into
    the view (z > 0, pixel inside); (0, 0) when none does."""
    z, u, v = point_depths(cam, points)
    W, H = cam["width"], cam["height"]
    ok = (z > 0) & (u >= -0.5) & (u < W - 0.5) & (v >= -0.5) & (v < H - 0.5)
    zs = np.sort(z[ok])
    if zs.size == 0:
        return 0.0, 0.0
    return 0.5 * quantile_sorted(zs, 0.05), 1.5 * quantile_sorted(zs, 0.95)


def ref_score(cam_t, cam_c, b_target, sigma_b, alpha_min):
    _, _, _, _, Rt, tt = cam64(cam_t)
    _, _, _, _, Rc, tc = cam64(cam_c)
    ct, cc = -Rt.T @ tt, -Rc.T @ tc
    b = float(np.linalg.norm(cc - ct))
    alpha = math.acos(max(-1.0, min(1.0, float(Rt[2] @ Rc[2]))))
    return math.exp(-(b - b_target) ** 2 / (2.0 * sigma_b ** 2)) * max(alpha / alpha_min, 1.0)


def select_reference(cams, target, b_target, sigma_b, alpha_min):
    """The candidate maximising S_ref, and every candidate's score."""
    scores = np.array([ref_score(cams[target], cams[c], b_target, sigma_b, alpha_min) if c != target
                       else -np.inf for c in range(len(cams))])
    return int(np.argmax(scores)), scores


def fuse(cam, depth, grey=None):
    """World points (float32, (n, 3)) of the kept pixels of one depth map,
    row-major: R^T (z ((x - cx)/fx, (y - cy)/fy, 1) - t); with the view's
    grey image also their intensities / 255 (float32, (n,))."""
    fx, fy, cx, cy, R, t = cam64(cam)
    ys, xs = np.nonzero(depth > 0)
    z = depth[ys, xs].astype(np.float64)
    Xc = np.stack([z * ((xs - cx) / fx), z * ((ys - cy) / fy), z], 1) - t
    P = (Xc @ R).astype(np.float32)
    if grey is None:
        return P
    return P, (np.asarray(grey)[ys, xs].astype(np.float32) / np.float32(255.0))


def depth_map(grey_t, grey_r, cam_t, cam_r, d_min, d_max, n_planes, p1, p2, conf_min=CONF_MIN):
    """The whole per-view chain: Census, cost volume, SGM, winner."""
    C = cost_volume(census(grey_t), census(grey_r), cam_t, cam_r, d_min, d_max, n_planes)
    S = sgm(C, p1, p2)
    depth, conf, k = winner(S, d_min, d_max, conf_min)
    return dict(cost=C, agg=S, depth=depth, conf=conf, k=k)
