"""Seeded generators: parameters, cameras, scenes, clouds, images (inputs only)."""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Degree-0 colour encoding used for inputs: colour = f00 * Y00 + 1/2 with the
# orthonormal constant Y00 = 1 / (2 sqrt(pi)); f00 = (colour - 1/2) * 2 sqrt(pi).
_DC_SCALE = 2.0 * math.sqrt(math.pi)


def param_rows(sh_degree: int) -> int:
    """Number of canonical rows for SH degree D: 11 + 3 (D+1)^2."""
    return 11 + 3 * (sh_degree + 1) ** 2


def sh_coeffs(sh_degree: int) -> int:
    return (sh_degree + 1) ** 2


def make_camera(width, height, fx, fy, cx, cy, R, t) -> dict:
    vm = np.zeros((3, 4), np.float32)
    vm[:, :3] = np.asarray(R, np.float64)
    vm[:, 3] = np.asarray(t, np.float64)
    return dict(width=int(width), height=int(height), fx=float(np.float32(fx)),
                fy=float(np.float32(fy)), cx=float(np.float32(cx)),
                cy=float(np.float32(cy)), viewmat=vm)


def look_at_camera(eye, target, width, height, hfov_deg=60.0, up=(0.0, 1.0, 0.0)) -> dict:
    """Pinhole camera at `eye` looking at `target`; OpenCV axes, world +y up.

    fx = fy = W / (2 tan(hfov/2)), principal point at the image centre.
    """
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, np.float64))
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f])
    t = -R @ eye
    fx = width / (2.0 * math.tan(math.radians(hfov_deg) / 2.0))
    return make_camera(width, height, fx, fx, width / 2.0, height / 2.0, R, t)


def ring_cameras(n=60, width=1920, height=1440, radius=4.5, height_y=0.8,
                 target=(0.0, 0.3, 0.0), hfov_deg=60.0) -> list:
    """n cameras evenly spaced on a horizontal ring, all looking at `target`."""
    cams = []
    for i in range(n):
        a = 2.0 * math.pi * i / n
        eye = (radius * math.sin(a), height_y, radius * math.cos(a))
        cams.append(look_at_camera(eye, target, width, height, hfov_deg))
    return cams


def random_image(seed, height, width, lo=0.0, hi=1.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, (3, height, width)).astype(np.float32)


def random_normal(seed, shape, std=1.0) -> np.ndarray:
    """float32 array of the given shape, entries N(0, std^2) drawn in C order
    (network weights, feature rows and output gradients of tests)."""
    rng = np.random.default_rng(seed)
    return (std * rng.standard_normal(shape)).astype(np.float32)


def cfg1_inputs(seed=0, n=1000, width=128, height=128, focal=128.0):
    """Small parity workload.

    Draw order: means U[-1,1]^3 (n,3); log-scales N(-3, 0.5^2) (n,3);
    quaternions N(0, I4) normalised (n,4); opacity logits N(0,1) (n,);
    DC colour coefficients U[-sqrt(pi), sqrt(pi)] (n,3), i.e. degree-0 colours
    uniform in [0, 1]; target image U[0,1]^(3,H,W).  Means are then shifted by
    +4 along z.  Camera: identity pose, fx = fy = focal, principal point at the
    image centre.
    """
    rng = np.random.default_rng(seed)
    means = rng.uniform(-1.0, 1.0, (n, 3))
    log_s = rng.normal(-3.0, 0.5, (n, 3))
    q = rng.normal(0.0, 1.0, (n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    logit = rng.normal(0.0, 1.0, n)
    half = math.sqrt(math.pi)
    dc = rng.uniform(-half, half, (n, 3))
    target = rng.uniform(0.0, 1.0, (3, height, width))
    means[:, 2] += 4.0
    P = np.zeros((param_rows(0), n), np.float32)
    P[0:3] = means.T
    P[3:6] = log_s.T
    P[6:10] = q.T
    P[10] = logit
    P[11:14] = dc.T
    cam = make_camera(width, height, focal, focal, width / 2.0, height / 2.0,
                      np.eye(3), np.zeros(3))
    return P, cam, target.astype(np.float32)


def random_gaussians(seed, n, sh_degree=0, centre=(0.0, 0.0, 4.0), spread=1.0,
                     log_scale_mu=-3.0, log_scale_sigma=0.5, sh_sigma=0.3):
    """Generic random Gaussians around `centre` (used for edge-case tests).

    Draw order: means, log-scales, quaternions, logits, DC, higher SH.
    """
    rng = np.random.default_rng(seed)
    K = sh_coeffs(sh_degree)
    means = rng.uniform(-spread, spread, (n, 3)) + np.asarray(centre)
    log_s = rng.normal(log_scale_mu, log_scale_sigma, (n, 3))
    q = rng.normal(0.0, 1.0, (n, 4))
    logit = rng.normal(0.0, 1.0, n)
    half = math.sqrt(math.pi)
    dc = rng.uniform(-half, half, (n, 3))
    hi = rng.normal(0.0, sh_sigma, (n, K - 1, 3))
    P = np.zeros((param_rows(sh_degree), n), np.float32)
    P[0:3] = means.T
    P[3:6] = log_s.T
    P[6:10] = q.T
    P[10] = logit
    P[11:14] = dc.T
    if K > 1:
        P[14:] = hi.reshape(n, -1).T
    return P


# ---------------------------------------------------------------------------
# Spheres + planes scene
# ---------------------------------------------------------------------------

@dataclass
class Scene:
    centres: np.ndarray          # (S, 3)
    radii: np.ndarray            # (S,)
    planes: list                 # [(origin, u_axis, v_axis, normal, u_len, v_len)]
    base: np.ndarray             # (S + n_planes, 3) base colours
    freq: np.ndarray             # (S + n_planes, 3) texture frequencies
    phase: np.ndarray            # (S + n_planes, 3) texture phases
    areas: np.ndarray = field(default=None)

    @property
    def total_area(self) -> float:
        return float(self.areas.sum())


def spheres_planes_scene(seed=0, n_spheres=20) -> Scene:
    """20 random spheres (r in [0.2, 1]) plus floor, back wall and side wall.

    Draw order: disc radius U (S,), disc angle U (S,), centre y U[-0.5,1.5] (S,),
    radius U[0.2,1] (S,), base colours U[0.15,0.85] (S+3,3), texture
    frequencies U[2,9] (S+3,3), phases U[0,2pi] (S+3,3).
    """
    rng = np.random.default_rng(seed)
    rd = 2.5 * np.sqrt(rng.uniform(0, 1, n_spheres))
    th = rng.uniform(0, 2 * np.pi, n_spheres)
    cy = rng.uniform(-0.5, 1.5, n_spheres)
    radii = rng.uniform(0.2, 1.0, n_spheres)
    centres = np.stack([rd * np.cos(th), cy, rd * np.sin(th)], 1)
    planes = [
        # floor y = -1.5, x,z in [-6, 6], normal +y
        (np.array([-6.0, -1.5, -6.0]), np.array([1.0, 0, 0]), np.array([0, 0, 1.0]),
         np.array([0, 1.0, 0]), 12.0, 12.0),
        # back wall z = -6, x in [-6,6], y in [-1.5, 4.5], normal +z
        (np.array([-6.0, -1.5, -6.0]), np.array([1.0, 0, 0]), np.array([0, 1.0, 0]),
         np.array([0, 0, 1.0]), 12.0, 6.0),
        # side wall x = -6, z in [-6,6], y in [-1.5, 4.5], normal +x
        (np.array([-6.0, -1.5, -6.0]), np.array([0, 0, 1.0]), np.array([0, 1.0, 0]),
         np.array([1.0, 0, 0]), 12.0, 6.0),
    ]
    ns = n_spheres + len(planes)
    base = rng.uniform(0.15, 0.85, (ns, 3))
    freq = rng.uniform(2.0, 9.0, (ns, 3))
    phase = rng.uniform(0.0, 2 * np.pi, (ns, 3))
    areas = np.concatenate([4 * np.pi * radii ** 2,
                            [p[4] * p[5] for p in planes]])
    return Scene(centres, radii, planes, base, freq, phase, areas)


def _texture(scene: Scene, sid: np.ndarray, p: np.ndarray) -> np.ndarray:
    """Procedural colour: base + sinusoidal detail + checker, clipped to [0.02, 0.98]."""
    b = scene.base[sid]
    f = scene.freq[sid]
    ph = scene.phase[sid]
    s = np.sin(f * p[:, [0, 1, 2]] + ph) * np.sin(f * p[:, [1, 2, 0]] * 0.7 + ph * 1.3)
    chk = ((np.floor(p[:, 0] * 2.0) + np.floor(p[:, 1] * 2.0) + np.floor(p[:, 2] * 2.0)) % 2)
    c = b + 0.25 * s + 0.08 * (chk[:, None] - 0.5)
    return np.clip(c, 0.02, 0.98)


def sample_surface(scene: Scene, n: int, seed: int):
    """Area-weighted surface samples: returns points (n,3), normals (n,3), colours (n,3).

    Draw order: surface choice (multinomial over areas), then per surface in
    index order: spheres draw N(0,I3) directions; planes draw U[0,1]^2.
    """
    rng = np.random.default_rng(seed)
    counts = rng.multinomial(n, scene.areas / scene.areas.sum())
    pts, nrm, sid = [], [], []
    S = len(scene.radii)
    for s in range(len(counts)):
        k = counts[s]
        if k == 0:
            continue
        if s < S:
            d = rng.normal(0, 1, (k, 3))
            d /= np.linalg.norm(d, axis=1, keepdims=True)
            pts.append(scene.centres[s] + scene.radii[s] * d)
            nrm.append(d)
        else:
            o, ua, va, nn, ul, vl = scene.planes[s - S]
            uv = rng.uniform(0, 1, (k, 2))
            pts.append(o + uv[:, :1] * ul * ua + uv[:, 1:] * vl * va)
            nrm.append(np.broadcast_to(nn, (k, 3)).copy())
        sid.append(np.full(k, s))
    pts = np.concatenate(pts)
    nrm = np.concatenate(nrm)
    sid = np.concatenate(sid)
    col = _texture(scene, sid, pts)
    return pts, nrm, col


def _quat_mul(a, b):
    w1, x1, y1, z1 = a.T
    w2, x2, y2, z2 = b.T
    return np.stack([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2], 1)


def surface_gaussians(scene: Scene, n: int, seed: int, sh_degree=0, opacity=None,
                      logit_sigma=None, sh_sigma=0.05, thickness=0.1, size=0.6):
    """Flat Gaussians on the scene surface (ground truth / workload scenes).

    Tangential scale s_t = size * sqrt(A_total / n), normal scale
    thickness * s_t; local z along the surface normal with a random in-plane
    angle.  Opacity is either fixed (`opacity`) or logit ~ N(0, logit_sigma^2).
    Draw order: surface samples (seed), then from default_rng(seed + 1): in-plane
    angles U[0,2pi] (n,), logits (if random) (n,), higher SH N(0, sh_sigma^2).
    """
    pts, nrm, col = sample_surface(scene, n, seed)
    rng = np.random.default_rng(seed + 1)
    ang = rng.uniform(0, 2 * np.pi, n)
    s_t = size * math.sqrt(scene.total_area / n)
    # rotation taking +z onto the normal, composed with a spin about z
    qa = np.stack([1.0 + nrm[:, 2], -nrm[:, 1], nrm[:, 0], np.zeros(n)], 1)
    bad = qa[:, 0] < 1e-6                     # normal == -z: rotate pi about x
    qa[bad] = np.array([0.0, 1.0, 0.0, 0.0])
    qa /= np.linalg.norm(qa, axis=1, keepdims=True)
    qs = np.stack([np.cos(ang / 2), np.zeros(n), np.zeros(n), np.sin(ang / 2)], 1)
    q = _quat_mul(qa, qs)
    if opacity is not None:
        logit = np.full(n, math.log(opacity / (1.0 - opacity)))
    else:
        logit = rng.normal(0.0, logit_sigma if logit_sigma else 0.5, n)
    K = sh_coeffs(sh_degree)
    P = np.zeros((param_rows(sh_degree), n), np.float32)
    P[0:3] = pts.T
    P[3:5] = math.log(s_t)
    P[5] = math.log(thickness * s_t)
    P[6:10] = q.T
    P[10] = logit
    P[11:14] = ((col - 0.5) * _DC_SCALE).T
    if K > 1:
        P[14:] = rng.normal(0.0, sh_sigma, (n, (K - 1) * 3)).T
    return P


def noisy_cloud(scene: Scene, n: int, seed: int, noise=0.01):
    """Point cloud standing in for the dense geometry prior: surface samples plus
    isotropic N(0, noise^2) jitter.  Returns points (n,3) float32, colours (n,3).

    Draw order: surface samples (seed), then jitter from default_rng(seed + 7).
    """
    pts, _, col = sample_surface(scene, n, seed)
    rng = np.random.default_rng(seed + 7)
    pts = pts + rng.normal(0.0, noise, pts.shape)
    return pts.astype(np.float32), col.astype(np.float32)


def ba_tracks(seed, n_cams=60, n_points=2000, width=1920, height=1440, max_views=8, noise_px=0.5,
              outlier_frac=0.01, rot_noise_deg=0.5, centre_noise=0.02, point_noise=0.02):
    """Synthetic bundle-adjustment problem on the spheres-and-planes scene.

    Ground truth: the ring cameras (rotation R_i, centre c_i) and n_points
    surface samples P_j.  A point is observed by a camera when it lies
    0.2 or more in front of it and projects inside the image (no occlusion
    test; sparse tracks), by at most max_views of those cameras chosen at
    random; points seen fewer than twice are dropped.  The measurements are
    made here, for input generation only, by the pinhole projection
    u = fx x/z + cx, v = fy y/z + cy of x = R (P - c), plus N(0, noise_px^2)
    pixel noise; a fraction outlier_frac of them is replaced by a uniform
    random pixel.  Initial state: rotations perturbed by exp([w]x) with
    w ~ N(0, rot_noise^2 I3) (radians from degrees), centres by
    N(0, centre_noise^2 I3), points by N(0, point_noise^2 I3); camera 0 keeps
    its true pose and camera 1 its true centre coordinate along the axis of
    its largest baseline component to camera 0 (the fixed gauge).

    Draw order (default_rng(seed)): scene (spheres_planes_scene(seed)),
    points (sample_surface(scene, n_points, seed + 1)), then from
    default_rng(seed + 2): per point a permutation of its visible cameras,
    noise (n_obs, 2), outlier mask (n_obs,), outlier pixels (n_out, 2),
    rotation noise (n_cams, 3), centre noise (n_cams, 3), point noise (m, 3).
    Observations are ordered by point, then camera.
    """
    scene = spheres_planes_scene(seed)
    pts = sample_surface(scene, n_points, seed + 1)[0]
    cams = ring_cameras(n_cams, width, height)
    R = np.stack([np.asarray(c["viewmat"][:, :3], np.float64) for c in cams])
    t = np.stack([np.asarray(c["viewmat"][:, 3], np.float64) for c in cams])
    # orthonormalise the float32-stored rotations so that the truth is exact
    U, _, Vt = np.linalg.svd(R)
    R = U @ Vt
    centre = -np.einsum("cji,cj->ci", R, t)
    fx, fy, cx, cy = (float(cams[0][k]) for k in ("fx", "fy", "cx", "cy"))
    xc = np.einsum("cij,mcj->mci", R, pts[:, None, :] - centre[None, :, :])
    z = xc[..., 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        u = fx * xc[..., 0] / z + cx
        v = fy * xc[..., 1] / z + cy
    vis = (z > 0.2) & (u >= 0) & (u < width) & (v >= 0) & (v < height)
    rng = np.random.default_rng(seed + 2)
    keep, obs_cam, obs_pt = [], [], []
    for j in range(pts.shape[0]):
        cs = np.nonzero(vis[j])[0]
        if cs.size < 2:
            continue
        cs = np.sort(rng.permutation(cs)[:max_views])
        m = len(keep)
        keep.append(j)
        obs_cam.append(cs)
        obs_pt.append(np.full(cs.size, m))
    keep = np.asarray(keep)
    obs_cam = np.concatenate(obs_cam).astype(np.uint32)
    obs_pt = np.concatenate(obs_pt).astype(np.uint32)
    P = pts[keep]
    uv = np.stack([u[keep[obs_pt], obs_cam], v[keep[obs_pt], obs_cam]], 1)
    uv = uv + rng.normal(0.0, noise_px, uv.shape)
    out = rng.uniform(0.0, 1.0, obs_cam.size) < outlier_frac
    uv[out] = rng.uniform(0.0, 1.0, (int(out.sum()), 2)) * np.array([width, height])

    def rodrigues(w):
        th = np.linalg.norm(w, axis=1)[:, None, None]
        K = np.zeros((w.shape[0], 3, 3))
        K[:, 0, 1], K[:, 0, 2], K[:, 1, 2] = -w[:, 2], w[:, 1], -w[:, 0]
        K[:, 1, 0], K[:, 2, 0], K[:, 2, 1] = w[:, 2], -w[:, 1], w[:, 0]
        th = np.where(th == 0, 1e-300, th)
        return np.eye(3) + np.sin(th) / th * K + (1 - np.cos(th)) / th ** 2 * (K @ K)

    wn = rng.normal(0.0, math.radians(rot_noise_deg), (n_cams, 3))
    R0 = R @ rodrigues(wn)
    c0 = centre + rng.normal(0.0, centre_noise, centre.shape)
    P0 = P + rng.normal(0.0, point_noise, P.shape)
    axis = int(np.argmax(np.abs(centre[1] - centre[0])))
    R0[0], c0[0] = R[0], centre[0]
    c0[1, axis] = centre[1, axis]
    return dict(fx=fx, fy=fy, cx=cx, cy=cy, width=width, height=height, R_true=R, c_true=centre, P_true=P,
                obs_cam=obs_cam, obs_pt=obs_pt, obs_uv=uv, outlier=out, R0=R0, c0=c0, P0=P0, gauge_axis=axis)


def _value_noise(table: np.ndarray, p: np.ndarray) -> np.ndarray:
    """Trilinear interpolation of a periodic random lattice (table (n, n, n))
    at points p (m, 3) given in lattice units."""
    n = table.shape[0]
    f = np.floor(p)
    w = p - f
    i = f.astype(np.int64) % n
    out = np.zeros(p.shape[0])
    for dx in (0, 1):
        wx = w[:, 0] if dx else 1.0 - w[:, 0]
        for dy in (0, 1):
            wy = w[:, 1] if dy else 1.0 - w[:, 1]
            for dz in (0, 1):
                wz = w[:, 2] if dz else 1.0 - w[:, 2]
                out += wx * wy * wz * table[(i[:, 0] + dx) % n, (i[:, 1] + dy) % n, (i[:, 2] + dz) % n]
    return out


def textured_views(scene: Scene, cams: list, seed: int = 0, speckle=((0.012, 0.12), (0.04, 0.08)),
                   near=0.2):
    """Ray-cast greyscale views of the spheres-and-planes scene with their
    exact depth maps (multi-view stereo inputs).

    Pixel (x, y) of a camera (the float32-stored intrinsics and [R|t], taken
    as float64) casts the ray X(z) = R^T (z ((x - cx)/fx, (y - cy)/fy, 1) - t);
    its depth is the smallest camera z >= near at which it meets a sphere or
    a plane rectangle, 0 where it meets nothing.  Intensity = luma
    (0.299, 0.587, 0.114) of the scene's procedural colour at the hit plus
    solid value noise: for each (cell, amplitude) of `speckle`, amplitude x
    a trilinearly interpolated 64^3 lattice of U[-1, 1] values at the hit
    point divided by cell; clipped to [0, 1] and stored as uint8
    floor(255 v + 0.5).  Background pixels are 0.

    Draw order (default_rng(seed)): one 64^3 lattice per speckle octave.
    Returns (grey uint8 (V, H, W), depth float32 (V, H, W)).
    """
    rng = np.random.default_rng(seed)
    tables = [rng.uniform(-1.0, 1.0, (64, 64, 64)) for _ in speckle]
    S = len(scene.radii)
    greys, depths = [], []
    for cam in cams:
        W, H = cam["width"], cam["height"]
        vm = np.asarray(cam["viewmat"], np.float64)
        R, t = vm[:, :3], vm[:, 3]
        o = -R.T @ t
        ys, xs = np.mgrid[0:H, 0:W]
        dc = np.stack([(xs.ravel() - cam["cx"]) / cam["fx"], (ys.ravel() - cam["cy"]) / cam["fy"],
                       np.ones(W * H)], 1)
        d = dc @ R                      # world direction per unit camera depth
        best = np.full(W * H, np.inf)
        sid = np.full(W * H, -1, np.int64)
        for s in range(S):
            oc = o - scene.centres[s]
            a = (d * d).sum(1)
            b = 2.0 * (d @ oc)
            c = oc @ oc - scene.radii[s] ** 2
            disc = b * b - 4.0 * a * c
            ok = disc >= 0
            sq = np.sqrt(np.where(ok, disc, 0.0))
            z0 = (-b - sq) / (2.0 * a)
            z1 = (-b + sq) / (2.0 * a)
            z = np.where(z0 >= near, z0, z1)
            hit = ok & (z >= near) & (z < best)
            best = np.where(hit, z, best)
            sid = np.where(hit, s, sid)
        for k, (po, ua, va, nn, ul, vl) in enumerate(scene.planes):
            den = d @ nn
            with np.errstate(divide="ignore", invalid="ignore"):
                z = ((po - o) @ nn) / den
                q = o + z[:, None] * d - po
                u, v = q @ ua, q @ va
            hit = (np.abs(den) > 1e-12) & (z >= near) & (z < best) & (u >= 0) & (u <= ul) & (v >= 0) & (v <= vl)
            best = np.where(hit, z, best)
            sid = np.where(hit, S + k, sid)
        hitm = sid >= 0
        p = o + best[hitm, None] * d[hitm]
        col = _texture(scene, sid[hitm], p)
        g = col @ np.array([0.299, 0.587, 0.114])
        for (cell, amp), tab in zip(speckle, tables):
            g = g + amp * _value_noise(tab, p / cell)
        grey = np.zeros(W * H)
        grey[hitm] = np.clip(g, 0.0, 1.0)
        greys.append(np.floor(255.0 * grey + 0.5).astype(np.uint8).reshape(H, W))
        dep = np.zeros(W * H)
        dep[hitm] = best[hitm]
        depths.append(dep.astype(np.float32).reshape(H, W))
    return np.stack(greys), np.stack(depths)
