"""Pins for the oracle's EWA projection: closed forms, a numerical Jacobian,
independent quaternion algebra, a library eigensolver and finite differences
of its backward."""

import math

import numpy as np
import pytest
import torch

import synth
from oracle import projection as pj
from oracle.projection import project, project_vjp


def _one(mu, log_s, q, logit=0.0, dc=(0.0, 0.0, 0.0), sh_degree=0):
    P = np.zeros((synth.param_rows(sh_degree), 1))
    P[0:3, 0] = mu
    P[3:6, 0] = log_s
    P[6:10, 0] = q
    P[10, 0] = logit
    P[11:14, 0] = dc
    return P


def _ident_cam(W=128, H=128, f=128.0):
    return synth.make_camera(W, H, f, f, W / 2, H / 2, np.eye(3), np.zeros(3))


def test_isotropic_on_axis_closed_form():
    # An isotropic Gaussian of scale s on the optical axis at depth z projects
    # to the image centre with Sigma2D = ((f s / z)^2 + 0.3) I.
    s, z, f = 0.05, 4.0, 128.0
    cam = _ident_cam(f=f)
    P = _one((0, 0, z), (math.log(s),) * 3, (0.3, -0.2, 0.5, 0.7))
    r = project(P, cam)
    var = (f * s / z) ** 2 + 0.3
    assert r["visible"][0]
    np.testing.assert_allclose([r["u"][0], r["v"][0]], [64.0, 64.0], rtol=0, atol=1e-12)
    np.testing.assert_allclose([r["A"][0], r["B"][0], r["C"][0]], [1 / var, 0.0, 1 / var], atol=1e-12)
    assert r["radius"][0] == math.ceil(3 * math.sqrt(var))
    assert r["depth32"][0] == np.float32(z)


def test_covariance_matches_numerical_jacobian():
    # Off-axis anisotropic Gaussian under a rotated camera: Sigma2D must equal
    # J_num W Sigma W^T J_num^T + 0.3 I with J_num the central-difference
    # Jacobian of x_c -> (fx x/z, fy y/z) (no clamp active here).
    cams = synth.ring_cameras(4, 320, 240)
    cam = cams[1]
    mu = np.array([0.3, 0.5, -0.2])
    log_s = np.array([-2.0, -2.7, -3.5])
    q = np.array([0.9, 0.1, -0.3, 0.2])
    P = _one(mu, log_s, q)
    r = project(P, cam, with_grad=True)
    Wm = np.asarray(cam["viewmat"], np.float64)
    xc = Wm[:, :3] @ mu + Wm[:, 3]

    def persp(p):
        return np.array([cam["fx"] * p[0] / p[2], cam["fy"] * p[1] / p[2]])

    h = 1e-6
    J = np.stack([(persp(xc + h * e) - persp(xc - h * e)) / (2 * h) for e in np.eye(3)], 1)
    qn = q / np.linalg.norm(q)
    # rotation from quaternion via v' = q v q*, built with quaternion products
    def qmul(a, b):
        w1, x1, y1, z1 = a
        w2, x2, y2, z2 = b
        return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                         w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])
    conj = qn * np.array([1, -1, -1, -1])
    R = np.stack([qmul(qmul(qn, np.r_[0, e]), conj)[1:] for e in np.eye(3)], 1)
    Sig = R @ np.diag(np.exp(2 * log_s)) @ R.T
    T = J @ Wm[:, :3]
    S2 = T @ Sig @ T.T + 0.3 * np.eye(2)
    Q = np.linalg.inv(S2)
    np.testing.assert_allclose([r["A"][0], r["B"][0], r["C"][0]], [Q[0, 0], Q[0, 1], Q[1, 1]], rtol=1e-7)
    np.testing.assert_allclose([r["u"][0], r["v"][0]], persp(xc) + [cam["cx"], cam["cy"]], rtol=1e-13)
    # radius against a library eigensolver: r = ceil(3 sqrt(lambda_max))
    lam = np.linalg.eigvalsh(S2).max()
    assert r["radius"][0] == math.ceil(3 * math.sqrt(lam))


def test_quat_to_rot_is_a_rotation():
    q = torch.as_tensor(np.random.default_rng(1).normal(size=(50, 4)))
    q = q / q.norm(dim=1, keepdim=True)
    R = pj.quat_to_rot(q).numpy()
    for Ri in R:
        np.testing.assert_allclose(Ri @ Ri.T, np.eye(3), atol=1e-14)
        assert abs(np.linalg.det(Ri) - 1) < 1e-13


def test_sigma2d_spd_and_conic_inverse():
    P = synth.random_gaussians(3, 300, sh_degree=2)
    cam = _ident_cam()
    r = project(P, cam, with_grad=True)
    aux = r["aux"]
    a, b, c = (aux[k].detach().numpy() for k in ("a", "b", "c"))
    vis = r["visible"]
    assert vis.sum() > 250
    assert (a[vis] > 0).all() and (a * c - b * b)[vis].min() > 0
    np.testing.assert_allclose((a * r["A"] + b * r["B"])[vis], 1.0, rtol=1e-12)
    np.testing.assert_allclose((b * r["A"] + c * r["B"])[vis], 0.0, atol=1e-12)


def test_dc_colour_closed_form():
    # Only the degree-0 coefficient: colour = f00 / (2 sqrt(pi)) + 1/2 for any view.
    P, cam, _ = synth.cfg1_inputs(0)
    r = project(P, cam)
    c = P[11:14].astype(np.float64) / (2 * math.sqrt(math.pi)) + 0.5
    np.testing.assert_allclose(np.stack([r["r"], r["g"], r["b"]]), c, rtol=1e-14, atol=1e-15)
    assert (c >= 0).all() and (c <= 1).all()


def test_culling_cases():
    cam = _ident_cam()
    P = np.concatenate([
        _one((0, 0, 0.1), (-3, -3, -3), (1, 0, 0, 0)),     # in front of the near plane
        _one((0, 0, -3), (-3, -3, -3), (1, 0, 0, 0)),      # behind the camera
        _one((40, 0, 4), (-3, -3, -3), (1, 0, 0, 0)),      # far off screen right
        _one((0, 0, 4), (-3, -3, -3), (1, 0, 0, 0)),       # centre: visible
        _one((-1.0, -1.0, 4), (-3, -3, -3), (1, 0, 0, 0)),  # inside, near a corner
    ], 1)
    r = project(P, cam)
    assert r["visible"].tolist() == [False, False, False, True, True]
    assert (r["tiles_touched"][:3] == 0).all() and (r["radius"][:3] == 0).all()


@pytest.mark.parametrize("deg", [0, 3])
def test_projection_vjp_finite_differences(deg):
    # <g, d out/d theta . v> by central differences vs the reverse-mode VJP,
    # on a view where some Gaussians sit beyond the J clamp (frozen branch).
    rng = np.random.default_rng(7 + deg)
    P = synth.random_gaussians(11, 40, sh_degree=deg, spread=1.6).astype(np.float64)
    P[0, :5] += 4.8                      # push a few just past the clamp limit,
    P[3:6, :5] = -0.7                    # large enough to stay on screen
    cam = synth.ring_cameras(8, 200, 150, radius=6.0)[0]
    P[0:3] = P[0:3] - np.array([[0], [0], [4.0]])   # centre near the ring origin
    base = project(P, cam)
    vis = base["visible"]
    assert vis.sum() > 20 and base["clamp_xy"].any()
    g2d = rng.normal(size=(9, P.shape[1]))
    G = project_vjp(P, cam, g2d, vis)
    for trial in range(3):
        V = rng.normal(size=P.shape)
        h = 1e-6

        def f(theta):
            r = project(theta, cam)
            return sum((g2d[i][vis] * r[k][vis]).sum() for i, k in enumerate(pj.OUT_FIELDS))

        rp, rm = project(P + h * V, cam), project(P - h * V, cam)
        assert (rp["clamp_xy"] == base["clamp_xy"]).all() and (rm["clamp_xy"] == base["clamp_xy"]).all()
        assert (rp["colour_clamped"] == base["colour_clamped"]).all()
        fd = (f(P + h * V) - f(P - h * V)) / (2 * h)
        an = (G * V).sum()
        assert abs(fd - an) <= 1e-6 * abs(an) + 1e-9, (fd, an)
