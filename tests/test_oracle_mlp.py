"""Pins for the seeding network's oracle: library bfloat16 rounding, the
normal distribution's closed forms, a permutation network evaluated by hand,
float64 finite differences, rotation/scale invariances of the features, the
matrix logarithm from scipy, scipy's rotation algebra and the fallback rules
on constructed cases."""

import math

import numpy as np
import pytest
import torch
from scipy.linalg import logm
from scipy.spatial.transform import Rotation
from scipy.stats import norm

import synth
from oracle import mlp
from oracle import seed as o_seed


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=4000) * 10.0 ** rng.integers(-6, 6, 4000),
                        [0.0, -0.0, 1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8), 3.0e38]])
    x = x.astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16(x), want)
    # ties go to the even mantissa
    assert mlp.bf16(np.float32(1 + 2 ** -8)) == 1.0
    assert mlp.bf16(np.float32(1 + 3 * 2 ** -8)) == 1 + 2 ** -6


def test_gelu_closed_forms():
    z = np.linspace(-6, 6, 97)
    np.testing.assert_allclose(mlp.gelu(z), z * norm.cdf(z), rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(mlp.gelu_grad(z), norm.cdf(z) + z * norm.pdf(z), rtol=1e-13, atol=1e-15)
    assert mlp.gelu_grad(np.array(0.0)) == 0.5


def _perm_net(seed):
    """Weights that pick and scale one input per output, with biases."""
    rng = np.random.default_rng(seed)
    parts, picks = [], []
    for (o, i) in ((64, 64), (64, 64), (64, 64), (8, 64)):
        p = rng.permutation(i)[:o]
        d = rng.uniform(0.5, 1.5, o)
        W = np.zeros((o, i))
        W[np.arange(o), p] = d
        b = rng.normal(size=o) * 0.1
        parts += [W, b]
        picks.append((p, d, b))
    return mlp.flatten(parts), picks


def test_forward_of_permutation_network_by_hand():
    w, picks = _perm_net(1)
    X = synth.random_normal(2, (5, 64)).astype(np.float64)
    Y, _ = mlp.forward(w, X, emulate=False)
    for r in range(5):
        h = X[r]
        for li, (p, d, b) in enumerate(picks):
            z = np.array([d[o] * h[p[o]] + b[o] for o in range(len(p))])
            h = z * norm.cdf(z) if li < 3 else z
        np.testing.assert_allclose(Y[r], h, rtol=1e-12, atol=1e-14)


def test_backward_matches_finite_differences():
    w = synth.random_normal(3, mlp.N_WEIGHTS, 0.25).astype(np.float64)
    X = synth.random_normal(4, (6, 64)).astype(np.float64)
    dY = synth.random_normal(5, (6, 8)).astype(np.float64)
    Y, cache = mlp.forward(w, X, emulate=False)
    g = mlp.backward(w, cache, dY, emulate=False)
    rng = np.random.default_rng(6)
    off = 0
    h = 1e-5
    for s in mlp.SHAPES:            # one direction per weight array
        k = int(np.prod(s))
        v = np.zeros(mlp.N_WEIGHTS)
        v[off:off + k] = rng.normal(size=k)
        fp = (mlp.forward(w + h * v, X, emulate=False)[0] * dY).sum()
        fm = (mlp.forward(w - h * v, X, emulate=False)[0] * dY).sum()
        fd = (fp - fm) / (2 * h)
        an = g @ v
        assert abs(fd - an) <= 1e-6 * abs(an) + 1e-9, (s, fd, an)
        off += k


def test_emulation_stays_within_bfloat16_bound():
    # Rounding every operand to 8 significant bits moves the outputs by at
    # most a few 2^-8 relative to their scale, and never leaves them equal.
    w = synth.random_normal(7, mlp.N_WEIGHTS, 0.15).astype(np.float64)
    X = synth.random_normal(8, (32, 64)).astype(np.float64)
    Ye, ce = mlp.forward(w, X, emulate=True)
    Yx, cx = mlp.forward(w, X, emulate=False)
    d = np.abs(Ye - Yx).max() / np.abs(Yx).max()
    assert 1e-5 < d < 3e-2
    dY = synth.random_normal(9, (32, 8)).astype(np.float64)
    ge = mlp.backward(w, ce, dY, emulate=True)
    gx = mlp.backward(w, cx, dY, emulate=False)
    d = np.abs(ge - gx).max() / np.abs(gx).max()
    assert 1e-5 < d < 3e-2


def _cloud(seed, n=300):
    rng = np.random.default_rng(seed)
    p = rng.normal(size=(n, 3)) * np.array([0.6, 0.3, 0.05])
    return p.astype(np.float32)


def _feat(points, i):
    ids, d2 = o_seed.knn_one(points, i)
    return mlp.frame_features(points, i, ids, d2)


def test_features_are_rigid_motion_invariant():
    P = _cloud(10)
    Q = Rotation.from_rotvec([0.4, -1.1, 0.7]).as_matrix()
    P2 = (P.astype(np.float64) @ Q.T + np.array([0.3, -0.2, 0.5])).astype(np.float32)
    for i in (0, 17, 123):
        x1, b1, m1 = _feat(P, i)
        x2, b2, m2 = _feat(P2, i)
        assert m1["gap12"] > 1e-3 and m1["gap01"] > 1e-3 and m1["m3"] > 1e-3
        np.testing.assert_allclose(x2, x1, atol=2e-4)
        np.testing.assert_allclose(b2["R"], Q @ b1["R"], atol=2e-4)


def test_features_scale_invariance_exact_power_of_two():
    P = _cloud(11)
    for i in (3, 50):
        x1, b1, _ = _feat(P, i)
        x2, b2, _ = _feat(P * np.float32(8.0), i)
        np.testing.assert_allclose(x2, x1, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(b2["log_scales"], b1["log_scales"] + math.log(8.0), rtol=0, atol=1e-12)


def test_features_structure():
    P = _cloud(12)
    for i in (0, 9, 200):
        ids, d2 = o_seed.knn_one(P, i)
        x, b, _ = mlp.frame_features(P, i, ids, d2)
        R = b["R"]
        np.testing.assert_allclose(R.T @ R, np.eye(3), atol=1e-12)
        assert abs(np.linalg.det(R) - 1) < 1e-12
        off = x[:48].reshape(16, 3)
        assert (off[:, 0] ** 3).sum() >= 0 and (off[:, 1] ** 3).sum() >= 0
        nb = P[ids].astype(np.float64)
        C = np.cov(nb.T, bias=True)                      # library covariance
        s_t = np.sqrt(d2[:3]).mean()
        np.testing.assert_allclose(x[48:57].reshape(3, 3), R.T @ C @ R / s_t ** 2, atol=1e-12)
        lam = np.sort(np.linalg.eigvalsh(C))[::-1]
        np.testing.assert_allclose(np.diag(x[48:57].reshape(3, 3)), lam / s_t ** 2, rtol=1e-9)
        np.testing.assert_allclose(np.linalg.norm(off, axis=1) * s_t, np.sqrt(d2), rtol=1e-9)
        assert (x[57:] == 0).all()
        # the base covariance is the plain seed's (matrix logarithm by scipy)
        s = o_seed.seed_points(P, np.zeros((len(P), 3)), [i])[0]
        np.testing.assert_allclose(mlp.log_sigma(b["log_scales"], R), logm(s["sigma"]).real, atol=1e-9)
        np.testing.assert_allclose(Rotation.from_quat(np.roll(b["q"], -1)).as_matrix(), R, atol=1e-12)


def test_planar_neighbourhood_has_flat_features():
    rng = np.random.default_rng(13)
    P = np.zeros((200, 3), np.float32)
    P[:, :2] = rng.uniform(-1, 1, (200, 2))
    x, b, _ = _feat(P, 7)
    assert np.abs(x[2:48:3]).max() < 1e-12
    assert abs(abs(b["R"][2, 2]) - 1) < 1e-12


def test_quaternion_helpers_match_scipy():
    rng = np.random.default_rng(14)
    qs = list(rng.normal(size=(20, 4))) + [np.array(v, float) for v in
                                           ([5, 1, 1, 1], [1, 5, 1, 1], [1, 1, 5, 1], [1, 1, 1, 5])]
    for q in qs:
        R = Rotation.from_quat(np.roll(q, -1)).as_matrix()
        np.testing.assert_allclose(mlp.rot_of_quat(q), R, atol=1e-12)
        q2 = mlp.quat_of_rot(R)
        qn = q / np.linalg.norm(q)
        assert min(np.abs(q2 - qn).max(), np.abs(q2 + qn).max()) < 1e-12
    for a, b in zip(qs[:10], qs[10:20]):
        want = (Rotation.from_quat(np.roll(a, -1)) * Rotation.from_quat(np.roll(b, -1))).as_matrix()
        np.testing.assert_allclose(mlp.rot_of_quat(mlp.quat_mul(a, b)), want, atol=1e-12)


def _pairs(seed, n=7):
    rng = np.random.default_rng(seed)
    R = Rotation.random(n, random_state=seed).as_matrix()
    logs = rng.normal(size=(n, 3)) - 3
    Y = rng.normal(size=(n, 8)) * 0.3
    Y[:, 3] += 1
    tq = rng.normal(size=(n, 4))
    tl = rng.normal(size=(n, 3)) - 3
    P = np.zeros((14, n))
    P[3:6] = tl.T
    P[6:10] = tq.T
    P[10] = rng.normal(size=n)
    return R, logs, Y, P


def test_targets_and_loss_by_matrix_logarithm():
    R, logs, Y, P = _pairs(15)
    M, lg = mlp.targets(P, range(P.shape[1]))
    per, loss, _ = mlp.seed_loss(Y, R, logs, M, lg)
    for j in range(len(Y)):
        Rt = Rotation.from_quat(np.roll(P[6:10, j], -1)).as_matrix()
        S_t = Rt @ np.diag(np.exp(2 * P[3:6, j])) @ Rt.T
        np.testing.assert_allclose(M[j], logm(S_t).real, atol=1e-9)
        Rh = R[j] @ Rotation.from_quat(np.roll(Y[j, 3:7], -1)).as_matrix()
        S_h = Rh @ np.diag(np.exp(2 * (logs[j] + Y[j, :3]))) @ Rh.T
        want = ((logm(S_h).real - logm(S_t).real) ** 2).sum() + (mlp.LOGIT0 + Y[j, 7] - P[10, j]) ** 2
        assert abs(per[j] - want) <= 1e-8 * want
    assert abs(loss - per.mean()) < 1e-12


def test_loss_gradient_finite_differences_and_invariances():
    R, logs, Y, P = _pairs(16)
    M, lg = mlp.targets(P, range(P.shape[1]))
    _, loss, g = mlp.seed_loss(Y, R, logs, M, lg)
    rng = np.random.default_rng(17)
    h = 1e-6
    for _ in range(4):
        V = rng.normal(size=Y.shape)
        fd = (mlp.seed_loss(Y + h * V, R, logs, M, lg)[1] - mlp.seed_loss(Y - h * V, R, logs, M, lg)[1]) / (2 * h)
        an = (g * V).sum()
        assert abs(fd - an) <= 1e-6 * abs(an) + 1e-10
    Y2 = Y.copy()
    Y2[:, 3:7] *= -2.5                      # q and -q, any scale
    assert abs(mlp.seed_loss(Y2, R, logs, M, lg)[1] - loss) < 1e-12 * loss


def test_zero_last_layer_gives_the_plain_seed():
    w = mlp.zero_last_layer(synth.random_normal(18, mlp.N_WEIGHTS).astype(np.float64))
    P = _cloud(19)
    ids = [4, 40, 140]
    nbr, d2 = o_seed.knn(P, ids)
    X, R, q, logs, _ = mlp.features(P, ids, nbr, d2)
    for emulate in (True, False):
        Y, _ = mlp.forward(w, X, emulate=emulate)
        np.testing.assert_array_equal(Y, np.tile(mlp.identity_output_bias(), (3, 1)))
    pca = np.random.default_rng(20).normal(size=(3, 14))
    out, fb, _ = mlp.apply(Y, R, q, logs, pca)
    assert not fb.any()
    np.testing.assert_array_equal(out[:, :3], pca[:, :3])
    np.testing.assert_array_equal(out[:, 11:], pca[:, 11:])
    assert (out[:, 10] == mlp.LOGIT0).all()
    for j, i in enumerate(ids):
        s = o_seed.seed_points(P, np.zeros((len(P), 3)), [i])[0]
        np.testing.assert_allclose(o_seed.sigma_from_params(out[j, 3:6], out[j, 6:10]), s["sigma"],
                                   rtol=1e-9, atol=1e-15)
    # a target equal to the base seed costs nothing
    M = mlp.log_sigma(logs, R)
    assert mlp.seed_loss(Y, R, logs, M, np.full(3, mlp.LOGIT0))[1] < 1e-25


@pytest.mark.parametrize("case,fallback", [
    ("nan", True), ("tiny_q", True), ("dlog_2.5", True), ("dlog_1.5", False),
    ("tilt_70", True), ("tilt_50", False), ("normal_in_plane", True)])
def test_fallback_rules(case, fallback):
    R = Rotation.from_rotvec([0.3, 0.2, -0.5]).as_matrix()
    q = mlp.quat_of_rot(R)
    ls = np.array([math.log(0.05), math.log(0.05), math.log(0.005)])
    y = mlp.identity_output_bias()
    if case == "nan":
        y[0] = np.nan
    elif case == "tiny_q":
        y[3:7] = 1e-7
    elif case == "dlog_2.5":
        y[1] = -2.5
    elif case == "dlog_1.5":
        y[1] = -1.5
    elif case.startswith("tilt"):
        a = math.radians(float(case[5:]))
        y[3:7] = [math.cos(a / 2), math.sin(a / 2), 0, 0]      # about e1: tilts e3 by a
    elif case == "normal_in_plane":
        y[0:3] = [-1.9, 0.0, 1.9]                              # smallest scale now along e1
    pca = np.arange(14, dtype=float)[None]
    out, fb, _ = mlp.apply(y[None], R[None], q[None], ls[None], pca)
    assert fb[0] == fallback
    if fallback:
        np.testing.assert_array_equal(out, pca)
    else:
        Rh = R @ mlp.rot_of_quat(y[3:7])
        np.testing.assert_allclose(mlp.rot_of_quat(out[0, 6:10]), Rh, atol=1e-12)
        np.testing.assert_allclose(out[0, 3:6], ls + y[:3], atol=0)
