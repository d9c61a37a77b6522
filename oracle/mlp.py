"""Learned seeding network (oracle; test infrastructure only).

PocketGS seeds each Gaussian from local surface statistics (Sec.
"Prior-Conditioned Gaussian Parameterization", equations for C_i and s_t).
The network here is not in the paper: it predicts corrections to that
disc-like seed from the point's neighbourhood.  Its definition is this
project's proposal; the oracle fixes the arithmetic, not the network's
quality (parity of the trained network's usefulness is measured by PSNR only).

Features of point i (neighbours p_k = its 16 nearest, nearest first;
C = covariance of the 16 about their centroid, as in the equation for C_i;
s_t = mean distance to the first 3 neighbours, as in the equation for s_t):
  * frame R = [e1 e2 e3] (columns): eigenvectors of C for the largest and the
    middle eigenvalue, each signed so that sum_k ((p_k - p_i) . e)^3 >= 0,
    and e3 = e1 x e2 (so e3 is the seed normal up to sign and det R = +1);
  * x[0:48]  = offsets (p_k - p_i) in the frame, / s_t, neighbour-major;
    x[48:57] = R^T C R / s_t^2, row-major; x[57:64] = 0.
Base seed: log-scales (log s_t, log s_t, log(r_normal s_t)), rotation R with
quaternion q_base, opacity logit(0.1): the covariance of the plain seed.

Network: 64 -> 64 -> 64 -> 64 -> 8, exact-erf GELU after each hidden layer,
flat weights [W1 (64x64, out-major), b1, W2, b2, W3, b3, W4 (8x64), b4].
Outputs y = (d log-scales (3), q_out (4), d logit (1)).  The seed is
log-scales + d, q_base (x) q_out/|q_out|, logit(0.1) + d logit, with a fall
back to the plain seed when y is not finite, |q_out| < 1e-6, a |d| exceeds 2,
or the axis of the smallest predicted scale is more than 60 degrees from the
plain seed's normal.  With W4 = 0 and b4 = (0,0,0,1,0,0,0,0) the network
returns the plain seed exactly.

Training loss per pair: ||log S_hat - log S*||_F^2 + (logit_hat - logit*)^2,
where log S = R diag(2 log s) R^T is the matrix logarithm of R diag(s^2) R^T;
the reported loss is the mean over pairs.

The GPU multiplies bfloat16 operands and accumulates in float32.  With
emulate=True, `forward` and `backward` round the same operands at the same
points (round to nearest, ties to even) and accumulate in float64.
"""

from __future__ import annotations

import math

import numpy as np
import torch

K_NN = 16
K_S = 3
IN = 64
HID = 64
OUT = 8
R_NORMAL = 0.1
LOGIT0 = math.log(0.1 / 0.9)
MAX_DLOG = 2.0
MIN_COS = 0.5          # cos 60 degrees
MIN_QNORM = 1e-6

SHAPES = [(HID, IN), (HID,), (HID, HID), (HID,), (HID, HID), (HID,), (OUT, HID), (OUT,)]
N_WEIGHTS = sum(int(np.prod(s)) for s in SHAPES)


# --------------------------------------------------------------- weights

def unflatten(w):
    w = np.asarray(w, np.float64)
    assert w.size == N_WEIGHTS
    out, off = [], 0
    for s in SHAPES:
        k = int(np.prod(s))
        out.append(w[off:off + k].reshape(s))
        off += k
    return out


def flatten(parts):
    return np.concatenate([np.asarray(p, np.float64).reshape(-1) for p in parts])


def identity_output_bias():
    b = np.zeros(OUT)
    b[3] = 1.0
    return b


def zero_last_layer(w):
    """Copy of w with W4 = 0 and b4 = (0,0,0,1,0,0,0,0)."""
    p = unflatten(np.array(w, np.float64, copy=True))
    p[6] = np.zeros_like(p[6])
    p[7] = identity_output_bias()
    return flatten(p)


# ------------------------------------------------------------ arithmetic

def bf16(x):
    """Round float32 values to bfloat16 (nearest, ties to even), as float64."""
    f = np.ascontiguousarray(np.asarray(x, np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    r = np.where(np.isnan(f), u | 0x400000, r)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(z):
    from scipy.special import erf
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    from scipy.special import erf
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def _id(a):
    return np.asarray(a, np.float64)


def forward(w, X, emulate=True):
    """Y (B, 8) for inputs X (B, 64), and the activations for `backward`.
    The float32 inputs are rounded to bfloat16 first when emulating."""
    W = unflatten(w)
    r = bf16 if emulate else _id
    h = np.asarray(X, np.float64)
    H, Z = [], []
    for l in range(3):
        hin = r(h)
        z = hin @ r(W[2 * l]).T + W[2 * l + 1]
        H.append(hin)
        Z.append(z)
        h = gelu(z)
    hin = r(h)
    H.append(hin)
    return hin @ r(W[6]).T + W[7], dict(H=H, Z=Z)


def backward(w, cache, dY, emulate=True):
    """Gradient of sum(dY * Y) with respect to the flat weights.  Weight
    gradients take the rounded output gradient and the rounded activation;
    bias gradients sum the unrounded output gradient."""
    W = unflatten(w)
    r = bf16 if emulate else _id
    grads = [None] * 8
    dz = np.asarray(dY, np.float64)
    for l in (3, 2, 1, 0):
        dzr = r(dz)
        grads[2 * l] = dzr.T @ cache["H"][l]
        grads[2 * l + 1] = dz.sum(0)
        if l:
            dz = (dzr @ r(W[2 * l])) * gelu_grad(cache["Z"][l - 1])
    return flatten(grads)


# ------------------------------------------------------------ geometry

def rot_of_quat(q):
    w, x, y, z = np.asarray(q, np.float64) / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def quat_of_rot(R):
    """Unit quaternion (w, x, y, z) of a rotation matrix (Shepperd's method:
    branch on the largest of the trace and the diagonal)."""
    R = np.asarray(R, np.float64)
    t = np.trace(R)
    d = np.diag(R)
    k = int(np.argmax([t, d[0], d[1], d[2]]))
    if k == 0:
        s = 2.0 * math.sqrt(1.0 + t)
        q = [0.25 * s, (R[2, 1] - R[1, 2]) / s, (R[0, 2] - R[2, 0]) / s, (R[1, 0] - R[0, 1]) / s]
    elif k == 1:
        s = 2.0 * math.sqrt(1.0 + d[0] - d[1] - d[2])
        q = [(R[2, 1] - R[1, 2]) / s, 0.25 * s, (R[0, 1] + R[1, 0]) / s, (R[0, 2] + R[2, 0]) / s]
    elif k == 2:
        s = 2.0 * math.sqrt(1.0 - d[0] + d[1] - d[2])
        q = [(R[0, 2] - R[2, 0]) / s, (R[0, 1] + R[1, 0]) / s, 0.25 * s, (R[1, 2] + R[2, 1]) / s]
    else:
        s = 2.0 * math.sqrt(1.0 - d[0] - d[1] + d[2])
        q = [(R[1, 0] - R[0, 1]) / s, (R[0, 2] + R[2, 0]) / s, (R[1, 2] + R[2, 1]) / s, 0.25 * s]
    q = np.asarray(q)
    return q / np.linalg.norm(q)


def quat_mul(a, b):
    """Hamilton product, so that rot_of_quat(a (x) b) = rot_of_quat(a) rot_of_quat(b)."""
    aw, av = a[0], np.asarray(a[1:], np.float64)
    bw, bv = b[0], np.asarray(b[1:], np.float64)
    return np.concatenate([[aw * bw - av @ bv], aw * bv + bw * av + np.cross(av, bv)])


def log_sigma(log_scales, R):
    """R diag(2 log s) R^T for arrays (..., 3) and (..., 3, 3)."""
    R = np.asarray(R, np.float64)
    return (R * (2.0 * np.asarray(log_scales, np.float64))[..., None, :]) @ np.swapaxes(R, -1, -2)


# ------------------------------------------------------------ features

def frame_features(points, i, nbr, d2, r_normal=R_NORMAL):
    """Features (64,), base seed dict and decision margins of point i from
    its neighbour ids `nbr` and squared distances `d2` (nearest first)."""
    P = np.asarray(points, np.float32).astype(np.float64)
    nb = P[np.asarray(nbr[:K_NN], np.int64)]
    off = nb - P[i]
    D = nb - nb.mean(0)
    C = (D.T @ D) / K_NN
    lam, vec = np.linalg.eigh(C)                       # ascending
    es, m3 = [], []
    for col in (2, 1):
        e = vec[:, col].copy()
        m = float(((off @ e) ** 3).sum())
        if m < 0:
            e = -e
        es.append(e)
        m3.append(abs(m) / max(1e-300, float((np.abs(off) ** 3).sum())))
    R = np.stack([es[0], es[1], np.cross(es[0], es[1])], 1)
    s_t = float(np.sqrt(np.asarray(d2[:K_S], np.float64)).mean())
    x = np.zeros(IN)
    x[:48] = ((off @ R) / s_t).reshape(-1)
    x[48:57] = ((R.T @ C @ R) / (s_t * s_t)).reshape(-1)
    top = max(lam[2], 1e-300)
    margins = dict(gap12=(lam[2] - lam[1]) / top, gap01=(lam[1] - lam[0]) / top, m3=min(m3))
    base = dict(R=R, q=quat_of_rot(R), s_t=s_t,
                log_scales=np.array([math.log(s_t), math.log(s_t), math.log(r_normal * s_t)]))
    return x, base, margins


def features(points, queries, nbr, d2, r_normal=R_NORMAL):
    """Stacked `frame_features` for the query indices; nbr/d2 are indexed by
    query position.  Returns X (n, 64), base R (n, 3, 3), base quaternions
    (n, 4), base log-scales (n, 3) and the margins."""
    X, Rs, qs, ls, mg = [], [], [], [], []
    for j, i in enumerate(queries):
        x, b, m = frame_features(points, int(i), nbr[j], d2[j], r_normal)
        X.append(x)
        Rs.append(b["R"])
        qs.append(b["q"])
        ls.append(b["log_scales"])
        mg.append(m)
    return np.asarray(X), np.asarray(Rs), np.asarray(qs), np.asarray(ls), mg


# ------------------------------------------------------------ targets / loss

def targets(params, ids):
    """Training targets of Gaussians `ids` from canonical parameters
    [F][n]: log S* (n, 3, 3) and logit* (n,)."""
    P = np.asarray(params, np.float64)
    Ms, lg = [], []
    for i in ids:
        Ms.append(log_sigma(P[3:6, i], rot_of_quat(P[6:10, i])))
        lg.append(P[10, i])
    return np.asarray(Ms), np.asarray(lg)


def _rot_t(q):
    w, x, y, z = q.unbind(-1)
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ], -2)


def seed_loss(Y, base_R, base_logs, target_M, target_logit):
    """Per-pair losses (n,), their mean, and the gradient of the mean with
    respect to Y (float64 reverse-mode differentiation)."""
    Yt = torch.as_tensor(np.asarray(Y, np.float64)).clone().requires_grad_(True)
    qo = Yt[:, 3:7] / torch.linalg.norm(Yt[:, 3:7], dim=1, keepdim=True)
    R = torch.as_tensor(np.asarray(base_R, np.float64)) @ _rot_t(qo)
    s = torch.as_tensor(np.asarray(base_logs, np.float64)) + Yt[:, 0:3]
    L = (R * (2.0 * s)[:, None, :]) @ R.transpose(1, 2)
    M = torch.as_tensor(np.asarray(target_M, np.float64))
    lg = LOGIT0 + Yt[:, 7]
    per = ((L - M) ** 2).sum((1, 2)) + (lg - torch.as_tensor(np.asarray(target_logit, np.float64))) ** 2
    loss = per.mean()
    loss.backward()
    return per.detach().numpy(), float(loss.detach()), Yt.grad.numpy()


# ------------------------------------------------------------ seed

def apply(Y, base_R, base_q, base_logs, pca_cols):
    """Seeded canonical columns (n, 14) from network outputs Y (n, 8) and the
    plain seed's columns `pca_cols` (n, 14), with the fallback mask and the
    margins of the three fallback comparisons."""
    Y = np.asarray(Y, np.float64)
    out = np.array(pca_cols, np.float64, copy=True)
    fb = np.zeros(len(Y), bool)
    margins = []
    for j, y in enumerate(Y):
        qn = float(np.linalg.norm(y[3:7])) if np.isfinite(y).all() else 0.0
        if not np.isfinite(y).all() or qn < MIN_QNORM:
            fb[j] = True
            margins.append(dict(dlog=np.inf, cos=np.inf, scale_gap=np.inf, qnorm=qn))
            continue
        qo = y[3:7] / qn
        Rh = base_R[j] @ rot_of_quat(qo)
        s = base_logs[j] + y[0:3]
        k = int(np.argmin(s))
        c = abs(float(Rh[:, k] @ base_R[j][:, 2]))
        ss = np.sort(s)
        dl = float(np.abs(y[0:3]).max())
        margins.append(dict(dlog=abs(dl - MAX_DLOG), cos=abs(c - MIN_COS), scale_gap=ss[1] - ss[0],
                            qnorm=qn))
        if dl > MAX_DLOG or c < MIN_COS:
            fb[j] = True
            continue
        out[j, 3:6] = s
        out[j, 6:10] = quat_mul(base_q[j], qo)
        out[j, 10] = LOGIT0 + y[7]
    return out, fb, margins
