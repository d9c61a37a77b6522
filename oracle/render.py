"""Per-pixel front-to-back compositing, replay trace and backward (oracle).

Forward (Sec. "Explicit Computation Graph"; thresholds inherited from 3D
Gaussian Splatting and not stated by the paper): for each pixel centre p and
its tile's sorted list,

    d      = (u - p_x, v - p_y)
    power  = -1/2 (A dx^2 + 2 B dx dy + C dy^2)      skip if power > 0
    alpha  = min(0.99, o exp(power))                 skip if alpha < 1/255
    if T (1 - alpha) < 1e-4: stop (this splat is excluded)
    C     += T alpha c;   T <- T (1 - alpha)

and finally C += T bg.  The contributors k = 0..K-1 of a pixel are the
splats that passed; T_k = prod_{j<k} (1 - alpha_j); n_contrib is one plus the
list position of the last contributor.

The paper composes C_out = C_in (1 - alpha) + alpha c: read back to front,
C_in of contributor k is the colour of everything behind it,
    C_in_k = sum_{j>k} alpha_j c_j prod_{k<i<j} (1 - alpha_i) + bg prod_{j>k} (1 - alpha_j),
and applying the recursion from the last contributor (C_in = bg) to the
first reproduces C exactly.  The replay trace S = {id, C_in, alpha} (Sec.
"Bandwidth-Efficient Forward Replay Cache") records, per pixel and per
contributor, the sorted-list index id, C_in and the clamped alpha; count(u)
is the number of entries.

Backward (equation "backward_chain"): with G = dL/dC of the pixel,
dL/dC_out_k = T_k G (unrolling dL/dC_in = dL/dC_out (1 - alpha)), so
    dL/dc_k     = alpha_k T_k G
    dL/dalpha_k = < T_k G, c_k - C_in_k >
Two ways to get T_k and C_in_k: `cached` walks the trace front to back with
T_k as the running product of the cached alphas and C_in_k read from the
trace; `recompute` walks the tile list back to front from n_contrib starting
at T_final, re-evaluates alpha, recovers T_k = T_{k+1} / (1 - alpha_k) and
accumulates C_in as it goes (the recompute-based backward of 3D Gaussian
Splatting).  Both are then chained through alpha to the 2D parameters:
    alpha unclamped: dL/do += exp(power) dL/dalpha,  dL/dpower = alpha dL/dalpha
    alpha clamped at 0.99: no gradient
    dL/dA = -1/2 dx^2 dL/dpower, dL/dB = -dx dy dL/dpower, dL/dC = -1/2 dy^2 dL/dpower
    dL/du = -(A dx + B dy) dL/dpower, dL/dv = -(B dx + C dy) dL/dpower
and scattered to the canonical Gaussian pi(id) (index-mapping equation:
gradient of the canonical index += gradient of the sorted element).

Near-threshold decisions: a pixel is `marginal` if any of its evaluated
splats has alpha within 2e-5 relative of 1/255, o exp(power) within 2e-5
relative of 0.99, or T (1 - alpha) within 5e-5 relative of 1e-4 while still
active.  A float32 renderer may legitimately take the other branch there.
"""

from __future__ import annotations

import numpy as np

ALPHA_MIN = 1.0 / 255.0
ALPHA_MAX = 0.99
T_MIN = 1e-4
MARGIN_ALPHA = 2e-5
MARGIN_T = 5e-5

GRAD_FIELDS = ("u", "v", "A", "B", "C", "o", "r", "g", "b")


def _tile_pixels(tile, TX, TW, TH, W, H):
    tx, ty = tile % TX, tile // TX
    lx, ly = np.meshgrid(np.arange(TW), np.arange(TH))
    gx = (tx * TW + lx).ravel()
    gy = (ty * TH + ly).ravel()
    inside = (gx < W) & (gy < H)
    return gx[inside], gy[inside]


def render_tile(proj, bins, tile, TX, TW, TH, W, H, bg):
    """Forward over one tile; returns a trace dict for the backward."""
    gx, gy = _tile_pixels(tile, TX, TW, TH, W, H)
    px = gx + 0.5
    py = gy + 0.5
    P = px.size
    s, e = (int(t) for t in bins["ranges"][tile])
    L = e - s
    ids = bins["values"][s:e].astype(np.int64)
    T = np.ones(P)
    C = np.zeros((3, P))
    done = np.zeros(P, bool)
    last = np.zeros(P, np.int64)
    marg = np.zeros(P, bool)
    contrib = np.zeros((L, P), bool)
    alpha = np.zeros((L, P))
    gauss = np.zeros((L, P))
    clamped = np.zeros((L, P), bool)
    T_before = np.zeros((L, P))
    dxs = np.zeros((L, P))
    dys = np.zeros((L, P))
    for j in range(L):
        g = ids[j]
        if done.all():
            break
        dx = proj["u"][g] - px
        dy = proj["v"][g] - py
        power = -0.5 * (proj["A"][g] * dx * dx + proj["C"][g] * dy * dy) - proj["B"][g] * dx * dy
        G = np.exp(power)
        raw = proj["o"][g] * G
        a = np.minimum(ALPHA_MAX, raw)
        active = ~done
        skip = (power > 0.0) | (a < ALPHA_MIN)
        test_T = T * (1.0 - a)
        term = active & ~skip & (test_T < T_MIN)
        ok = active & ~skip & ~term
        marg |= active & (np.abs(a - ALPHA_MIN) <= MARGIN_ALPHA * ALPHA_MIN)
        marg |= active & (np.abs(raw - ALPHA_MAX) <= MARGIN_ALPHA * ALPHA_MAX)
        marg |= active & ~skip & (np.abs(test_T - T_MIN) <= MARGIN_T * T_MIN)
        col = np.array([proj["r"][g], proj["g"][g], proj["b"][g]])
        contrib[j] = ok
        alpha[j] = a
        gauss[j] = G
        clamped[j] = raw > ALPHA_MAX
        T_before[j] = T
        dxs[j] = dx
        dys[j] = dy
        C += np.where(ok, T * a, 0.0)[None, :] * col[:, None]
        T = np.where(ok, test_T, T)
        last = np.where(ok, j + 1, last)
        done |= term
    C_final = C + T[None, :] * np.asarray(bg, np.float64)[:, None]
    # C_in of every contributor: the over-recursion from the back, starting at bg
    C_in = np.zeros((L, 3, P))
    acc = np.tile(np.asarray(bg, np.float64)[:, None], (1, P))
    for j in range(L - 1, -1, -1):
        ok = contrib[j]
        if not ok.any():
            continue
        g = ids[j]
        col = np.array([proj["r"][g], proj["g"][g], proj["b"][g]])
        C_in[j] = np.where(ok[None, :], acc, 0.0)
        a = alpha[j]
        acc = np.where(ok[None, :], a[None, :] * col[:, None] + (1.0 - a[None, :]) * acc, acc)
    return dict(tile=tile, s=s, gx=gx, gy=gy, ids=ids, C=C_final, T=T, last=last,
                marg=marg, contrib=contrib, alpha=alpha, gauss=gauss, clamped=clamped,
                T_before=T_before, C_in=C_in, dx=dxs, dy=dys, over=acc)


def render_forward(proj, bins, cam, tile_w=16, tile_h=16, bg=(0.0, 0.0, 0.0), tiles=None):
    """Image (3,H,W), T_final (H,W), n_contrib (H,W), count (H,W), marginal (H,W)
    and the per-tile traces.  `tiles` restricts the work to a subset of tiles
    (other pixels stay zero / one)."""
    W, H = int(cam["width"]), int(cam["height"])
    TX, TY = proj["tiles"]
    if tiles is None:
        tiles = range(TX * TY)
    image = np.zeros((3, H, W))
    T_final = np.ones((H, W))
    n_contrib = np.zeros((H, W), np.int64)
    count = np.zeros((H, W), np.int64)
    marginal = np.zeros((H, W), bool)
    traces = []
    for t in tiles:
        tr = render_tile(proj, bins, int(t), TX, tile_w, tile_h, W, H, bg)
        image[:, tr["gy"], tr["gx"]] = tr["C"]
        T_final[tr["gy"], tr["gx"]] = tr["T"]
        n_contrib[tr["gy"], tr["gx"]] = tr["last"]
        count[tr["gy"], tr["gx"]] = tr["contrib"].sum(0)
        marginal[tr["gy"], tr["gx"]] = tr["marg"]
        traces.append(tr)
    return dict(image=image, T_final=T_final, n_contrib=n_contrib, count=count,
                marginal=marginal, traces=traces, bg=np.asarray(bg, np.float64))


def replay_entries(fwd, x, y):
    """Replay-trace entries of pixel (x, y): list of (id, alpha, C_in[3])."""
    for tr in fwd["traces"]:
        hit = np.nonzero((tr["gx"] == x) & (tr["gy"] == y))[0]
        if hit.size:
            p = hit[0]
            js = np.nonzero(tr["contrib"][:, p])[0]
            return [(tr["s"] + j, tr["alpha"][j, p], tr["C_in"][j, :, p]) for j in js]
    return []


def _dalpha_cached(tr, G):
    """dL/dalpha and dL/dc for every (list position, pixel) from the trace."""
    L, P = tr["alpha"].shape
    d_alpha = np.zeros((L, P))
    d_col = np.zeros((L, 3, P))
    T = np.ones(P)
    for j in range(L):
        ok = tr["contrib"][j]
        if not ok.any():
            continue
        g = tr["ids"][j]
        a = tr["alpha"][j]
        gk = T[None, :] * G                          # dL/dC_out_k = T_k G
        d_col[j] = np.where(ok[None, :], a[None, :] * gk, 0.0)
        col = tr["colours"][g][:, None]
        d_alpha[j] = np.where(ok, (gk * (col - tr["C_in"][j])).sum(0), 0.0)
        T = np.where(ok, T * (1.0 - a), T)
    return d_alpha, d_col


def _dalpha_recompute(tr, G, proj, bg):
    """Same quantities from T_final and n_contrib, walking back to front."""
    L, P = tr["alpha"].shape
    d_alpha = np.zeros((L, P))
    d_col = np.zeros((L, 3, P))
    T = tr["T"].copy()
    acc = np.tile(bg[:, None], (1, P))
    px = tr["gx"] + 0.5
    py = tr["gy"] + 0.5
    for j in range(L - 1, -1, -1):
        live = j < tr["last"]
        if not live.any():
            continue
        g = tr["ids"][j]
        dx = proj["u"][g] - px
        dy = proj["v"][g] - py
        power = -0.5 * (proj["A"][g] * dx * dx + proj["C"][g] * dy * dy) - proj["B"][g] * dx * dy
        a = np.minimum(ALPHA_MAX, proj["o"][g] * np.exp(power))
        ok = live & ~((power > 0.0) | (a < ALPHA_MIN))
        Tk = np.where(ok, T / (1.0 - a), T)
        col = np.array([proj["r"][g], proj["g"][g], proj["b"][g]])[:, None]
        gk = Tk[None, :] * G
        d_col[j] = np.where(ok[None, :], a[None, :] * gk, 0.0)
        d_alpha[j] = np.where(ok, (gk * (col - acc)).sum(0), 0.0)
        acc = np.where(ok[None, :], a[None, :] * col + (1.0 - a[None, :]) * acc, acc)
        T = Tk
    return d_alpha, d_col


def render_backward(proj, bins, fwd, dL_dimage, variant="cached"):
    """Gradients of <dL_dimage, image> with respect to the 2D parameters.

    Returns (grad2d (9, n) float64 in GRAD_FIELDS order, indexed by canonical
    id, and `tainted` (n,) bool: Gaussians that could contribute at a
    marginal pixel).
    """
    n = proj["n"]
    grad = np.zeros((9, n))
    tainted = np.zeros(n, bool)
    colours = np.stack([proj["r"], proj["g"], proj["b"]], 1)
    dimg = np.asarray(dL_dimage, np.float64)
    for tr in fwd["traces"]:
        if tr["alpha"].shape[0] == 0:
            continue
        tr["colours"] = colours
        G = dimg[:, tr["gy"], tr["gx"]]
        if variant == "cached":
            d_alpha, d_col = _dalpha_cached(tr, G)
        elif variant == "recompute":
            d_alpha, d_col = _dalpha_recompute(tr, G, proj, fwd["bg"])
        else:
            raise ValueError(variant)
        ok = tr["contrib"]
        free = ok & ~tr["clamped"]
        d_o = np.where(free, tr["gauss"] * d_alpha, 0.0)
        d_pow = np.where(free, tr["alpha"] * d_alpha, 0.0)
        ids = tr["ids"]
        Ag = proj["A"][ids][:, None]
        Bg = proj["B"][ids][:, None]
        Cg = proj["C"][ids][:, None]
        dx, dy = tr["dx"], tr["dy"]
        per = np.stack([
            -(Ag * dx + Bg * dy) * d_pow,
            -(Bg * dx + Cg * dy) * d_pow,
            -0.5 * dx * dx * d_pow,
            -dx * dy * d_pow,
            -0.5 * dy * dy * d_pow,
            d_o,
            d_col[:, 0], d_col[:, 1], d_col[:, 2],
        ])                                              # (9, L, P)
        sums = per.sum(2)                               # (9, L)
        for f in range(9):
            np.add.at(grad[f], ids, sums[f])
        if tr["marg"].any():
            # A near-threshold decision at a pixel changes only that pixel's
            # contributions: it can add or drop a splat there and shifts T
            # and C_in for the others.  Every splat of the tile that could
            # contribute at such a pixel under either decision is tainted.
            for p in np.nonzero(tr["marg"])[0]:
                dx = proj["u"][ids] - (tr["gx"][p] + 0.5)
                dy = proj["v"][ids] - (tr["gy"][p] + 0.5)
                power = -0.5 * (proj["A"][ids] * dx * dx + proj["C"][ids] * dy * dy) \
                    - proj["B"][ids] * dx * dy
                a = np.minimum(ALPHA_MAX, proj["o"][ids] * np.exp(power))
                near = (power <= 0.0) & (a >= ALPHA_MIN * (1.0 - MARGIN_ALPHA))
                tainted[ids[near]] = True
    return grad, tainted
