"""Helpers for GPU parity tests: run the HIP path through the C ABI and the
oracle on the same seeded inputs, and compare with the stated tolerances.

Tolerance rule (images 1e-5, gradients 1e-4 relative): element-wise
|x - y| <= tol * (|y| + max|y| over the block), a block being one image
plane or one gradient field, which absorbs near-zero values on a black
background and cancelling gradient sums.  A gradient field that is zero in
exact arithmetic (e.g. the rotation of an isotropic Gaussian) is compared
with an absolute floor of 1e-6 x tol x the largest gradient of the set.
"""

from __future__ import annotations

import sys

import numpy as np
import torch

IMG_TOL = 1e-5
GRAD_TOL = 1e-4


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def assert_block_close(got, want, tol, mask=None, what="", atol=0.0):
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    assert got.shape == want.shape, (what, got.shape, want.shape)
    scale = np.abs(want).max() if want.size else 0.0
    err = np.abs(got - want)
    bound = tol * (np.abs(want) + scale) + atol
    bad = err > bound
    if mask is not None:
        bad &= mask
    if bad.any():
        idx = np.argwhere(bad)[:5]
        raise AssertionError(f"{what}: {bad.sum()} of {bad.size} beyond tol {tol}; first at "
                             f"{idx.tolist()} got {got[tuple(idx[0])]} want {want[tuple(idx[0])]} "
                             f"scale {scale}")


# float32 unit roundoff
U32 = 2.0 ** -24


def assert_cin_close(got, want, what=""):
    """Replay-trace C_in of one pixel's entries (K x 3, front to back) against
    the oracle.  The kernel forms C_in_k by the over recursion
    C_in_k = alpha_{k+1} c_{k+1} + (1 - alpha_{k+1}) C_in_{k+1} in float32,
    starting from the background behind the last entry, so entry k carries
    the rounding of the K - 1 - k steps behind it: each step rounds three
    operations (<= 3u of the running value) and brings the error of its
    alpha, o e^power evaluated in float32 with |power| <= ln 255 (<= ~8u);
    the (1 - alpha) factor never amplifies earlier error.  Bound per entry:
    16 u (K - k) (1 + max|C_in|), u = 2^-24, i.e. ~1e-6 for the last entry
    and ~1e-4 for a front entry with a hundred entries behind it."""
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    k = np.arange(len(want))
    bound = 16 * U32 * (len(want) - k)[:, None] * (1.0 + np.abs(want).max())
    err = np.abs(got - want)
    assert (err <= bound).all(), (what, float((err / bound).max()), len(want))
    return float((err / bound).max()) if len(want) else 0.0


def max_rel(got, want, floor_frac=1e-3):
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    big = np.abs(want) > floor_frac * np.abs(want).max()
    if not big.any():
        return 0.0
    return float((np.abs(got - want)[big] / np.abs(want)[big]).max())


def run_gpu(P, cam, sh_degree, cached=True, bg=(0.0, 0.0, 0.0), dl_dimage=None,
            capacity=None, tile=(16, 16), trace_words=None):
    """One view through the HIP path; returns numpy copies of every output."""
    from paper_2601_17354_amd.raster import Rasterizer
    dev = torch.device("cuda")
    n = P.shape[1]
    params = torch.as_tensor(np.ascontiguousarray(P, np.float32), device=dev)
    kw = {} if trace_words is None else {"trace_words": trace_words}
    R = Rasterizer(n, sh_degree, cam["width"], cam["height"], tile=tile, cached=cached,
                   capacity=capacity, **kw)
    R.forward_checked(params, cam, bg)
    torch.cuda.synchronize()
    out = dict(
        proj=R.proj.cpu().numpy()[:n].T, radius=R.radius.cpu().numpy()[:n],
        rect=R.rect.cpu().numpy()[:, :n].view(np.uint32), touched=R.touched.cpu().numpy()[:n],
        num_pairs=int(R.num_pairs.item()), image=R.image.cpu().numpy(),
        t_final=R.t_final.cpu().numpy(), n_contrib=R.n_contrib.cpu().numpy(),
        ranges=R.ranges.cpu().numpy(), flags=R.read_flags(), rast=R,
    )
    npairs = min(out["num_pairs"], R.capacity)
    out["keys"] = R.keys[:npairs].cpu().numpy().view(np.uint64)
    out["values"] = R.values[:npairs].cpu().numpy()
    if cached:
        out["count"] = R.trace["count"].cpu().numpy().reshape(cam["height"], cam["width"])
    if dl_dimage is not None:
        grads = torch.zeros_like(params)
        dl = torch.as_tensor(np.ascontiguousarray(dl_dimage, np.float32), device=dev)
        R.backward(params, cam, dl, grads, bg)
        torch.cuda.synchronize()
        out["grad2d"] = R.grad2d.cpu().numpy()[:n, :9].T
        out["grads"] = grads.cpu().numpy()
    return out


def trace_entries(out, cam, x, y, tile=(16, 16)):
    """Replay-trace entries (id, alpha, C_in) of pixel (x, y), decoded from the
    per-wave groups of the GPU trace (layout documented at pgs_replay); alpha
    is None for the 3-word layout, which does not store it."""
    R = out["rast"]
    tw, th = tile
    nt = tw * th
    TX = (cam["width"] + tw - 1) // tw
    t = (y // th) * TX + (x // tw)
    p = (y % th) * tw + (x % tw)
    w, lane = p // 64, p % 64
    start, end = (int(v) for v in out["ranges"][:, t])
    steps = int(R.trace["steps"][t, w].item())
    masks = R.trace["mask"][w, start:start + steps].cpu().numpy().view(np.uint64)
    ebase = int(R.trace["base"][t, w].item()) & 0xFFFFFFFF
    cursor, ents = 0, []
    for j, m in enumerate(masks):
        m = int(m)
        if (m >> lane) & 1:
            ents.append((start + j, ebase + cursor + bin(m & ((1 << lane) - 1)).count("1")))
        cursor += bin(m).count("1")
    assert len(ents) == int(out["count"][y, x])
    e = torch.as_tensor([q for _, q in ents], dtype=torch.int64, device=R.device)
    words = R.trace["entry"].shape[1]
    rec = R.trace["entry"][e].cpu().numpy().reshape(-1, words)
    alpha = rec[:, 3] if words == 4 else None
    return np.asarray([i for i, _ in ents], np.int64), alpha, rec[:, :3]
