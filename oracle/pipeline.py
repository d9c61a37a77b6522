"""One view through the whole oracle: project -> bin/sort -> composite, and
the gradient back to the canonical parameters (render backward, index map,
projection backward)."""

from __future__ import annotations

import numpy as np

from .binning import bin_and_sort
from .projection import project, project_vjp
from .render import render_backward, render_forward


def forward(params, cam, tile_w=16, tile_h=16, bg=(0.0, 0.0, 0.0), tiles=None):
    proj = project(params, cam, tile_w, tile_h)
    bins = bin_and_sort(proj)
    fwd = render_forward(proj, bins, cam, tile_w, tile_h, bg, tiles)
    return proj, bins, fwd


def backward(params, cam, proj, bins, fwd, dL_dimage, variant="cached"):
    """Returns (canonical grads (F, n), grad2d (9, n), tainted (n,))."""
    g2d, tainted = render_backward(proj, bins, fwd, dL_dimage, variant)
    grads = project_vjp(params, cam, g2d, proj["visible"])
    return grads, g2d, tainted


def image(params, cam, tile_w=16, tile_h=16, bg=(0.0, 0.0, 0.0)):
    return forward(params, cam, tile_w, tile_h, bg)[2]["image"]


def decisions(params, cam, tile_w=16, tile_h=16, bg=(0.0, 0.0, 0.0)):
    """Every discrete outcome of the forward pass, for freezing branches in
    finite-difference checks: visibility, radius, rectangles, sorted order and
    per-pixel contributor sets with their clamp flags."""
    proj, bins, fwd = forward(params, cam, tile_w, tile_h, bg)
    parts = [proj["visible"], proj["radius"], proj["rect"], bins["values"], bins["ranges"],
             proj["colour_clamped"], proj["clamp_xy"]]
    for tr in fwd["traces"]:
        parts.append(tr["contrib"])
        parts.append(tr["clamped"] & tr["contrib"])
    return [np.asarray(p) for p in parts]


def same_decisions(a, b) -> bool:
    return len(a) == len(b) and all(x.shape == y.shape and np.array_equal(x, y) for x, y in zip(a, b))
