"""Adam on the canonical parameter layout (oracle).

The index-mapping subsection of PocketGS keeps optimizer moments aligned with
the canonical (never reordered) parameter buffer.  Adam itself is Kingma & Ba
(2015) with bias correction:

    m <- b1 m + (1 - b1) g
    v <- b2 v + (1 - b2) g^2
    p <- p - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)

with a learning rate per parameter row.  Defaults b1 = 0.9, b2 = 0.999,
eps = 1e-15 (the paper states none of these; 3D Gaussian Splatting values).
"""

from __future__ import annotations

import numpy as np

BETA1 = 0.9
BETA2 = 0.999
EPS = 1e-15


def adam_step(p, g, m, v, lr_rows, step, b1=BETA1, b2=BETA2, eps=EPS):
    """One step; p, g, m, v are (F, n); lr_rows is (F,); step counts from 1.
    Returns new (p, m, v) as float64 arrays."""
    p = np.asarray(p, np.float64)
    g = np.asarray(g, np.float64)
    m = b1 * np.asarray(m, np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** step)
    vhat = v / (1.0 - b2 ** step)
    lr = np.asarray(lr_rows, np.float64)[:, None]
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v

