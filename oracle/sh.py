"""Real spherical-harmonic basis (oracle).

Colour in 3D Gaussian Splatting is a real-SH expansion evaluated at the unit
view direction (inherited by PocketGS; its canonical buffer stores colour "c"
as per-Gaussian parameters, overview figure and index-mapping subsection).

Definition used here (textbook real SH with the Condon-Shortley phase kept in
the associated Legendre function P_l^m):

    Y_l0  = K_l0 P_l(z)
    Y_lm  = sqrt(2) K_lm P_l^m(z) cos(m phi)         m > 0
    Y_l-m = sqrt(2) K_lm P_l^m(z) sin(m phi)         m > 0
    K_lm  = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!)

and P_l^m(z) = (-1)^m (1 - z^2)^(m/2) d^m/dz^m P_l(z).  In Cartesian form
(1 - z^2)^(m/2) cos(m phi) = Re (x + i y)^m and ... sin(m phi) = Im (x + i y)^m,
so the basis is a polynomial in (x, y, z) with no pole singularity; that is
the form evaluated below (torch float64, differentiable).
Coefficient index k = l*l + l + m.
"""

from __future__ import annotations

import math

import numpy as np
import torch


def _legendre_deriv_coeffs(l: int, m: int) -> np.ndarray:
    """Power-series coefficients (ascending) of d^m/dz^m P_l(z)."""
    leg = np.polynomial.legendre.Legendre.basis(l).deriv(m)
    return np.polynomial.legendre.leg2poly(leg.coef)


def _norm(l: int, m: int) -> float:
    return math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - m) / math.factorial(l + m))


def sh_basis(d: torch.Tensor, degree: int) -> torch.Tensor:
    """Y_k(d) for unit directions d (n,3) -> (n, (degree+1)^2), float64."""
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    # (x + i y)^m real and imaginary parts by recurrence
    re = [torch.ones_like(x)]
    im = [torch.zeros_like(x)]
    for m in range(1, degree + 1):
        r_prev, i_prev = re[m - 1], im[m - 1]
        re.append(r_prev * x - i_prev * y)
        im.append(r_prev * y + i_prev * x)
    out = []
    for l in range(degree + 1):
        for m in range(-l, l + 1):
            am = abs(m)
            c = _legendre_deriv_coeffs(l, am)
            poly = torch.zeros_like(z)
            for p in range(len(c) - 1, -1, -1):       # Horner in z
                poly = poly * z + float(c[p])
            poly = poly * ((-1.0) ** am)
            if m == 0:
                out.append(_norm(l, 0) * poly)
            elif m > 0:
                out.append(math.sqrt(2.0) * _norm(l, am) * poly * re[am])
            else:
                out.append(math.sqrt(2.0) * _norm(l, am) * poly * im[am])
    return torch.stack(out, 1)
