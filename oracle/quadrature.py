"""Quadrature grid for the RPA zeroth density-response moment (oracle side).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper integrates G_main (Sec. 2.2, eq. Gmain) over the whole real axis
and the offset term over the positive half axis, each with an exponentially
convergent rule.  The rule is read here as an n-point Gauss-Legendre rule
on (-1, 1) mapped onto (0, inf) by

    z(x) = s (1 + x) / (1 - x),      dz/dx = 2 s / (1 - x)^2,

with s > 0 a scale (default: the median of the energy differences D).  The
G_main integrand is even in z, so its integral over the real line is twice
the half-line integral.  Nodes and weights come from numpy's ``leggauss``.
"""
from __future__ import annotations

import numpy as np


def default_scale(D: np.ndarray) -> float:
    """Median of the particle-hole energy differences (reading of the paper's
    unspecified grid scale)."""
    return float(np.median(D))


def mapped_gauss_legendre(nquad: int, scale: float):
    """Return (z[nquad], w[nquad]) such that sum_j w_j g(z_j) ~ int_0^inf g(z) dz."""
    if nquad < 1:
        raise ValueError("nquad must be >= 1")
    if not scale > 0.0:
        raise ValueError("scale must be positive")
    x, wx = np.polynomial.legendre.leggauss(nquad)
    z = scale * (1.0 + x) / (1.0 - x)
    w = wx * 2.0 * scale / (1.0 - x) ** 2
    return z, w
