"""Quadrature rules for the oracle (test infrastructure; see package header).

The paper does not state its quadrature.  The reading used here: every
polynomial integrand is integrated exactly, and the facet rule, which also
integrates the non-polynomial upwind weight |Q*.n|, is the Gauss-Legendre rule
with ceil((3k+4)/2) points on each facet.  The cell rule is the collapsed
(Duffy) Gauss rule with ceil((3k+3)/2) points per direction, exact for total
degree 3k+2 (the advection volume term w.(Q*.grad)Q has degree
(k+1)+(k+1)+k).
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial import legendre
from scipy import special


def facet_points(k: int) -> int:
    """Number of Gauss-Legendre points per facet for pressure degree k."""
    return math.ceil((3 * k + 4) / 2)


def cell_points_1d(k: int) -> int:
    """Collapsed-rule points per direction for pressure degree k."""
    return math.ceil((3 * k + 3) / 2)


def gauss_legendre_01(n: int):
    """n-point Gauss-Legendre rule on [0, 1]: (points, weights), weights sum to 1."""
    x, w = legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def triangle_rule(n: int):
    """Collapsed Gauss rule on the reference triangle {xi, eta >= 0, xi + eta <= 1}.

    a ~ Gauss-Legendre(n), b ~ Gauss-Jacobi(n, alpha=1, beta=0) on [-1, 1];
    xi = (1+a)(1-b)/4, eta = (1+b)/2, weight w_a w_b / 8.  Exact for total
    degree 2n-1.  Returns (points[nq, 2], weights[nq]); weights sum to 1/2.
    """
    a, wa = legendre.leggauss(n)
    b, wb = special.roots_jacobi(n, 1.0, 0.0)
    A, B = np.meshgrid(a, b, indexing="ij")
    WA, WB = np.meshgrid(wa, wb, indexing="ij")
    xi = (1.0 + A) * (1.0 - B) / 4.0
    eta = (1.0 + B) / 2.0
    pts = np.stack([xi.ravel(), eta.ravel()], axis=1)
    return pts, (WA * WB).ravel() / 8.0
