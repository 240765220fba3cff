"""Documented orthonormal bases (oracle side; test infrastructure).

The paper's spaces (Section "Discontinuous Galerkin spaces", and the trace
space of Section "Hybridisation"): velocity [P_{k+1}(K)]^2, pressure P_k(K),
trace P_k(F).  Any basis spans them; the coefficient layout exchanged with the
GPU library is fixed to these bases so both sides can be compared entry by
entry:

* cell: the orthonormal Dubiner (Koornwinder) basis on the reference triangle
  {(xi, eta): xi, eta >= 0, xi + eta <= 1}.  With r = 2 xi - 1, s = 2 eta - 1,
  a = 2 (1 + r) / (1 - s) - 1 and b = s,
      phi_ij = sqrt(2 (2i+1) (i+j+1)) P_i(a) ((1-b)/2)^i P_j^{(2i+1,0)}(b),
  i + j <= m, ordered by total degree d = i + j, then by i ascending.
* facet: mu_i(t) = sqrt(2i+1) P_i(2t - 1), t in [0, 1] running from the facet's
  lower global vertex id to the higher one.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre
from scipy import special


def dubiner_indices(m: int):
    return [(i, d - i) for d in range(m + 1) for i in range(d + 1)]


def dim_p(m: int) -> int:
    return (m + 1) * (m + 2) // 2


def _jacobi(n, alpha, beta, x):
    if n < 0:
        return np.zeros_like(x)
    return special.eval_jacobi(n, alpha, beta, x)


def _djacobi(n, alpha, beta, x):
    """Derivative of P_n^{(alpha,beta)} via d/dx P_n = (n+alpha+beta+1)/2 P_{n-1}^{(alpha+1,beta+1)}."""
    if n == 0:
        return np.zeros_like(x)
    return 0.5 * (n + alpha + beta + 1) * special.eval_jacobi(n - 1, alpha + 1, beta + 1, x)


def dubiner(m: int, xi, eta, derivatives: bool = True):
    """Values (and xi-, eta-derivatives) of the degree-m Dubiner basis.

    Returns arrays of shape (npts, dim_p(m)).
    """
    xi = np.asarray(xi, dtype=np.float64).ravel()
    eta = np.asarray(eta, dtype=np.float64).ravel()
    r = 2.0 * xi - 1.0
    s = 2.0 * eta - 1.0
    b = s
    with np.errstate(divide="ignore", invalid="ignore"):
        a = np.where(np.abs(1.0 - s) > 1e-300, 2.0 * (1.0 + r) / (1.0 - s) - 1.0, -1.0)
    h = 0.5 * (1.0 - b)  # (1-b)/2
    idx = dubiner_indices(m)
    V = np.empty((xi.size, len(idx)))
    Dx = np.empty_like(V)
    Dy = np.empty_like(V)
    for col, (i, j) in enumerate(idx):
        norm = np.sqrt(2.0 * (2 * i + 1) * (i + j + 1))
        Pa = _jacobi(i, 0.0, 0.0, a)
        Pb = _jacobi(j, 2 * i + 1.0, 0.0, b)
        V[:, col] = norm * Pa * h**i * Pb
        if derivatives:
            dPa = _djacobi(i, 0.0, 0.0, a)
            dPb = _djacobi(j, 2 * i + 1.0, 0.0, b)
            him1 = h ** (i - 1) if i >= 1 else np.zeros_like(h)
            # d/dxi: da/dxi = 4/(1-s) = 2/h
            Dx[:, col] = norm * dPa * 2.0 * him1 * Pb if i >= 1 else 0.0
            # d/deta: da/deta = (1+a)/h, db/deta = 2
            dg = (-0.5 * i * him1 * Pb if i >= 1 else 0.0) + h**i * dPb
            Dy[:, col] = norm * ((dPa * (1.0 + a) * him1 * Pb if i >= 1 else 0.0) + 2.0 * Pa * dg)
    if derivatives:
        return V, Dx, Dy
    return V


def legendre01(k: int, t):
    """Orthonormal Legendre basis mu_0..mu_k on [0, 1] at t; shape (npts, k+1)."""
    t = np.asarray(t, dtype=np.float64).ravel()
    out = np.empty((t.size, k + 1))
    for i in range(k + 1):
        c = np.zeros(i + 1)
        c[i] = 1.0
        out[:, i] = np.sqrt(2 * i + 1) * legendre.legval(2.0 * t - 1.0, c)
    return out
