"""Tetrahedral meshes, quadrature and bases for the three-dimensional oracle
(test infrastructure: only tests and the benchmark's CPU leg use it).

The paper states its method for d = 2 and 3 alike (Sections "Discontinuous
Galerkin spaces" and "Hybridisation": velocity [P_{k+1}(K)]^d, pressure
P_k(K), trace P_k(F)) and computes in 2D only; the three-dimensional
workload is the unit cube cut into n^3 cubes of six tetrahedra each.

* Mesh: any conforming mesh of positively oriented tetrahedra (the workload
  is the Kuhn split of the cube, whose neighbouring cubes meet in matching
  triangles).
* Local facet f of a cell is the triangle opposite its local vertex f.
  Facets are the distinct sorted vertex triples (lo < mid < hi), numbered in
  lexicographic order; the facet's own coordinates (s, t) place
  x = v_lo + s (v_mid - v_lo) + t (v_hi - v_lo).
* Quadrature: the collapsed (Duffy) Gauss rule on the reference tetrahedron
  {xi, eta, zeta >= 0, xi + eta + zeta <= 1}, Gauss-Jacobi in each collapsed
  direction, exact for total degree 2n - 1; facets use the triangle rule of
  the two-dimensional oracle (exact for 2n - 1).
* Bases: any basis spans the spaces.  Here the monomials x'^a y'^b z'^c of
  total degree <= m in the centred coordinates x' = (d + 1)(x - centroid),
  ordered by degree then lexicographically, orthonormalised on
  the reference cell by the Cholesky factor of their exact mass matrix
  (Gram-Schmidt in the monomial order, taken twice); likewise on the reference triangle
  for the facet unknowns, with the inner product of the triangle's area
  measure scaled to total 1, so that on a physical facet of area |F|
  int_F mu_i mu_j = |F| delta_ij.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
from scipy import special

from .quadrature import triangle_rule

# -------------------------------------------------------------- quadrature


def tet_rule(n: int):
    """Collapsed Gauss rule on the reference tetrahedron, exact for total
    degree 2n - 1: points (nq, 3), weights (nq,) summing to 1/6."""
    a, wa = special.roots_jacobi(n, 0.0, 0.0)
    b, wb = special.roots_jacobi(n, 1.0, 0.0)
    c, wc = special.roots_jacobi(n, 2.0, 0.0)
    A, B, C = np.meshgrid(a, b, c, indexing="ij")
    WA, WB, WC = np.meshgrid(wa, wb, wc, indexing="ij")
    # (a, b, c) in [-1, 1]^3 -> the tetrahedron
    zeta = (1.0 + C) / 2.0
    eta = (1.0 + B) / 2.0 * (1.0 - zeta)
    xi = (1.0 + A) / 2.0 * (1.0 - eta - zeta)
    pts = np.stack([xi.ravel(), eta.ravel(), zeta.ravel()], axis=1)
    return pts, (WA * WB * WC).ravel() / 64.0


def cell_points_1d(k: int) -> int:
    """Collapsed-rule points per direction for pressure degree k (exact for
    3k + 2: the advection volume term)."""
    return math.ceil((3 * k + 3) / 2)


def facet_points_1d(k: int) -> int:
    """Triangle-rule points per direction on a facet (exact for 3k + 3, which
    also carries the upwind weight |Q*.n|, evaluated by the same rule on both
    sides)."""
    return math.ceil((3 * k + 4) / 2)


# ------------------------------------------------------------------- bases


def monomial_exponents(m: int, d: int):
    """Exponent tuples of total degree <= m in d variables, by degree, then
    lexicographically (largest first power first)."""
    out = []
    for deg in range(m + 1):
        out += sorted((e for e in itertools.product(range(deg + 1), repeat=d) if sum(e) == deg), reverse=True)
    return out


def dim_p3(m: int) -> int:
    return (m + 1) * (m + 2) * (m + 3) // 6


def dim_p2(m: int) -> int:
    return (m + 1) * (m + 2) // 2


def _monomials(exps, pts, derivatives=False):
    pts = np.atleast_2d(pts)
    V = np.stack([np.prod(pts ** np.array(e)[None, :], axis=1) for e in exps], axis=1)
    if not derivatives:
        return V
    d = pts.shape[1]
    D = []
    for ax in range(d):
        cols = []
        for e in exps:
            e = np.array(e)
            if e[ax] == 0:
                cols.append(np.zeros(pts.shape[0]))
            else:
                e2 = e.copy()
                e2[ax] -= 1
                cols.append(e[ax] * np.prod(pts ** e2[None, :], axis=1))
        D.append(np.stack(cols, axis=1))
    return V, D


class OrthoBasis:
    """Monomials of degree <= m on the reference simplex of dimension d,
    orthonormalised by the Cholesky factor of their exact mass matrix (the
    reference measure scaled by `scale`)."""

    def __init__(self, m: int, d: int, scale: float = 1.0):
        self.m, self.d = m, d
        self.exps = monomial_exponents(m, d)
        # monomials of (d + 1)(x - centroid): far better conditioned than x^a
        self.shift, self.stretch = 1.0 / (d + 1), float(d + 1)
        if d == 3:
            pts, w = tet_rule(m + 2)
        else:
            pts, w = triangle_rule(m + 2)
        w = w * scale
        V = _monomials(self.exps, self._local(pts))
        G = V.T @ (w[:, None] * V)
        # phi = monomials @ C with phi^T W phi = I; the monomial Gram matrix is
        # ill-conditioned, so the factorisation is repeated once on the result
        # (the second pass is a near-identity triangular correction)
        C = np.linalg.inv(np.linalg.cholesky(G)).T
        C2 = np.linalg.inv(np.linalg.cholesky(C.T @ G @ C)).T
        self.C = C @ C2
        self.dim = len(self.exps)

    def _local(self, pts):
        return (np.atleast_2d(pts) - self.shift) * self.stretch

    def eval(self, pts, derivatives=False):
        if not derivatives:
            return _monomials(self.exps, self._local(pts)) @ self.C
        V, D = _monomials(self.exps, self._local(pts), True)
        return V @ self.C, [self.stretch * (Di @ self.C) for Di in D]


# -------------------------------------------------------------------- mesh


class TetMesh:
    """Topology and affine geometry of a tetrahedral mesh (local facet f
    opposite local vertex f)."""

    LOCAL_FACETS = np.array([[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]])

    def __init__(self, coords, cells):
        coords = np.asarray(coords, dtype=np.float64)
        cells = np.asarray(cells, dtype=np.int64)
        self.coords, self.cells = coords, cells
        self.ncells = nc = cells.shape[0]
        tri = np.sort(cells[:, self.LOCAL_FACETS], axis=2).reshape(-1, 3)
        facets, inverse = np.unique(tri, axis=0, return_inverse=True)
        self.facets = facets
        self.nfacets = facets.shape[0]
        self.cell_facets = inverse.reshape(nc, 4)
        fc = -np.ones((self.nfacets, 4), dtype=np.int64)
        order = np.argsort(inverse, kind="stable")
        cf = np.repeat(np.arange(nc), 4)[order]
        lf = np.tile(np.arange(4), nc)[order]
        Fs = inverse[order]
        first = np.ones(Fs.size, dtype=bool)
        first[1:] = Fs[1:] != Fs[:-1]
        fc[Fs[first], 0], fc[Fs[first], 1] = cf[first], lf[first]
        second = ~first
        if np.any(second[1:] & second[:-1]):
            raise ValueError("non-manifold facet")
        fc[Fs[second], 2], fc[Fs[second], 3] = cf[second], lf[second]
        self.facet_cells = fc
        self.interior = fc[:, 2] >= 0
        self.nb_cell = -np.ones((nc, 4), dtype=np.int64)
        self.nb_facet = -np.ones((nc, 4), dtype=np.int64)
        I = np.nonzero(self.interior)[0]
        self.nb_cell[fc[I, 0], fc[I, 1]] = fc[I, 2]
        self.nb_facet[fc[I, 0], fc[I, 1]] = fc[I, 3]
        self.nb_cell[fc[I, 2], fc[I, 3]] = fc[I, 0]
        self.nb_facet[fc[I, 2], fc[I, 3]] = fc[I, 1]
        v = coords[cells]
        self.v0 = v[:, 0]
        self.J = np.stack([v[:, 1] - v[:, 0], v[:, 2] - v[:, 0], v[:, 3] - v[:, 0]], axis=2)  # columns
        self.detJ = np.linalg.det(self.J)
        if np.any(self.detJ <= 0):
            raise ValueError("cells must be positively oriented")
        self.absdet = np.abs(self.detJ)
        self.invJ = np.linalg.inv(self.J)
        # outward unit normals and areas per (cell, local facet)
        self.normal = np.empty((nc, 4, 3))
        self.area_cf = np.empty((nc, 4))
        for f in range(4):
            a, b, c = (v[:, i] for i in self.LOCAL_FACETS[f])
            nrm = np.cross(b - a, c - a)
            opp = v[:, f]
            sgn = np.sign(np.einsum("kd,kd->k", nrm, a - opp))
            nrm *= sgn[:, None]
            ln = np.linalg.norm(nrm, axis=1)
            self.normal[:, f] = nrm / ln[:, None]
            self.area_cf[:, f] = 0.5 * ln
        self.area = self.area_cf[fc[:, 0], fc[:, 1]]
        self.hF = self.area  # h_F is the facet's measure (Section "Notation")
        # facet coordinates: x = v_lo + s (v_mid - v_lo) + t (v_hi - v_lo)
        fv = coords[facets]
        self.facet_v0 = fv[:, 0]
        self.facet_E = np.stack([fv[:, 1] - fv[:, 0], fv[:, 2] - fv[:, 0]], axis=2)  # (nF, 3, 2)

    def to_reference(self, K, x):
        """Reference coordinates in cell K of physical points x (..., 3)."""
        return np.einsum("...ab,...b->...a", self.invJ[K], x - self.v0[K])

    def to_facet(self, F, x):
        """Facet coordinates (s, t) on facet F of physical points x (..., 3)."""
        E = self.facet_E[F]
        r = x - self.facet_v0[F]
        G = np.einsum("...da,...db->...ab", E, E)
        rhs = np.einsum("...da,...d->...a", E, r)
        return np.linalg.solve(G, rhs[..., None])[..., 0]
