"""Mesh topology and affine geometry (oracle side; test infrastructure).

Conventions that are part of the documented data layout:

* the reference map of cell K with vertices (v0, v1, v2), in the order given
  by the cell array, is x = v0 + (v1 - v0) xi + (v2 - v0) eta;
* facets are the distinct vertex pairs (lo, hi), lo < hi, numbered in
  lexicographic order of (lo, hi); the trace parameter t runs from lo to hi.

The notation follows Section "Notation": for an interior facet the cell with
the smaller id is K+ and the other K-; h_F is the facet length.
"""
from __future__ import annotations

import numpy as np

# local facet f of a triangle is the edge opposite local vertex f
LOCAL_EDGES = ((1, 2), (0, 2), (0, 1))


class Mesh:
    def __init__(self, coords, cells):
        coords = np.asarray(coords, dtype=np.float64)
        cells = np.asarray(cells, dtype=np.int64)
        if coords.ndim != 2 or coords.shape[1] != 2 or cells.ndim != 2 or cells.shape[1] != 3:
            raise ValueError("2D triangle mesh expected")
        self.coords = coords
        self.cells = cells
        self.ncells = cells.shape[0]
        nc = self.ncells

        # --- facets ---------------------------------------------------------
        pairs = np.empty((nc, 3, 2), dtype=np.int64)
        for f, (a, b) in enumerate(LOCAL_EDGES):
            pairs[:, f, 0] = np.minimum(cells[:, a], cells[:, b])
            pairs[:, f, 1] = np.maximum(cells[:, a], cells[:, b])
        flat = pairs.reshape(-1, 2)
        facets, inverse = np.unique(flat, axis=0, return_inverse=True)
        self.facets = facets  # (nf, 2) = (lo, hi)
        self.nfacets = facets.shape[0]
        self.cell_facets = inverse.reshape(nc, 3)

        # facet -> (K+, f+, K-, f-), K+ the smaller cell id
        fc = -np.ones((self.nfacets, 4), dtype=np.int64)
        for K in range(nc):
            for f in range(3):
                F = self.cell_facets[K, f]
                if fc[F, 0] < 0:
                    fc[F, 0], fc[F, 1] = K, f
                elif fc[F, 2] < 0:
                    fc[F, 2], fc[F, 3] = K, f
                else:
                    raise ValueError("non-manifold facet")
        self.facet_cells = fc
        self.interior = fc[:, 2] >= 0

        # neighbour across each local facet
        self.nb_cell = -np.ones((nc, 3), dtype=np.int64)
        self.nb_facet = -np.ones((nc, 3), dtype=np.int64)
        for F in np.nonzero(self.interior)[0]:
            Kp, fp, Km, fm = fc[F]
            self.nb_cell[Kp, fp], self.nb_facet[Kp, fp] = Km, fm
            self.nb_cell[Km, fm], self.nb_facet[Km, fm] = Kp, fp

        # --- geometry -------------------------------------------------------
        v = coords[cells]  # (nc, 3, 2)
        J = np.stack([v[:, 1] - v[:, 0], v[:, 2] - v[:, 0]], axis=2)  # columns
        self.v0 = v[:, 0]
        self.J = J
        self.detJ = J[:, 0, 0] * J[:, 1, 1] - J[:, 0, 1] * J[:, 1, 0]
        if np.any(np.abs(self.detJ) < 1e-300):
            raise ValueError("degenerate cell")
        self.absdet = np.abs(self.detJ)
        self.invJ = np.linalg.inv(J)

        self.normal = np.empty((nc, 3, 2))
        self.hF_cell = np.empty((nc, 3))
        for f, (a, b) in enumerate(LOCAL_EDGES):
            e = v[:, b] - v[:, a]
            ln = np.linalg.norm(e, axis=1)
            n = np.stack([e[:, 1], -e[:, 0]], axis=1) / ln[:, None]
            out = np.einsum("kd,kd->k", n, v[:, a] - v[:, f])
            n[out < 0] *= -1.0
            self.normal[:, f] = n
            self.hF_cell[:, f] = ln
        self.hF = np.linalg.norm(coords[facets[:, 1]] - coords[facets[:, 0]], axis=1)

    def to_reference(self, K, x):
        """Reference coordinates of physical points x (..., 2) in cells K (broadcast)."""
        d = x - self.v0[K]
        return np.einsum("...ad,...d->...a", self.invJ[K], d)

    def facet_points(self, t):
        """Physical points x(t) on every facet, t from lo to hi; shape (nf, nt, 2)."""
        xlo = self.coords[self.facets[:, 0]]
        xhi = self.coords[self.facets[:, 1]]
        return xlo[:, None, :] + np.asarray(t)[None, :, None] * (xhi - xlo)[:, None, :]
