"""Mesh topology and affine geometry (oracle side; test infrastructure).

Conventions that are part of the documented data layout:

* the reference map of cell K with vertices (v0, v1, v2), in the order given
  by the cell array, is x = v0 + (v1 - v0) xi + (v2 - v0) eta;
* facets are the distinct vertex pairs (lo, hi), lo < hi, numbered in
  lexicographic order of (lo, hi); the trace parameter t runs from lo to hi.
* periodic meshes: an optional vertex_rep array names, for every vertex,
  the vertex it is identified with (itself if none).  Topology (facets,
  neighbours, the facet parameter direction) uses the classes of identified
  vertices, numbered by the rank of their representative; geometry uses
  every cell's own vertex coordinates.  Without vertex_rep the classes are
  the vertices themselves.

The notation follows Section "Notation": for an interior facet the cell with
the smaller id is K+ and the other K-; h_F is the facet length.
"""
from __future__ import annotations

import numpy as np

# local facet f of a triangle is the edge opposite local vertex f
LOCAL_EDGES = ((1, 2), (0, 2), (0, 1))


class Mesh:
    def __init__(self, coords, cells, vertex_rep=None):
        coords = np.asarray(coords, dtype=np.float64)
        cells = np.asarray(cells, dtype=np.int64)
        if coords.ndim != 2 or coords.shape[1] != 2 or cells.ndim != 2 or cells.shape[1] != 3:
            raise ValueError("2D triangle mesh expected")
        self.coords = coords
        self.cells = cells
        self.ncells = cells.shape[0]
        nc = self.ncells
        nv = coords.shape[0]
        if vertex_rep is None:
            vclass = np.arange(nv, dtype=np.int64)
        else:
            rep = np.asarray(vertex_rep, dtype=np.int64)
            if rep.shape != (nv,) or rep.min() < 0 or rep.max() >= nv:
                raise ValueError("vertex_rep must map every vertex to a vertex")
            _, vclass = np.unique(rep, return_inverse=True)
        self.periodic = vertex_rep is not None
        self.vclass = vclass
        self.tcells = tc = vclass[cells]  # cells in topological vertex ids

        # --- facets ---------------------------------------------------------
        pairs = np.empty((nc, 3, 2), dtype=np.int64)
        for f, (a, b) in enumerate(LOCAL_EDGES):
            if np.any(tc[:, a] == tc[:, b]):
                raise ValueError("a cell edge joins identified vertices")
            pairs[:, f, 0] = np.minimum(tc[:, a], tc[:, b])
            pairs[:, f, 1] = np.maximum(tc[:, a], tc[:, b])
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
        # facet length as seen from K+; both sides of an identified facet must agree
        self.hF = self.hF_cell[fc[:, 0], fc[:, 1]]
        Ii = np.nonzero(self.interior)[0]
        if np.any(np.abs(self.hF_cell[fc[Ii, 2], fc[Ii, 3]] - self.hF[Ii]) > 1e-12 * self.hF[Ii]):
            raise ValueError("the two sides of a facet differ in length")

    def to_reference(self, K, x):
        """Reference coordinates of physical points x (..., 2) in cells K (broadcast)."""
        d = x - self.v0[K]
        return np.einsum("...ad,...d->...a", self.invJ[K], d)

    def cell_facet_points(self, t):
        """Physical points x(t) on every local facet of every cell, t running
        from the facet's lo to its hi vertex; shape (nc, 3, nt, 2)."""
        t = np.asarray(t, dtype=np.float64)
        out = np.empty((self.ncells, 3, t.size, 2))
        for f, (a, b) in enumerate(LOCAL_EDGES):
            va, vb = self.coords[self.cells[:, a]], self.coords[self.cells[:, b]]
            fwd = (self.tcells[:, a] < self.tcells[:, b])[:, None]
            xlo, xhi = np.where(fwd, va, vb), np.where(fwd, vb, va)
            out[:, f] = xlo[:, None, :] + t[None, :, None] * (xhi - xlo)[:, None, :]
        return out

    def facet_points(self, t):
        """Physical points x(t) on every facet as seen from K+, t from lo to hi;
        shape (nf, nt, 2)."""
        fc = self.facet_cells
        return self.cell_facet_points(t)[fc[:, 0], fc[:, 1]]
