"""Passive DG tracer (Appendix "DG tracer advection"; oracle side, test
infrastructure).

* P_CG: the L2 projection of a velocity Q in DG_{k+1} onto the continuous
  space CG_{k+1} = DG_{k+1} n C^0 (component by component), built here from
  a nodal Lagrange basis at the equispaced points of the reference triangle,
  glued along the topological vertices and facets of the mesh (so it is
  continuous across periodic identifications too), assembled with the cell
  rule and solved directly.
* a(chi, q, U) = (q, div(chi U))_Omega - sum_{interior F} <q^up [[chi U.n]]>_F
  with the tracer q and the test chi in DG_k (the pressure space, the degree
  k' = k of the paper's runs), U = P_CG(Q) and q^up the value of q on the
  upwind side (U.n+ >= 0: K+).  Facets on walls carry no term, as printed.
* time stepping (eqs. advection_update_stages, advection_update_final): the
  explicit tableau of the IMEX scheme, q_0 = q^n,
  q_i = q^n + dt sum_{j<i} a^ex_ij M^-1 a(., q_j, P_CG(Q_j)),
  q^{n+1} = q^n + dt sum_j b^ex_j M^-1 a(., q_j, P_CG(Q_j)) with Q_j the
  stage velocities of the step.  The final sum is printed from j = 1; for
  IMEX Euler (b^ex = (1, 0)) that would leave q unchanged, so it is read
  from j = 0.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .basis import dubiner
from .mesh import LOCAL_EDGES


def _lagrange_nodes(m: int):
    """Equispaced nodes of degree m on the reference triangle, ordered: the
    three vertices (0,0), (1,0), (0,1); the m-1 interior nodes of each local
    edge f (edge opposite vertex f, from its first to its second vertex in
    LOCAL_EDGES); then the interior nodes."""
    V = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    nodes = [V[0], V[1], V[2]]
    kinds = [("v", 0, 0), ("v", 1, 0), ("v", 2, 0)]
    for f, (a, b) in enumerate(LOCAL_EDGES):
        for r in range(1, m):
            nodes.append(V[a] + (V[b] - V[a]) * r / m)
            kinds.append(("e", f, r - 1))
    for j in range(1, m):
        for i in range(1, m - j):
            nodes.append(np.array([i / m, j / m]))
            kinds.append(("c", len(kinds), 0))
    return np.array(nodes), kinds


class CGSpace:
    """CG_m on a (possibly periodic) triangle mesh of the oracle's Mesh class."""

    def __init__(self, disc):
        self.disc = d = disc
        mesh = d.mesh
        self.m = m = d.k + 1
        nodes, kinds = _lagrange_nodes(m)
        Vn = dubiner(m, nodes[:, 0], nodes[:, 1], derivatives=False)  # (nodes, ns)
        self.T = np.linalg.inv(Vn)  # L_a = sum_s T[s, a] phi_s
        nc, ns = mesh.ncells, d.nsu
        nvt = int(mesh.vclass.max()) + 1
        nF = mesh.nfacets
        nint = (m - 1) * (m - 2) // 2
        self.ndof = nvt + nF * (m - 1) + nc * nint
        l2g = np.empty((nc, ns), dtype=np.int64)
        for K in range(nc):
            cint = 0
            for a, (kind, f, r) in enumerate(kinds):
                if kind == "v":
                    l2g[K, a] = mesh.tcells[K, f]
                elif kind == "e":
                    va, vb = LOCAL_EDGES[f]
                    F = mesh.cell_facets[K, f]
                    # node r counted from the edge's first local vertex; the
                    # global order runs from the facet's lower topological id
                    fwd = mesh.tcells[K, va] < mesh.tcells[K, vb]
                    rr = r if fwd else m - 2 - r
                    l2g[K, a] = nvt + F * (m - 1) + rr
                else:
                    l2g[K, a] = nvt + nF * (m - 1) + K * nint + cint
                    cint += 1
        self.l2g = l2g
        # local masses of the Lagrange basis by the cell rule
        MK = np.einsum("sa,kst,tb->kab", self.T, np.einsum("kq,qs,qt->kst", d.cw, d.Vu, d.Vu), self.T)
        rows = np.repeat(l2g[:, :, None], ns, axis=2)
        cols = np.repeat(l2g[:, None, :], ns, axis=1)
        self.M = sp.csr_matrix((MK.ravel(), (rows.ravel(), cols.ravel())), shape=(self.ndof, self.ndof))
        self._lu = spla.splu(self.M.tocsc())
        self.Mdg = np.einsum("kq,qs,qt->kst", d.cw, d.Vu, d.Vu)

    def project(self, Q):
        """Dubiner coefficients (layout of Q) of P_CG(Q)."""
        d = self.disc
        nc, ns = d.mesh.ncells, d.nsu
        Qc = np.asarray(Q).reshape(nc, 2, ns)
        out = np.empty_like(Qc)
        for c in range(2):
            loc = np.einsum("sa,kst,kt->ka", self.T, self.Mdg, Qc[:, c])  # (L_a, Q_c)_K
            b = np.zeros(self.ndof)
            np.add.at(b, self.l2g, loc)
            u = self._lu.solve(b)
            out[:, c] = np.einsum("sa,ka->ks", self.T, u[self.l2g])
        return out.reshape(-1)


def tracer_operator(disc, U):
    """Sparse A with a(chi, q, U) = chi^T A q for the DG_k tracer (pressure
    basis), U the Dubiner coefficients of a continuous velocity."""
    d = disc
    mesh = d.mesh
    nc, npp = mesh.ncells, d.npp
    val, grad = d.eval_cell(U)                 # (nc, nq, 2), (nc, nq, 2 comp, 2 deriv)
    div = grad[..., 0, 0] + grad[..., 1, 1]
    gchiU = np.einsum("kqid,kqd->kqi", d.gp, val)  # grad chi_i . U
    vol = np.einsum("kq,kqi,qj->kij", d.cw, gchiU + d.Vp[None] * div[..., None], d.Vp)
    rows = [np.repeat(np.arange(nc)[:, None, None] * npp + np.arange(npp)[None, :, None], npp, 2).ravel()]
    cols = [np.repeat(np.arange(nc)[:, None, None] * npp + np.arange(npp)[None, None, :], npp, 1).ravel()]
    vals = [vol.ravel()]
    ucf = d.eval_cf(U)                         # (nc, 3, nqf, 2)
    fc = mesh.facet_cells
    I = np.nonzero(mesh.interior)[0]
    Kp, fp, Km, fm = fc[I, 0], fc[I, 1], fc[I, 2], fc[I, 3]
    un = np.einsum("iqd,id->iq", ucf[Kp, fp], d.n[Kp, fp])  # U.n+ from K+
    W = d.cf_w[Kp, fp]
    up = un >= 0.0
    phi = {+1: d.cf_Bp[Kp, fp], -1: d.cf_Bp[Km, fm]}
    cell = {+1: Kp, -1: Km}
    # -<q^up [[chi U.n]]> = -sum_sides <q^up chi_side U.n_side>,  U.n_- = -U.n+
    for sr in (+1, -1):
        for sc in (+1, -1):
            sel = up if sc == +1 else ~up
            blk = -sr * np.einsum("iq,iq,iqa,iqb->iab", W, un * sel, phi[sr], phi[sc])
            rows.append(np.repeat((cell[sr][:, None] * npp + np.arange(npp))[:, :, None], npp, 2).ravel())
            cols.append(np.repeat((cell[sc][:, None] * npp + np.arange(npp))[:, None, :], npp, 1).ravel())
            vals.append(blk.ravel())
    n = nc * npp
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))


class Tracer:
    """Explicit DG tracer transport in the IMEX step (test infrastructure)."""

    def __init__(self, disc, tableau, dt):
        self.disc = disc
        self.tab = tableau
        self.dt = float(dt)
        self.cg = CGSpace(disc)
        d = disc
        Mp = np.einsum("kq,qs,qt->kst", d.cw, d.Vp, d.Vp)
        self.Mp_inv = np.linalg.inv(Mp)

    def minv(self, v):
        d = self.disc
        return np.einsum("kst,kt->ks", self.Mp_inv, v.reshape(d.mesh.ncells, d.npp)).reshape(-1)

    def rate(self, q, Q):
        return self.minv(tracer_operator(self.disc, self.cg.project(Q)) @ q)

    def step(self, q, stages):
        """One step given the stage velocities Q_0 = Q^n, ..., Q_{s-1}."""
        tab, dt = self.tab, self.dt
        s = tab.s
        R = []
        for i in range(s):
            qi = q.copy()
            for j in range(i):
                qi = qi + dt * tab.Aex[i, j] * R[j]
            R.append(self.rate(qi, stages[i]))
        out = q.copy()
        for j in range(s):
            out = out + dt * tab.bex[j] * R[j]
        return out
