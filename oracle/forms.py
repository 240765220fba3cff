"""Weak forms of the HDG discretisation (oracle side; test infrastructure).

Every operator is assembled as a SciPy sparse matrix from element integrals
evaluated by quadrature at physical points that are mapped back into each
cell, so the two sides of a facet always see the same physical points.  The
unknown layout is the documented one: Q[cell][c*ns + s] (component-major),
p[cell][s], lambda[facet][m].

Forms (Section 2 of the paper):

* mass m(Q, w) = (w.Q)_Omega;
* implicit advection f_im(w, Q, Q*), eq. (f_impl): volume term, central facet
  term, interior-penalty term with weight alpha/h_F on interior and boundary
  facets, upwind term with weight delta_up |Q*.n+|;
* weak pressure gradient g(w, p, lambda) and constraint Gamma(psi, mu, Q, p,
  lambda) from Section "Hybridisation" (the two-sided facet sums written as
  sums over cell boundaries);
* weak divergence Div(psi, F) of Section "Splitting method", read as the
  central-flux form  sum_K [ -(grad psi, F)_K + <psi {F}.n_K>_dK ]  with
  {F}.n = 0 on walls, so that Div(1, F) = 0 and the singular mixed problems
  stay solvable;
* the BDM interpolant Q* = P(Q) (Section "Original fully-implicit DG
  method"), read as: Q*|_K in [P_{k+1}(K)]^2 with normal moments against
  P_{k+1}(F) equal to those of {Q}.n on interior facets and zero on walls,
  and interior moments against the first-kind Nedelec space of degree k
  equal to those of Q.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .basis import dim_p, dubiner, legendre01
from .mesh import Mesh
from .quadrature import cell_points_1d, facet_points, gauss_legendre_01, triangle_rule


def _block_diag_coo(blocks, row_off, col_off):
    """COO triplets for dense blocks (nb, r, c) placed at row_off[b], col_off[b]."""
    nb, r, c = blocks.shape
    rr = row_off[:, None, None] + np.arange(r)[None, :, None]
    cc = col_off[:, None, None] + np.arange(c)[None, None, :]
    rr = np.broadcast_to(rr, blocks.shape)
    cc = np.broadcast_to(cc, blocks.shape)
    return rr.ravel(), cc.ravel(), blocks.ravel()


class Discretisation:
    """Spaces, quadrature tables and assembled forms for one mesh and degree k."""

    def __init__(self, coords, cells, k: int, tau: float = 1.0, alpha: float = 1.0,
                 delta_up: float = 1.0):
        if k < 1:
            raise ValueError("pressure degree k >= 1 expected")
        self.mesh = mesh = coords if isinstance(coords, Mesh) else Mesh(coords, cells)
        self.k = k
        self.tau, self.alpha, self.delta_up = float(tau), float(alpha), float(delta_up)
        nc = mesh.ncells
        self.nsu = dim_p(k + 1)
        self.nu = 2 * self.nsu
        self.npp = dim_p(k)
        self.nf = k + 1
        self.nQ = nc * self.nu
        self.nP = nc * self.npp
        self.nT = mesh.nfacets * self.nf

        # ---- cell quadrature ------------------------------------------------
        pq, wq = triangle_rule(cell_points_1d(k))
        self.cell_ref = pq
        self.Vu, dxu, dyu = dubiner(k + 1, pq[:, 0], pq[:, 1])
        self.Vp, dxp, dyp = dubiner(k, pq[:, 0], pq[:, 1])
        self.cw = wq[None, :] * mesh.absdet[:, None]  # (nc, nq)
        self.cx = mesh.v0[:, None, :] + np.einsum("kab,qb->kqa", mesh.J, pq)
        iJ = mesh.invJ
        # physical gradients [K, q, s, d] = sum_a dref[q, s, a] invJ[K, a, d]
        self.gu = dxu[None, :, :, None] * iJ[:, None, None, 0, :] + dyu[None, :, :, None] * iJ[:, None, None, 1, :]
        self.gp = dxp[None, :, :, None] * iJ[:, None, None, 0, :] + dyp[None, :, :, None] * iJ[:, None, None, 1, :]

        # ---- facet quadrature, per (cell, local facet) ----------------------
        t, wt = gauss_legendre_01(facet_points(k))
        self.ft = t
        self.mu = legendre01(k, t)          # trace basis (nqf, nf)
        self.nu_bdm = legendre01(k + 1, t)  # BDM facet moments (nqf, k+2)
        Fcf = mesh.cell_facets             # (nc, 3)
        self.cf_x = mesh.cell_facet_points(t)  # (nc, 3, nqf, 2), each cell's own geometry
        self.cf_w = wt[None, None, :] * mesh.hF[Fcf][:, :, None]
        Kidx = np.repeat(np.arange(nc), 3 * t.size).reshape(nc, 3, t.size)
        ref = mesh.to_reference(Kidx, self.cf_x)  # (nc, 3, nqf, 2)
        r = ref.reshape(-1, 2)
        self.cf_Bu = dubiner(k + 1, r[:, 0], r[:, 1], derivatives=False).reshape(nc, 3, t.size, self.nsu)
        self.cf_Bp = dubiner(k, r[:, 0], r[:, 1], derivatives=False).reshape(nc, 3, t.size, self.npp)
        self.n = mesh.normal                 # (nc, 3, 2)

        self._static = None

    # ------------------------------------------------------------------ eval
    def split(self, Q):
        """(nQ,) -> (nc, 2, nsu)"""
        return np.asarray(Q).reshape(self.mesh.ncells, 2, self.nsu)

    def eval_cell(self, Q):
        """Values (nc, nq, 2) and gradients (nc, nq, 2 comp, 2 deriv) at cell points."""
        Qc = self.split(Q)
        val = np.einsum("qs,kcs->kqc", self.Vu, Qc)
        grad = np.einsum("kqsd,kcs->kqcd", self.gu, Qc)
        return val, grad

    def eval_cf(self, Q):
        """Values (nc, 3, nqf, 2) of each cell's own polynomial at its facet points."""
        return np.einsum("kfqs,kcs->kfqc", self.cf_Bu, self.split(Q))

    def eval_cf_pressure(self, p):
        return np.einsum("kfqs,ks->kfq", self.cf_Bp, np.asarray(p).reshape(-1, self.npp))

    def eval_trace(self, lam):
        """Trace values on every facet at its quadrature points (nF, nqf)."""
        return np.asarray(lam).reshape(-1, self.nf) @ self.mu.T

    # ---------------------------------------------------------------- masses
    def mass(self):
        nc = self.mesh.ncells
        ms = np.einsum("kq,qi,qj->kij", self.cw, self.Vu, self.Vu)
        blk = np.zeros((nc, 2, self.nsu, 2, self.nsu))
        blk[:, 0, :, 0, :] = ms
        blk[:, 1, :, 1, :] = ms
        off = np.arange(nc) * self.nu
        r, c, v = _block_diag_coo(blk.reshape(nc, self.nu, self.nu), off, off)
        return sp.csr_matrix((v, (r, c)), shape=(self.nQ, self.nQ))

    def l2_project_velocity(self, fun):
        """L2 projection of fun(x, y) -> (..., 2) onto V_Q, using the cell rule."""
        vals = fun(self.cx[..., 0], self.cx[..., 1])  # (nc, nq, 2)
        ms = np.einsum("kq,qi,qj->kij", self.cw, self.Vu, self.Vu)
        rhs = np.einsum("kq,qi,kqc->kci", self.cw, self.Vu, vals)
        coef = np.linalg.solve(ms[:, None], rhs[..., None])[..., 0]
        return coef.reshape(-1)

    def l2_project_pressure(self, fun):
        vals = fun(self.cx[..., 0], self.cx[..., 1])
        ms = np.einsum("kq,qi,qj->kij", self.cw, self.Vp, self.Vp)
        rhs = np.einsum("kq,qi,kq->ki", self.cw, self.Vp, vals)
        return np.linalg.solve(ms, rhs[..., None])[..., 0].reshape(-1)

    def pressure_integral(self, p):
        """int_Omega p dx by the cell rule."""
        vals = np.einsum("qs,ks->kq", self.Vp, np.asarray(p).reshape(-1, self.npp))
        return float(np.sum(self.cw * vals))

    def domain_area(self):
        return float(np.sum(self.cw))

    def constant_pressure(self):
        return self.l2_project_pressure(lambda x, y: np.ones_like(x))

    def constant_trace(self):
        """Coefficients of the trace function equal to 1 on every facet."""
        w = gauss_legendre_01(self.ft.size)[1]
        proj = np.linalg.solve(self.mu.T @ (w[:, None] * self.mu), self.mu.T @ w)
        return np.tile(proj, self.mesh.nfacets)

    def kinetic_energy(self, Q):
        val, _ = self.eval_cell(Q)
        return 0.5 * float(np.sum(self.cw[:, :, None] * val * val))

    # -------------------------------------------------------------- f_im
    def advection(self, Qs):
        """Sparse A with f_im(w, Q, Qs) = w^T A Q  (eq. f_impl)."""
        mesh = self.mesh
        nc, nsu, nu = mesh.ncells, self.nsu, self.nu
        rows, cols, vals = [], [], []

        # volume: -(w . (Qs . grad) Q)_K, same scalar block for both components
        qs, _ = self.eval_cell(Qs)
        adv = np.einsum("kqd,kqjd->kqj", qs, self.gu)
        sblk = -np.einsum("kq,qi,kqj->kij", self.cw, self.Vu, adv)
        blk = np.zeros((nc, 2, nsu, 2, nsu))
        blk[:, 0, :, 0, :] = sblk
        blk[:, 1, :, 1, :] = sblk
        off = np.arange(nc) * nu
        r, c, v = _block_diag_coo(blk.reshape(nc, nu, nu), off, off)
        rows.append(r); cols.append(c); vals.append(v)

        qcf = self.eval_cf(Qs)  # (nc, 3, nqf, 2)
        fc = mesh.facet_cells
        I = np.nonzero(mesh.interior)[0]
        Kp, fp, Km, fm = fc[I, 0], fc[I, 1], fc[I, 2], fc[I, 3]
        n = self.n[Kp, fp]  # n+
        W = self.cf_w[Kp, fp]
        h = mesh.hF[I]
        qn = 0.5 * np.einsum("iqd,id->iq", qcf[Kp, fp] + qcf[Km, fm], n)
        phi = {+1: self.cf_Bu[Kp, fp], -1: self.cf_Bu[Km, fm]}
        cell = {+1: Kp, -1: Km}
        nn = np.einsum("ia,ib->iab", n, n)
        for sr in (+1, -1):
            for sc in (+1, -1):
                central = 0.5 * sc * np.einsum("iq,iq,iqa,iqb->iab", W, qn, phi[sr], phi[sc])
                upwind = -self.delta_up * sr * sc * np.einsum("iq,iq,iqa,iqb->iab", W, np.abs(qn), phi[sr], phi[sc])
                pen = -self.alpha * sr * sc * np.einsum("iq,iqa,iqb->iab", W, phi[sr], phi[sc]) / h[:, None, None]
                b = np.einsum("cd,iab->icadb", np.eye(2), central + upwind) + np.einsum("icd,iab->icadb", nn, pen)
                r, c, v = _block_diag_coo(b.reshape(-1, nu, nu), cell[sr] * nu, cell[sc] * nu)
                rows.append(r); cols.append(c); vals.append(v)

        B = np.nonzero(~mesh.interior)[0]
        Kb, fb = fc[B, 0], fc[B, 1]
        n = self.n[Kb, fb]
        W = self.cf_w[Kb, fb]
        pen = -self.alpha * np.einsum("iq,iqa,iqb->iab", W, self.cf_Bu[Kb, fb], self.cf_Bu[Kb, fb]) / mesh.hF[B][:, None, None]
        b = np.einsum("icd,iab->icadb", np.einsum("ia,ib->iab", n, n), pen)
        r, c, v = _block_diag_coo(b.reshape(-1, nu, nu), Kb * nu, Kb * nu)
        rows.append(r); cols.append(c); vals.append(v)

        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(self.nQ, self.nQ))

    # ------------------------------------------------- g, Gamma and friends
    def static_operators(self):
        """Sparse operators of g and Gamma (independent of the state).

        g(w, p, lam)            = w^T (Gp p + Gl lam)
        Gamma(psi, mu, Q, p, l) = psi^T (Dv Q + Tpp p + Tpl l) + mu^T (Cl Q + Elp p + Fll l)
        Div(psi, F)             = psi^T Dc F
        """
        if self._static is not None:
            return self._static
        mesh = self.mesh
        nc, nu, npp, nf, nsu = mesh.ncells, self.nu, self.npp, self.nf, self.nsu
        tau = self.tau
        Kall = np.arange(nc)

        # (p, div w)_K: Gp[K, (c,i), s] = sum_q cw Vp[q,s] d_c phi_i
        Gp_blk = np.einsum("kq,qs,kqic->kcis", self.cw, self.Vp, self.gu).reshape(nc, nu, npp)
        r, c, v = _block_diag_coo(Gp_blk, Kall * nu, Kall * npp)
        Gp = sp.csr_matrix((v, (r, c)), shape=(self.nQ, self.nP))

        # -<lam, w.n_K>_dK, per (cell, local facet)
        Gl_blk = -np.einsum("kfq,qm,kfqi,kfc->kfcim", self.cf_w, self.mu, self.cf_Bu, self.n).reshape(nc, 3, nu, nf)
        Fcf = mesh.cell_facets
        r, c, v = _block_diag_coo(Gl_blk.reshape(nc * 3, nu, nf), np.repeat(Kall, 3) * nu, Fcf.ravel() * nf)
        Gl = sp.csr_matrix((v, (r, c)), shape=(self.nQ, self.nT))

        Tpp_blk = tau * np.einsum("kfq,kfqs,kfqt->kst", self.cf_w, self.cf_Bp, self.cf_Bp)
        r, c, v = _block_diag_coo(Tpp_blk, Kall * npp, Kall * npp)
        Tpp = sp.csr_matrix((v, (r, c)), shape=(self.nP, self.nP))

        Tpl_blk = -tau * np.einsum("kfq,kfqs,qm->kfsm", self.cf_w, self.cf_Bp, self.mu)
        r, c, v = _block_diag_coo(Tpl_blk.reshape(nc * 3, npp, nf), np.repeat(Kall, 3) * npp, Fcf.ravel() * nf)
        Tpl = sp.csr_matrix((v, (r, c)), shape=(self.nP, self.nT))

        self.blocks = dict(Gp=Gp_blk, Gl=Gl_blk, Tpp=Tpp_blk, Tpl=Tpl_blk,
                           M=np.einsum("kq,qi,qj->kij", self.cw, self.Vu, self.Vu))
        Dv = Gp.T.tocsr()
        Cl = (-Gl.T).tocsr()
        Elp = (-Tpl.T).tocsr()

        F_blk = -tau * np.einsum("kfq,qm,qn->kfmn", self.cf_w, self.mu, self.mu)
        r, c, v = _block_diag_coo(F_blk.reshape(nc * 3, nf, nf), Fcf.ravel() * nf, Fcf.ravel() * nf)
        Fll = sp.csr_matrix((v, (r, c)), shape=(self.nT, self.nT))

        # weak divergence, central flux
        Dc_vol = -np.einsum("kq,kqsc,qi->ksci", self.cw, self.gp, self.Vu)
        Dc_vol = Dc_vol.reshape(nc, npp, nu)
        r, c, v = _block_diag_coo(Dc_vol, Kall * npp, Kall * nu)
        rows, cols, vals = [r], [c], [v]
        fc = mesh.facet_cells
        I = np.nonzero(mesh.interior)[0]
        side = [(fc[I, 0], fc[I, 1]), (fc[I, 2], fc[I, 3])]
        for (Kr, frr) in side:
            W = self.cf_w[Kr, frr]
            n = self.n[Kr, frr]
            for (Kc, fcc) in side:
                b = 0.5 * np.einsum("iq,iqs,iqj,ic->iscj", W, self.cf_Bp[Kr, frr], self.cf_Bu[Kc, fcc], n)
                r, c, v = _block_diag_coo(b.reshape(-1, npp, nu), Kr * npp, Kc * nu)
                rows.append(r); cols.append(c); vals.append(v)
        Dc = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                           shape=(self.nP, self.nQ))
        self._static = dict(Gp=Gp, Gl=Gl, Dv=Dv, Tpp=Tpp, Tpl=Tpl, Cl=Cl, Elp=Elp, Fll=Fll, Dc=Dc)
        return self._static

    def g(self, p, lam):
        s = self.static_operators()
        return s["Gp"] @ p + s["Gl"] @ lam

    def gamma(self, Q, p, lam):
        s = self.static_operators()
        return (s["Dv"] @ Q + s["Tpp"] @ p + s["Tpl"] @ lam,
                s["Cl"] @ Q + s["Elp"] @ p + s["Fll"] @ lam)

    def div_c(self, F):
        return self.static_operators()["Dc"] @ F

    def div_c_points(self, fcell, fcf):
        """Div(psi, f) for f given at cell points (nc, nq, 2) and at each cell's
        facet points (nc, 3, nqf, 2) (one-sided values; averaged here)."""
        mesh = self.mesh
        vol = -np.einsum("kq,kqsc,kqc->ks", self.cw, self.gp, fcell)
        nb, nbf = mesh.nb_cell, mesh.nb_facet
        inter = nb >= 0
        fn = np.where(inter[:, :, None, None], fcf[np.maximum(nb, 0), np.maximum(nbf, 0)], 0.0)
        favg = 0.5 * (fcf + fn)
        flux = np.einsum("kfqc,kfc->kfq", favg, self.n) * inter[:, :, None]
        fac = np.einsum("kfq,kfqs,kfq->ks", self.cf_w, self.cf_Bp, flux)
        return (vol + fac).reshape(-1)

    def boundary_normal_flux(self, fcf):
        """-sum over wall facets <mu n.f>, for f given at facet points (nc, 3, nqf, 2)."""
        mesh = self.mesh
        out = np.zeros((mesh.nfacets, self.nf))
        fc = mesh.facet_cells
        B = np.nonzero(~mesh.interior)[0]
        Kb, fb = fc[B, 0], fc[B, 1]
        fn = np.einsum("iqc,ic->iq", fcf[Kb, fb], self.n[Kb, fb])
        out[B] = -np.einsum("iq,qm,iq->im", self.cf_w[Kb, fb], self.mu, fn)
        return out.reshape(-1)

    def convection_points(self, Q):
        """(Q . grad) Q with the broken gradient, at cell points and facet points."""
        val, grad = self.eval_cell(Q)
        cell = np.einsum("kqd,kqcd->kqc", val, grad)
        Qc = self.split(Q)
        # gradients at facet points need the basis gradients there
        return cell, self._convection_facets(Qc)

    def _convection_facets(self, Qc):
        mesh = self.mesh
        nc = mesh.ncells
        ref = mesh.to_reference(np.repeat(np.arange(nc), 3 * self.ft.size).reshape(nc, 3, -1), self.cf_x)
        r = ref.reshape(-1, 2)
        V, dx, dy = dubiner(self.k + 1, r[:, 0], r[:, 1])
        V = V.reshape(nc, 3, -1, self.nsu)
        dx = dx.reshape(V.shape)
        dy = dy.reshape(V.shape)
        iJ = mesh.invJ
        gx = dx * iJ[:, None, None, None, 0, 0] + dy * iJ[:, None, None, None, 1, 0]
        gy = dx * iJ[:, None, None, None, 0, 1] + dy * iJ[:, None, None, None, 1, 1]
        val = np.einsum("kfqs,kcs->kfqc", V, Qc)
        dQx = np.einsum("kfqs,kcs->kfqc", gx, Qc)
        dQy = np.einsum("kfqs,kcs->kfqc", gy, Qc)
        return val[..., 0:1] * dQx + val[..., 1:2] * dQy

    # ------------------------------------------------------------ projection
    def nedelec_basis(self, x, K):
        """First-kind Nedelec space of degree k on cell K at physical points x (..., 2):
        [P_{k-1}]^2 plus x'^perp times homogeneous P_{k-1}, x' = (x - centroid)/h_K.
        Returns (..., k(k+2), 2)."""
        mesh = self.mesh
        k = self.k
        centroid = mesh.coords[mesh.cells[K]].mean(axis=-2)
        hK = np.sqrt(mesh.absdet[K])
        xp = (x - centroid[..., None, :]) / hK[..., None, None]
        X, Y = xp[..., 0], xp[..., 1]
        funcs = []
        for d in range(k):
            for a in range(d + 1):
                m = X ** (d - a) * Y ** a
                z = np.zeros_like(m)
                funcs.append(np.stack([m, z], -1))
                funcs.append(np.stack([z, m], -1))
        for a in range(k):
            m = X ** (k - 1 - a) * Y ** a
            funcs.append(np.stack([-Y * m, X * m], -1))
        return np.stack(funcs, axis=-2)

    def bdm_project(self, Q):
        """Q* = P(Q): BDM interpolant with averaged normal moments (reading of the
        paper's reference to an external definition; see module header)."""
        mesh = self.mesh
        nc, nsu, nu, k = mesh.ncells, self.nsu, self.nu, self.k
        nm = k + 2
        A = np.zeros((nc, nu, nu))
        rhs = np.zeros((nc, nu))
        qcf = self.eval_cf(Q)
        nb, nbf = mesh.nb_cell, mesh.nb_facet
        inter = nb >= 0
        for f in range(3):
            W = self.cf_w[:, f]
            n = self.n[:, f]
            A[:, f * nm:(f + 1) * nm, :] = np.einsum("kq,qm,kqi,kc->kmci", W, self.nu_bdm, self.cf_Bu[:, f], n).reshape(nc, nm, nu)
            qnb = qcf[np.maximum(nb[:, f], 0), np.maximum(nbf[:, f], 0)]
            avg = 0.5 * (qcf[:, f] + qnb)
            flux = np.einsum("kqc,kc->kq", avg, n) * inter[:, f][:, None]
            rhs[:, f * nm:(f + 1) * nm] = np.einsum("kq,qm,kq->km", W, self.nu_bdm, flux)
        v = self.nedelec_basis(self.cx, np.arange(nc))  # (nc, nq, nn, 2)
        r0 = 3 * nm
        A[:, r0:, :] = np.einsum("kq,kqlc,qi->klci", self.cw, v, self.Vu).reshape(nc, -1, nu)
        val, _ = self.eval_cell(Q)
        rhs[:, r0:] = np.einsum("kq,kqlc,kqc->kl", self.cw, v, val)
        return np.linalg.solve(A, rhs[..., None])[..., 0].reshape(-1)
