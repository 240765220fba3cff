"""Weak forms of the HDG discretisation on tetrahedra (oracle side; test
infrastructure).

The same forms as the two-dimensional oracle (Section 2 of the paper: the
mass, f_im of eq. (f_impl), g and Gamma of Section "Hybridisation", the weak
divergence of Section "Splitting method" in its central-flux reading, the
BDM interpolant of Section "Original fully-implicit DG method"), for d = 3:

* spaces: velocity [P_{k+1}(K)]^3, pressure P_k(K), trace P_k(F) on every
  triangle F (Section "Discontinuous Galerkin spaces");
* layout: Q[cell][c*nsu + s] (component-major), p[cell][s],
  lambda[facet][m], with the bases of the tetrahedral module (orthonormal on
  the reference cell; trace basis in the facet's own coordinates, so both
  cells of a facet see the same trace function);
* h_F is the facet's area (Section "Notation");
* every facet integral is taken at the facet's own quadrature points,
  mapped into each neighbouring cell, so the two sides see the same points;
* the BDM interpolant: Q*|_K in [P_{k+1}(K)]^3 with normal moments against
  P_{k+1}(F) equal to those of {Q}.n on interior facets and zero on walls,
  and interior moments against the first-kind Nedelec space of degree k,
  [P_{k-1}]^3 + x' x [homogeneous P_{k-1}]^3 with x' = (x - centroid)/h_K,
  equal to those of Q.  The counts add up: 4 dim P_{k+1}(F) +
  k(k+2)(k+3)/2 = dim [P_{k+1}(K)]^3.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .forms import _block_diag_coo
from .quadrature import triangle_rule
from .tet import OrthoBasis, TetMesh, cell_points_1d, dim_p2, dim_p3, facet_points_1d, monomial_exponents, tet_rule

D = 3  # spatial dimension
NFC = 4  # facets per cell


class Discretisation3D:
    """Spaces, quadrature tables and assembled forms for one tetrahedral mesh
    and pressure degree k."""

    def __init__(self, coords, cells, k: int, tau: float = 1.0, alpha: float = 1.0,
                 delta_up: float = 1.0):
        if k < 1:
            raise ValueError("pressure degree k >= 1 expected")
        self.mesh = mesh = coords if isinstance(coords, TetMesh) else TetMesh(coords, cells)
        self.k = k
        self.dim = D
        self.tau, self.alpha, self.delta_up = float(tau), float(alpha), float(delta_up)
        nc = mesh.ncells
        self.nsu = dim_p3(k + 1)
        self.nu = D * self.nsu
        self.npp = dim_p3(k)
        self.nf = dim_p2(k)
        self.nQ = nc * self.nu
        self.nP = nc * self.npp
        self.nT = mesh.nfacets * self.nf
        self.basis_u = OrthoBasis(k + 1, 3)
        self.basis_p = OrthoBasis(k, 3)

        # ---- cell quadrature ------------------------------------------------
        pq, wq = tet_rule(cell_points_1d(k))
        self.cell_ref = pq
        self.Vu, dU = self.basis_u.eval(pq, True)
        self.Vp, dP = self.basis_p.eval(pq, True)
        self.cw = wq[None, :] * mesh.absdet[:, None]
        self.cx = mesh.v0[:, None, :] + np.einsum("kab,qb->kqa", mesh.J, pq)
        iJ = mesh.invJ
        # physical gradients [K, q, s, d] = sum_a dref_a[q, s] invJ[K, a, d]
        self.gu = sum(dU[a][None, :, :, None] * iJ[:, None, None, a, :] for a in range(D))
        self.gp = sum(dP[a][None, :, :, None] * iJ[:, None, None, a, :] for a in range(D))

        # ---- facet quadrature: each facet's own points ----------------------
        pf, wf = triangle_rule(facet_points_1d(k))
        self.fpts, self.fw = pf, wf
        self.mu = OrthoBasis(k, 2, scale=2.0).eval(pf)            # (nqf, nf)
        self.nu_bdm = OrthoBasis(k + 1, 2, scale=2.0).eval(pf)    # (nqf, dim P_{k+1}(F))
        Fcf = mesh.cell_facets
        fx = mesh.facet_v0[:, None, :] + np.einsum("fda,qa->fqd", mesh.facet_E, pf)  # (nF, nqf, 3)
        self.cf_x = fx[Fcf]                                       # (nc, 4, nqf, 3)
        self.cf_w = wf[None, None, :] * 2.0 * mesh.area[Fcf][:, :, None]
        Kidx = np.repeat(np.arange(nc), NFC * pf.shape[0]).reshape(nc, NFC, -1)
        ref = mesh.to_reference(Kidx, self.cf_x).reshape(-1, D)
        nq = pf.shape[0]
        self.cf_Bu = self.basis_u.eval(ref).reshape(nc, NFC, nq, self.nsu)
        self.cf_Bp = self.basis_p.eval(ref).reshape(nc, NFC, nq, self.npp)
        self.n = mesh.normal
        self._static = None

    # ------------------------------------------------------------------ eval
    def split(self, Q):
        return np.asarray(Q).reshape(self.mesh.ncells, D, self.nsu)

    def eval_cell(self, Q):
        """Values (nc, nq, 3) and gradients (nc, nq, 3 comp, 3 deriv) at cell points."""
        Qc = self.split(Q)
        return np.einsum("qs,kcs->kqc", self.Vu, Qc), np.einsum("kqsd,kcs->kqcd", self.gu, Qc)

    def eval_cf(self, Q):
        return np.einsum("kfqs,kcs->kfqc", self.cf_Bu, self.split(Q))

    def eval_cf_pressure(self, p):
        return np.einsum("kfqs,ks->kfq", self.cf_Bp, np.asarray(p).reshape(-1, self.npp))

    def eval_trace(self, lam):
        return np.asarray(lam).reshape(-1, self.nf) @ self.mu.T

    def _points(self, x):
        return [x[..., a] for a in range(D)]

    # ---------------------------------------------------------------- masses
    def _vel_block(self, sblk):
        nc = sblk.shape[0]
        blk = np.zeros((nc, D, self.nsu, D, self.nsu))
        for c in range(D):
            blk[:, c, :, c, :] = sblk
        return blk.reshape(nc, self.nu, self.nu)

    def mass(self):
        nc = self.mesh.ncells
        ms = np.einsum("kq,qi,qj->kij", self.cw, self.Vu, self.Vu)
        off = np.arange(nc) * self.nu
        r, c, v = _block_diag_coo(self._vel_block(ms), off, off)
        return sp.csr_matrix((v, (r, c)), shape=(self.nQ, self.nQ))

    def l2_project_velocity(self, fun):
        """L2 projection of fun(x, y, z) -> (..., 3) onto V_Q by the cell rule."""
        vals = fun(*self._points(self.cx))
        ms = np.einsum("kq,qi,qj->kij", self.cw, self.Vu, self.Vu)
        rhs = np.einsum("kq,qi,kqc->kci", self.cw, self.Vu, vals)
        return np.linalg.solve(ms[:, None], rhs[..., None])[..., 0].reshape(-1)

    def l2_project_pressure(self, fun):
        vals = fun(*self._points(self.cx))
        ms = np.einsum("kq,qi,qj->kij", self.cw, self.Vp, self.Vp)
        rhs = np.einsum("kq,qi,kq->ki", self.cw, self.Vp, vals)
        return np.linalg.solve(ms, rhs[..., None])[..., 0].reshape(-1)

    def pressure_integral(self, p):
        vals = np.einsum("qs,ks->kq", self.Vp, np.asarray(p).reshape(-1, self.npp))
        return float(np.sum(self.cw * vals))

    def domain_area(self):
        return float(np.sum(self.cw))

    def constant_pressure(self):
        return self.l2_project_pressure(lambda x, y, z: np.ones_like(x))

    def constant_trace(self):
        """Coefficients of the trace function equal to 1 on every facet."""
        w = self.fw
        proj = np.linalg.solve(self.mu.T @ (w[:, None] * self.mu), self.mu.T @ w)
        return np.tile(proj, self.mesh.nfacets)

    def kinetic_energy(self, Q):
        val, _ = self.eval_cell(Q)
        return 0.5 * float(np.sum(self.cw[:, :, None] * val * val))

    # -------------------------------------------------------------- f_im
    def advection(self, Qs):
        """Sparse A with f_im(w, Q, Qs) = w^T A Q (eq. f_impl)."""
        mesh = self.mesh
        nc, nu = mesh.ncells, self.nu
        rows, cols, vals = [], [], []
        qs, _ = self.eval_cell(Qs)
        adv = np.einsum("kqd,kqjd->kqj", qs, self.gu)
        sblk = -np.einsum("kq,qi,kqj->kij", self.cw, self.Vu, adv)
        off = np.arange(nc) * nu
        r, c, v = _block_diag_coo(self._vel_block(sblk), off, off)
        rows.append(r); cols.append(c); vals.append(v)

        qcf = self.eval_cf(Qs)
        fc = mesh.facet_cells
        I = np.nonzero(mesh.interior)[0]
        Kp, fp, Km, fm = fc[I, 0], fc[I, 1], fc[I, 2], fc[I, 3]
        n = self.n[Kp, fp]
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
                b = np.einsum("cd,iab->icadb", np.eye(D), central + upwind) + np.einsum("icd,iab->icadb", nn, pen)
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
        """Sparse operators of g, Gamma and Div, in the two-dimensional oracle's
        notation (g = Gp p + Gl lam, Gamma = (Dv Q + Tpp p + Tpl lam,
        Cl Q + Elp p + Fll lam), Div = Dc F)."""
        if self._static is not None:
            return self._static
        mesh = self.mesh
        nc, nu, npp, nf = mesh.ncells, self.nu, self.npp, self.nf
        tau = self.tau
        Kall = np.arange(nc)
        Fcf = mesh.cell_facets

        Gp_blk = np.einsum("kq,qs,kqic->kcis", self.cw, self.Vp, self.gu).reshape(nc, nu, npp)
        r, c, v = _block_diag_coo(Gp_blk, Kall * nu, Kall * npp)
        Gp = sp.csr_matrix((v, (r, c)), shape=(self.nQ, self.nP))

        Gl_blk = -np.einsum("kfq,qm,kfqi,kfc->kfcim", self.cf_w, self.mu, self.cf_Bu, self.n).reshape(nc, NFC, nu, nf)
        r, c, v = _block_diag_coo(Gl_blk.reshape(nc * NFC, nu, nf), np.repeat(Kall, NFC) * nu, Fcf.ravel() * nf)
        Gl = sp.csr_matrix((v, (r, c)), shape=(self.nQ, self.nT))

        Tpp_blk = tau * np.einsum("kfq,kfqs,kfqt->kst", self.cf_w, self.cf_Bp, self.cf_Bp)
        r, c, v = _block_diag_coo(Tpp_blk, Kall * npp, Kall * npp)
        Tpp = sp.csr_matrix((v, (r, c)), shape=(self.nP, self.nP))

        Tpl_blk = -tau * np.einsum("kfq,kfqs,qm->kfsm", self.cf_w, self.cf_Bp, self.mu)
        r, c, v = _block_diag_coo(Tpl_blk.reshape(nc * NFC, npp, nf), np.repeat(Kall, NFC) * npp, Fcf.ravel() * nf)
        Tpl = sp.csr_matrix((v, (r, c)), shape=(self.nP, self.nT))

        self.blocks = dict(Gp=Gp_blk, Gl=Gl_blk, Tpp=Tpp_blk, Tpl=Tpl_blk,
                           M=np.einsum("kq,qi,qj->kij", self.cw, self.Vu, self.Vu))
        F_blk = -tau * np.einsum("kfq,qm,qn->kfmn", self.cf_w, self.mu, self.mu)
        r, c, v = _block_diag_coo(F_blk.reshape(nc * NFC, nf, nf), Fcf.ravel() * nf, Fcf.ravel() * nf)
        Fll = sp.csr_matrix((v, (r, c)), shape=(self.nT, self.nT))

        Dc_vol = -np.einsum("kq,kqsc,qi->ksci", self.cw, self.gp, self.Vu).reshape(nc, npp, nu)
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
        self._static = dict(Gp=Gp, Gl=Gl, Dv=Gp.T.tocsr(), Tpp=Tpp, Tpl=Tpl, Cl=(-Gl.T).tocsr(),
                            Elp=(-Tpl.T).tocsr(), Fll=Fll, Dc=Dc)
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
        """Div(psi, f) for f given at cell points (nc, nq, 3) and at each cell's
        facet points (nc, 4, nqf, 3) (one-sided values; averaged here)."""
        mesh = self.mesh
        vol = -np.einsum("kq,kqsc,kqc->ks", self.cw, self.gp, fcell)
        nb, nbf = mesh.nb_cell, mesh.nb_facet
        inter = nb >= 0
        fn = np.where(inter[:, :, None, None], fcf[np.maximum(nb, 0), np.maximum(nbf, 0)], 0.0)
        flux = np.einsum("kfqc,kfc->kfq", 0.5 * (fcf + fn), self.n) * inter[:, :, None]
        return (vol + np.einsum("kfq,kfqs,kfq->ks", self.cf_w, self.cf_Bp, flux)).reshape(-1)

    def boundary_normal_flux(self, fcf):
        """-sum over wall facets <mu n.f>, for f given at facet points (nc, 4, nqf, 3)."""
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
        mesh = self.mesh
        nc = mesh.ncells
        Kidx = np.repeat(np.arange(nc), NFC * self.fpts.shape[0]).reshape(nc, NFC, -1)
        ref = mesh.to_reference(Kidx, self.cf_x).reshape(-1, D)
        V, dref = self.basis_u.eval(ref, True)
        sh = (nc, NFC, -1, self.nsu)
        V = V.reshape(sh)
        dref = [d.reshape(sh) for d in dref]
        iJ = mesh.invJ
        Qc = self.split(Q)
        fval = np.einsum("kfqs,kcs->kfqc", V, Qc)
        fac = np.zeros_like(fval)
        for x in range(D):
            gx = sum(dref[a] * iJ[:, None, None, None, a, x] for a in range(D))
            fac += fval[..., x:x + 1] * np.einsum("kfqs,kcs->kfqc", gx, Qc)
        return cell, fac

    # ------------------------------------------------------------ projection
    def nedelec_basis(self, x, K):
        """First-kind Nedelec space of degree k on cell K at physical points x
        (..., 3): [P_{k-1}]^3 plus x' x (m e_j) for homogeneous monomials m of
        degree k-1, j = 0, 1, and j = 2 with m free of z (the products with
        m = z q are combinations of the others, since x' x (x' q) = 0).
        Returns (..., k(k+2)(k+3)/2, 3)."""
        mesh = self.mesh
        k = self.k
        centroid = mesh.coords[mesh.cells[K]].mean(axis=-2)
        hK = np.cbrt(mesh.absdet[K])
        xp = (x - centroid[..., None, :]) / hK[..., None, None]
        funcs = []
        z0 = np.zeros(xp.shape[:-1])
        for e in monomial_exponents(k - 1, 3):
            m = np.prod(xp ** np.array(e), axis=-1)
            for c in range(D):
                f = [z0, z0, z0]
                f[c] = m
                funcs.append(np.stack(f, -1))
        for e in monomial_exponents(k - 1, 3):
            if sum(e) != k - 1:
                continue
            m = np.prod(xp ** np.array(e), axis=-1)
            for j in range(D):
                if j == 2 and e[2] > 0:
                    continue
                ej = np.zeros(3)
                ej[j] = 1.0
                funcs.append(np.cross(xp, ej) * m[..., None])
        return np.stack(funcs, axis=-2)

    def bdm_project(self, Q):
        """Q* = P(Q): BDM interpolant with averaged normal moments."""
        mesh = self.mesh
        nc, nu = mesh.ncells, self.nu
        nm = self.nu_bdm.shape[1]
        A = np.zeros((nc, nu, nu))
        rhs = np.zeros((nc, nu))
        qcf = self.eval_cf(Q)
        nb, nbf = mesh.nb_cell, mesh.nb_facet
        inter = nb >= 0
        for f in range(NFC):
            W = self.cf_w[:, f]
            n = self.n[:, f]
            A[:, f * nm:(f + 1) * nm, :] = np.einsum("kq,qm,kqi,kc->kmci", W, self.nu_bdm, self.cf_Bu[:, f], n).reshape(nc, nm, nu)
            qnb = qcf[np.maximum(nb[:, f], 0), np.maximum(nbf[:, f], 0)]
            flux = np.einsum("kqc,kc->kq", 0.5 * (qcf[:, f] + qnb), n) * inter[:, f][:, None]
            rhs[:, f * nm:(f + 1) * nm] = np.einsum("kq,qm,kq->km", W, self.nu_bdm, flux)
        v = self.nedelec_basis(self.cx, np.arange(nc))
        r0 = NFC * nm
        A[:, r0:, :] = np.einsum("kq,kqlc,qi->klci", self.cw, v, self.Vu).reshape(nc, -1, nu)
        val, _ = self.eval_cell(Q)
        rhs[:, r0:] = np.einsum("kq,kqlc,kqc->kl", self.cw, v, val)
        return np.linalg.solve(A, rhs[..., None])[..., 0].reshape(-1)
