"""Hybridised mixed solve (oracle side; test infrastructure).

Solves, for a given c > 0, the linear problem shared by the pressure increment
(Algorithm 2, Step II, c = 1), the final projection (Algorithm 1, c = dt b_{s-1})
and the pressure reconstruction (Section "Pressure reconstruction", c = 1):

    (U, w)_Omega - c g(w, p, lambda) = F_w(w)
    Gamma(psi, mu, U, p, lambda)     = F_psi(psi) + F_mu(mu)

for all (w, psi, mu).  Following the paper's solver (Section "Solvers and
preconditioners": Schur-complement reduction onto lambda), the cell unknowns
x_K = (U_K, p_K) are eliminated cell by cell:

    A_K x_K + B_K lambda_K = f_K,      sum_K L_K x_K + Fll lambda = f_mu,
    S = sum_K L_K A_K^{-1} B_K - Fll,  g = sum_K L_K A_K^{-1} f_K - f_mu,
    x_K = A_K^{-1} (f_K - B_K lambda_K).

S is singular: (U, p, lambda) = (0, 1, 1) solves the homogeneous problem.  The
trace system is solved directly with one trace coefficient pinned, and the
pressure level is then fixed by int_Omega p = 0, as the space V_p demands
(Section "Discontinuous Galerkin spaces").
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


class HDGSolver:
    def __init__(self, disc, c: float):
        self.disc = disc
        self.c = float(c)
        d = disc
        s = d.static_operators()
        b = d.blocks
        mesh = d.mesh
        nc, nu, npp, nf = mesh.ncells, d.nu, d.npp, d.nf
        nfc = mesh.cell_facets.shape[1]  # facets per cell: 3 (triangles), 4 (tetrahedra)
        nl = nu + npp
        self.nl = nl
        Mk = np.zeros((nc, nu, nu))
        for comp in range(nu // d.nsu):
            sl = slice(comp * d.nsu, (comp + 1) * d.nsu)
            Mk[:, sl, sl] = b["M"]
        A = np.zeros((nc, nl, nl))
        A[:, :nu, :nu] = Mk
        A[:, :nu, nu:] = -self.c * b["Gp"]
        A[:, nu:, :nu] = np.transpose(b["Gp"], (0, 2, 1))
        A[:, nu:, nu:] = b["Tpp"]
        self.Ainv = np.linalg.inv(A)
        # lambda columns of the cell rows, per local facet: [-c Gl ; Tpl]
        B = np.zeros((nc, nfc, nl, nf))
        B[:, :, :nu, :] = -self.c * b["Gl"]
        B[:, :, nu:, :] = b["Tpl"]
        self.B = B
        # mu rows of the cell unknowns, per local facet: [Cl, Elp] = [-Gl^T, -Tpl^T]
        L = np.zeros((nc, nfc, nf, nl))
        L[:, :, :, :nu] = -np.transpose(b["Gl"], (0, 1, 3, 2))
        L[:, :, :, nu:] = -np.transpose(b["Tpl"], (0, 1, 3, 2))
        self.L = L
        Sk = np.einsum("kfmi,kij,kgjn->kfgmn", L, self.Ainv, B)  # (nc, nfc, nfc, nf, nf)
        Fcf = mesh.cell_facets
        rows = (Fcf[:, :, None, None, None] * nf + np.arange(nf)[None, None, None, :, None])
        cols = (Fcf[:, None, :, None, None] * nf + np.arange(nf)[None, None, None, None, :])
        rows = np.broadcast_to(rows, Sk.shape)
        cols = np.broadcast_to(cols, Sk.shape)
        S = sp.csr_matrix((Sk.ravel(), (rows.ravel(), cols.ravel())), shape=(d.nT, d.nT))
        self.S = (S - s["Fll"]).tocsr()
        self._lu = spla.splu(self.S[1:, 1:].tocsc())
        self.one_p = d.constant_pressure()
        self.one_t = d.constant_trace()

    # ----------------------------------------------------------------------
    def _cell_rhs(self, Fw, Fpsi):
        d = self.disc
        nc = d.mesh.ncells
        return np.concatenate([np.asarray(Fw).reshape(nc, d.nu), np.asarray(Fpsi).reshape(nc, d.npp)], axis=1)

    def condensed_rhs(self, Fw, Fpsi, Fmu):
        d = self.disc
        f = self._cell_rhs(Fw, Fpsi)
        y = np.einsum("kfmi,kij,kj->kfm", self.L, self.Ainv, f)
        g = np.zeros((d.mesh.nfacets, d.nf))
        np.add.at(g, d.mesh.cell_facets, y)
        return g.reshape(-1) - np.asarray(Fmu)

    def solve_trace(self, g):
        lam = np.zeros(self.S.shape[0])
        lam[1:] = self._lu.solve(g[1:])
        return lam

    def back_substitute(self, Fw, Fpsi, lam):
        d = self.disc
        f = self._cell_rhs(Fw, Fpsi)
        lk = np.asarray(lam).reshape(-1, d.nf)[d.mesh.cell_facets]  # (nc, nfc, nf)
        f = f - np.einsum("kfin,kfn->ki", self.B, lk)
        x = np.einsum("kij,kj->ki", self.Ainv, f)
        return x[:, :d.nu].reshape(-1), x[:, d.nu:].reshape(-1)

    def normalise(self, p, lam):
        """Shift (p, lambda) by a constant so that int p = 0."""
        d = self.disc
        m = d.pressure_integral(p) / d.domain_area()
        return p - m * self.one_p, lam - m * self.one_t

    def solve(self, Fw, Fpsi, Fmu):
        g = self.condensed_rhs(Fw, Fpsi, Fmu)
        lam = self.solve_trace(g)
        U, p = self.back_substitute(Fw, Fpsi, lam)
        p, lam = self.normalise(p, lam)
        return U, p, lam


def monolithic_matrix(disc, c):
    """The full (U, p, lambda) operator H_c as one sparse matrix (rows w, psi, mu)."""
    s = disc.static_operators()
    M = disc.mass()
    return sp.bmat([[M, -c * s["Gp"], -c * s["Gl"]],
                    [s["Dv"], s["Tpp"], s["Tpl"]],
                    [s["Cl"], s["Elp"], s["Fll"]]]).tocsr()


def monolithic_solve(disc, c, Fw, Fpsi, Fmu):
    """Dense least-squares solve of the full system (tiny meshes only), normalised
    to int p = 0.  Used to pin the condensed solver."""
    H = monolithic_matrix(disc, c).toarray()
    rhs = np.concatenate([Fw, Fpsi, Fmu])
    x = np.linalg.lstsq(H, rhs, rcond=None)[0]
    nQ, nP = disc.nQ, disc.nP
    U, p, lam = x[:nQ], x[nQ:nQ + nP], x[nQ + nP:]
    m = disc.pressure_integral(p) / disc.domain_area()
    return U, p - m * disc.constant_pressure(), lam - m * disc.constant_trace()
