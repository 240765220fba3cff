"""IMEX-HDG time stepping (oracle side; test infrastructure).

* Butcher tableaux in the paper's form (Appendix A): s stages, implicit
  tableau with a zero first column (a^im_{i,0} = b^im_0 = 0).  IMEX Euler,
  SSP2(3,3,2) and SSP3(4,3,3) are printed in the paper; the SSP ones have
  nonzero entries in the first implicit column, which Algorithm 1 never
  uses (Q_0 = Q^n, implicit sums from j = 1).  SSP3(4,3,3) is taken as
  printed through Algorithm 1 (its dropped first column carries b^im_0 = 0;
  3 implicit stages, the solve counts of the paper's timing table);
  SSP2(3,3,2) would lose the implicit weight b^im_0 = 1/3 that way, so its
  printed stages all become implicit stages after an explicit stage 0.
  ARS(2,2,2) and ARS(2,3,3) are the Ascher-Ruuth-Spiteri schemes the paper
  cites; their coefficients are not printed there.  All are pinned by order
  conditions in the tests.
* ``stage_residual`` / ``final_residual``: eqs. (imex_residual) and
  (final_residual), the recursion that replaces f_im(Q_j) by
  (M Q_j - r_j) / a_jj.
* ``IMEXHDG.richardson``: Algorithm 2 (Steps I-III), with the weak divergence
  as the right-hand side of the psi-equation of Step II (the printed Step II
  puts it on the w-line with swapped test functions; the mixed-Poisson reading
  delta Q + grad p = 0, div delta Q = b fixes it to the psi-equation).  This
  is reading A of Step II.  Reading B (``step2_reading="B"``) replaces Step II
  and Step III by the mixed solve of the stage's own operator H_{a_ii dt}
  with w-data (Qbar, w) and constraint data -Gamma(psi, mu, Q, p, lambda) of
  the current iterate, then adds its solution (U, dp, dlambda) to the iterate:
  a fixed point has U = 0, so Qbar = 0, delta r = 0 and Gamma = 0, which are
  eqs. (imex_implicit_solve) and (imex_implicit_solve_constraint); the printed
  Step II uses H_1 and no constraint residual, so its fixed point is only
  close to the stage solution.
* ``IMEXHDG.step``: Algorithm 1; the final projection uses c = dt b^im_{s-1}
  (Algorithm 1 prints b^im, eq. (Q_nplus1_equation) prints b^ex; b^ex_{s-1}
  vanishes for the schemes used, which would make the system singular).
* ``IMEXHDG.reconstruct``: eq. (pressure_reconstruction_compact) with
  f_p = -f + (Q.grad_h)Q.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse.linalg as spla

from .hdg import HDGSolver


@dataclass(frozen=True)
class Tableau:
    name: str
    Aex: np.ndarray
    bex: np.ndarray
    Aim: np.ndarray
    bim: np.ndarray

    @property
    def s(self) -> int:
        return self.Aex.shape[0]

    @property
    def c(self) -> np.ndarray:
        return self.Aex.sum(axis=1)


def imex_euler() -> Tableau:
    return Tableau("imex_euler",
                   np.array([[0.0, 0.0], [1.0, 0.0]]), np.array([1.0, 0.0]),
                   np.array([[0.0, 0.0], [0.0, 1.0]]), np.array([0.0, 1.0]))


def ars222() -> Tableau:
    g = 1.0 - 1.0 / np.sqrt(2.0)
    d = 1.0 - 1.0 / (2.0 * g)
    return Tableau("ars222",
                   np.array([[0.0, 0.0, 0.0], [g, 0.0, 0.0], [d, 1.0 - d, 0.0]]),
                   np.array([d, 1.0 - d, 0.0]),
                   np.array([[0.0, 0.0, 0.0], [0.0, g, 0.0], [0.0, 1.0 - g, g]]),
                   np.array([0.0, 1.0 - g, g]))


def ars233() -> Tableau:
    g = (3.0 + np.sqrt(3.0)) / 6.0
    return Tableau("ars233",
                   np.array([[0.0, 0.0, 0.0], [g, 0.0, 0.0], [g - 1.0, 2.0 * (1.0 - g), 0.0]]),
                   np.array([0.0, 0.5, 0.5]),
                   np.array([[0.0, 0.0, 0.0], [0.0, g, 0.0], [0.0, 1.0 - 2.0 * g, g]]),
                   np.array([0.0, 0.5, 0.5]))


def _pad_explicit_stage0(name, Ae, be, Ai, bi) -> Tableau:
    """The paper's SSP tableaux (Appendix A) start with an implicit stage,
    against its form a^im_{i,0} = b^im_0 = 0.  Reading: an explicit stage 0
    (Q_0 = Q^n) goes in front and the printed tableau becomes rows and
    columns 1..s-1, so every printed implicit stage is solved."""
    m = Ae.shape[0]
    pad = lambda A: np.pad(A, ((1, 0), (1, 0)))
    return Tableau(name, pad(Ae), np.concatenate([[0.0], be]), pad(Ai), np.concatenate([[0.0], bi]))


def ssp2_332() -> Tableau:
    """SSP2(3,3,2) as printed (Appendix A); the printed abscissae (0, 1, 1/2)
    are not the row sums of the printed explicit tableau, which are used."""
    h, t = 0.5, 1.0 / 3.0
    Ae = np.array([[0.0, 0.0, 0.0], [h, 0.0, 0.0], [h, h, 0.0]])
    Ai = np.array([[0.25, 0.0, 0.0], [0.0, 0.25, 0.0], [t, t, t]])
    return _pad_explicit_stage0("ssp2_332", Ae, np.array([t, t, t]), Ai, np.array([t, t, t]))


def ssp3_433() -> Tableau:
    """SSP3(4,3,3) as printed (Appendix A), read through Algorithm 1: s = 4,
    stage 0 is Q^n, and the printed first implicit column (alpha, -alpha, 0,
    beta), which Algorithm 1 does not use, is left out (its weight b^im_0 is
    zero).  Stages 1..3 are implicit with diagonal alpha."""
    a, b, e = 0.24169426078821, 0.06042356519705, 0.12915286960590
    d = 0.5 - a - b - e
    Ae = np.array([[0.0, 0.0, 0.0, 0.0], [0.0, 0.0, 0.0, 0.0], [0.0, 1.0, 0.0, 0.0], [0.0, 0.25, 0.25, 0.0]])
    Ai = np.array([[a, 0.0, 0.0, 0.0], [-a, a, 0.0, 0.0], [0.0, 1.0 - a, a, 0.0], [b, e, d, a]])
    w = np.array([0.0, 1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0])
    Ai[:, 0] = 0.0  # unused by Algorithm 1
    return Tableau("ssp3_433", Ae, w, Ai, w)


TABLEAUX = {"imex_euler": imex_euler, "ars222": ars222, "ars233": ars233, "ssp2_332": ssp2_332,
            "ssp3_433": ssp3_433}


def stage_residual(tab: Tableau, i: int, MQn, MQ, r, fex, dt):
    """r_i = M Q^n + sum_{j=1}^{i-1} a_ij/a_jj (M Q_j - r_j) + dt sum_{j=0}^{i-1} a^ex_ij f^ex_j.

    MQ, r: lists indexed by stage (entry 0 unused); fex: list of explicit
    forcing duals f^ex(t^n + c_j dt), or None for zero forcing."""
    out = MQn.copy()
    for j in range(1, i):
        out = out + tab.Aim[i, j] / tab.Aim[j, j] * (MQ[j] - r[j])
    if fex is not None:
        for j in range(0, i):
            out = out + dt * tab.Aex[i, j] * fex[j]
    return out


def final_residual(tab: Tableau, MQn, MQ, r, fex, dt):
    """r^{n+1} = M Q^n + sum_i b^im_i/a_ii (M Q_i - r_i) + dt sum_i b^ex_i f^ex_i."""
    out = MQn.copy()
    for i in range(1, tab.s):
        out = out + tab.bim[i] / tab.Aim[i, i] * (MQ[i] - r[i])
    if fex is not None:
        for i in range(tab.s):
            out = out + dt * tab.bex[i] * fex[i]
    return out


class IMEXHDG:
    def __init__(self, disc, dt: float, tableau: Tableau, n_richardson: int = 3,
                 forcing=None, pressure_update: str = "reconstruct", step2_reading: str = "A"):
        self.disc = disc
        self.dt = float(dt)
        self.tab = tableau
        self.nR = int(n_richardson)
        self.forcing = forcing  # callable f(x, y[, z], t) -> (..., d), or None
        if pressure_update not in ("reconstruct", "first_order"):
            raise ValueError(pressure_update)
        self.pressure_update = pressure_update
        if step2_reading not in ("A", "B"):
            raise ValueError(step2_reading)
        self.step2_reading = step2_reading
        self._stage_solvers = {}  # reading B: H_c per stage coefficient c = a_ii dt
        self.M = disc.mass()
        self.ops = disc.static_operators()
        self.hdg1 = HDGSolver(disc, 1.0)
        self.hdg_final = HDGSolver(disc, self.dt * tableau.bim[-1])
        self.log = []

    # ------------------------------------------------------------------
    def forcing_dual(self, t):
        """f^ex(w; t) = (w . f(t))_Omega as a dual vector (eq. f_expl)."""
        d = self.disc
        vals = self.forcing(*np.moveaxis(d.cx, -1, 0), t)
        return np.einsum("kq,qi,kqc->kci", d.cw, d.Vu, vals).reshape(-1)

    def reconstruct(self, Q, t):
        """Pressure reconstruction: mixed problem with psi-data Div(psi, f_p) and
        wall data -<mu n.f>; returns (p, lambda) with int p = 0."""
        d = self.disc
        cell, fac = d.convection_points(Q)
        if self.forcing is not None:
            fcell = self.forcing(*np.moveaxis(d.cx, -1, 0), t)
            ffac = self.forcing(*np.moveaxis(d.cf_x, -1, 0), t)
            cell = cell - fcell
            fac = fac - ffac
            Fmu = d.boundary_normal_flux(ffac)
        else:
            Fmu = np.zeros(d.nT)
        Fpsi = d.div_c_points(cell, fac)
        _, p, lam = self.hdg1.solve(np.zeros(d.nQ), Fpsi, Fmu)
        return p, lam

    def initial_state(self, velocity_fun, t: float = 0.0):
        Q = self.disc.l2_project_velocity(velocity_fun)
        p, lam = self.reconstruct(Q, t)
        return Q, p, lam

    # ------------------------------------------------------------------
    def richardson(self, r_i, a_ii, Qs, Q, p, lam):
        """Algorithm 2: n_R preconditioned Richardson iterations for stage i."""
        d = self.disc
        adt = a_ii * self.dt
        A = d.advection(Qs)
        lu = spla.splu((self.M - adt * A).tocsc())
        zQ, zT = np.zeros(d.nQ), np.zeros(d.nT)
        for _ in range(self.nR):
            dr = r_i - self.M @ Q + adt * (A @ Q + d.g(p, lam))
            Qbar = lu.solve(dr)                                  # Step I
            if self.step2_reading == "A":
                Fpsi = -d.div_c(Qbar) / adt
                dQ, dp, dl = self.hdg1.solve(zQ, Fpsi, zT)        # Step II
                Q = Q + Qbar + adt * dQ                           # Step III
            else:
                if adt not in self._stage_solvers:
                    self._stage_solvers[adt] = HDGSolver(d, adt)
                gpsi, gmu = d.gamma(Q, p, lam)
                dQ, dp, dl = self._stage_solvers[adt].solve(self.M @ Qbar, -gpsi, -gmu)
                Q = Q + dQ
            p = p + dp
            lam = lam + dl
            self.log.append(dict(dr=float(np.linalg.norm(dr)), Qbar=float(np.linalg.norm(Qbar))))
        return Q, p, lam

    def step(self, Q, p, lam, t):
        """Algorithm 1: one IMEX-HDG step from (Q^n, p^n, lambda^n) at time t."""
        d, tab, dt = self.disc, self.tab, self.dt
        s = tab.s
        MQn = self.M @ Q
        fex = None
        if self.forcing is not None:
            fex = [self.forcing_dual(t + tab.c[j] * dt) for j in range(s)]
        Qs_ = [Q] + [None] * (s - 1)
        ps_ = [p] + [None] * (s - 1)
        ls_ = [lam] + [None] * (s - 1)
        MQ = [MQn] + [None] * (s - 1)
        r = [None] * s
        for i in range(1, s):
            r[i] = stage_residual(tab, i, MQn, MQ, r, fex, dt)
            Qstar = d.bdm_project(Qs_[i - 1])
            Qs_[i], ps_[i], ls_[i] = self.richardson(r[i], tab.Aim[i, i], Qstar, Qs_[i - 1], ps_[i - 1], ls_[i - 1])
            MQ[i] = self.M @ Qs_[i]
        rn = final_residual(tab, MQn, MQ, r, fex, dt)
        Qn, dp, dl = self.hdg_final.solve(rn, np.zeros(d.nP), np.zeros(d.nT))
        if self.pressure_update == "reconstruct":
            pn, ln = self.reconstruct(Qn, t + dt)
        else:
            pn, ln = self.hdg1.normalise(ps_[-1] + dp, ls_[-1] + dl)
        self.last_final = (dp, dl)
        self.last_stages = Qs_  # stage velocities Q_0 = Q^n, ..., Q_{s-1} (the tracer transport uses them)
        return Qn, pn, ln

    def run(self, Q, p, lam, t0, nsteps, callback=None):
        t = t0
        for n in range(nsteps):
            Q, p, lam = self.step(Q, p, lam, t)
            t += self.dt
            if callback is not None:
                callback(n + 1, t, Q, p, lam)
        return Q, p, lam
