"""Pins of the oracle's IMEX-HDG time stepping (CPU only).

P9:  tableau order conditions (including the IMEX coupling conditions), and
     the observed order of the stage-residual recursion on a scalar linear
     ODE with explicit forcing.
P10: after a step, Gamma(psi, mu, Q^{n+1}, dp, dlambda) = 0: the hybridised
     normal flux is single-valued and divergence-free cell by cell.
P11: zero forcing: the kinetic energy never increases (upwind and penalty
     terms only dissipate).
P12: Taylor-Green vortex: the velocity error decreases under refinement with
     dt ~ h at least at the rate the paper reports (h^k); the reconstructed
     pressure of the exact velocity converges to the exact pressure.
P13: a zero state with zero forcing stays exactly zero.
"""
import itertools

import numpy as np
import pytest

import hdg_inputs as hi
from oracle.forms import Discretisation
from oracle.imex import IMEXHDG, TABLEAUX, ars222, ars233, final_residual, imex_euler, ssp3_433, stage_residual


def _conds(tab):
    Ae, be, Ai, bi = tab.Aex, tab.bex, tab.Aim, tab.bim
    ce, ci = Ae.sum(1), Ai.sum(1)
    return Ae, be, ce, Ai, bi, ci


@pytest.mark.parametrize("name,order", [("imex_euler", 1), ("ars222", 2), ("ars233", 3)])
def test_p9_order_conditions(name, order):
    tab = TABLEAUX[name]()
    Ae, be, ce, Ai, bi, ci = _conds(tab)
    # the paper's structural assumptions: explicit tableau strictly lower
    # triangular, implicit first column and b_0^im zero
    assert np.allclose(np.triu(Ae), 0) and np.allclose(Ai[:, 0], 0) and bi[0] == 0
    assert np.allclose(ce, ci)
    assert abs(be.sum() - 1) < 1e-15 and abs(bi.sum() - 1) < 1e-15
    if order >= 2:
        for b, c in itertools.product((be, bi), (ce, ci)):
            assert abs(b @ c - 0.5) < 1e-15
    if order >= 3:
        for b, c in itertools.product((be, bi), (ce, ci)):
            assert abs(b @ c**2 - 1 / 3) < 1e-15
        for b, A, c in itertools.product((be, bi), (Ae, Ai), (ce, ci)):
            assert abs(b @ A @ c - 1 / 6) < 1e-15


@pytest.mark.parametrize("name,stages", [("ssp2_332", 4), ("ssp3_433", 4)])
def test_p9_ssp_order_conditions(name, stages):
    """The paper's SSP tableaux in its form (stage 0 = Q^n, zero first
    implicit column): SSP2(3,3,2) with an explicit stage in front of its
    printed stages, SSP3(4,3,3) as printed through Algorithm 1 (first
    implicit column unused).  Both satisfy every second-order condition,
    coupling conditions with the different explicit and implicit abscissae
    included; for SSP3(4,3,3) that holds only because the printed beta is
    alpha/4 to the 14 printed digits (hence the tolerance).  Neither reading
    meets the third-order conditions."""
    tab = TABLEAUX[name]()
    assert tab.s == stages
    Ae, be, ce, Ai, bi, ci = _conds(tab)
    assert np.allclose(np.triu(Ae), 0) and np.allclose(Ai[:, 0], 0) and bi[0] == 0
    assert np.allclose(Ai[0], 0) and np.all(np.diag(Ai)[1:] > 0)
    tol = 1e-13
    assert abs(be.sum() - 1) < tol and abs(bi.sum() - 1) < tol
    for b, c in itertools.product((be, bi), (ce, ci)):
        assert abs(b @ c - 0.5) < tol
    third = [abs(b @ c**2 - 1 / 3) for b, c in itertools.product((be, bi), (ce, ci))]
    third += [abs(b @ A @ c - 1 / 6) for b, A, c in itertools.product((be, bi), (Ae, Ai), (ce, ci))]
    assert max(third) > 1e-3


@pytest.mark.parametrize("name,step1,hdg", [("imex_euler", 2, 4), ("ssp3_433", 6, 8)])
def test_solve_counts_match_the_timing_tables(name, step1, hdg):
    """With n_R = 2 an s-stage scheme makes n_R (s-1) Step I solves and
    n_R (s-1) + 2 mixed solves per step; the paper's timing tables list 2 / 4
    for IMEX Euler and 6 / 8 for SSP3(4,3,3)."""
    s = TABLEAUX[name]().s
    assert 2 * (s - 1) == step1 and 2 * (s - 1) + 2 == hdg


@pytest.mark.parametrize("name,order", [("imex_euler", 1), ("ars222", 2), ("ars233", 3), ("ssp2_332", 2),
                                        ("ssp3_433", 2)])
def test_p9_scalar_ode_order(name, order):
    """y' = lam y + g(t), lam implicit, g explicit; exact y = 1 + sin t."""
    tab = TABLEAUX[name]()
    lam = -2.0
    g = lambda t: np.cos(t) - lam * (1.0 + np.sin(t))
    errs = []
    for nt in (20, 40, 80):
        dt = 1.0 / nt
        y, t = 1.0, 0.0
        for _ in range(nt):
            MQn = np.array([y])
            fex = [np.array([g(t + tab.c[j] * dt)]) for j in range(tab.s)]
            MQ, r = [MQn] + [None] * (tab.s - 1), [None] * tab.s
            for i in range(1, tab.s):
                r[i] = stage_residual(tab, i, MQn, MQ, r, fex, dt)
                MQ[i] = r[i] / (1.0 - dt * tab.Aim[i, i] * lam)
            y = float(final_residual(tab, MQn, MQ, r, fex, dt)[0])
            t += dt
        errs.append(abs(y - (1.0 + np.sin(1.0))))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates.min() > order - 0.15, rates


def _cfg(n, k, seed=0, dt=1e-3, tab=None, nR=3):
    X, C = hi.unit_square_mesh(n)
    d = Discretisation(X, C, k)
    st = IMEXHDG(d, dt, tab or ars222(), nR)
    par = hi.stream_function_params(seed)
    Q, p, lam = st.initial_state(lambda x, y: hi.streamfunction_velocity(par, x, y))
    return d, st, Q, p, lam


@pytest.mark.parametrize("n,k", [(8, 1), (6, 3)])
def test_p10_p11_constraint_and_energy(n, k):
    d, st, Q, p, lam = _cfg(n, k, dt=2e-3)
    ke = [d.kinetic_energy(Q)]
    t = 0.0
    for _ in range(4):
        Q, p, lam = st.step(Q, p, lam, t)
        t += st.dt
        dp, dl = st.last_final
        gp, gm = d.gamma(Q, dp, dl)
        ops = d.static_operators()
        # backward-error scale: |operator| |argument| of the largest term
        scale = max(abs(ops["Dv"]).sum(axis=1).max() * np.abs(Q).max(),
                    abs(ops["Cl"]).sum(axis=1).max() * np.abs(Q).max(),
                    abs(ops["Tpl"]).sum(axis=1).max() * np.abs(dl).max())
        assert np.abs(gp).max() < 1e-12 * scale
        assert np.abs(gm).max() < 1e-12 * scale
        ke.append(d.kinetic_energy(Q))
        assert abs(d.pressure_integral(p)) < 1e-12
    assert np.all(np.diff(ke) <= 1e-12 * ke[0]), ke


@pytest.mark.slow
def test_p11_config1_energy_decreases():
    """The small parity workload: n=16, k=1, ARS(2,2,2), dt=1e-3, 10 steps, n_R=3."""
    d, st, Q, p, lam = _cfg(16, 1)
    ke = [d.kinetic_energy(Q)]
    for s in range(10):
        Q, p, lam = st.step(Q, p, lam, s * 1e-3)
        ke.append(d.kinetic_energy(Q))
    assert np.all(np.diff(ke) < 0)


def test_p13_zero_state_stays_zero():
    X, C = hi.unit_square_mesh(4)
    d = Discretisation(X, C, 2)
    st = IMEXHDG(d, 1e-2, ars233(), 2)
    Q, p, lam = np.zeros(d.nQ), np.zeros(d.nP), np.zeros(d.nT)
    Q, p, lam = st.step(Q, p, lam, 0.0)
    assert not Q.any() and not p.any() and not lam.any()


def _tg_errors(d, Q, p, t):
    val, _ = d.eval_cell(Q)
    ex = hi.taylor_green_velocity(d.cx[..., 0], d.cx[..., 1], t)
    eq = np.sqrt(np.sum(d.cw[..., None] * (val - ex) ** 2))
    pv = np.einsum("qs,ks->kq", d.Vp, p.reshape(-1, d.npp))
    ep = np.sqrt(np.sum(d.cw * (pv - hi.taylor_green_pressure(d.cx[..., 0], d.cx[..., 1], t)) ** 2))
    return eq, ep


@pytest.mark.parametrize("tab,k,ns,minrate", [(imex_euler, 1, (4, 8, 16), 0.8), (ars222, 2, (4, 8), 2.0),
                                              (ssp3_433, 2, (4, 8), 2.0)])
def test_p12_taylor_green_convergence(tab, k, ns, minrate):
    T = 0.5
    errs = []
    for n in ns:
        X, C = hi.unit_square_mesh(n)
        d = Discretisation(X, C, k)
        nt = n // 2
        st = IMEXHDG(d, T / nt, tab(), 2, forcing=hi.taylor_green_forcing)
        Q, p, lam = st.initial_state(lambda x, y: hi.taylor_green_velocity(x, y, 0.0))
        Q, p, lam = st.run(Q, p, lam, 0.0, nt)
        errs.append(_tg_errors(d, Q, p, T))
    errs = np.array(errs)
    rates = np.log2(errs[:-1] / errs[1:])
    assert rates[:, 0].min() > minrate, rates
    assert rates[:, 1].min() > minrate, rates


@pytest.mark.parametrize("k", [1, 2])
def test_p12_pressure_reconstruction_of_exact_velocity(k):
    errs = []
    for n in (4, 8, 16):
        X, C = hi.unit_square_mesh(n)
        d = Discretisation(X, C, k)
        st = IMEXHDG(d, 0.1, imex_euler(), 1, forcing=hi.taylor_green_forcing)
        Q, p, lam = st.initial_state(lambda x, y: hi.taylor_green_velocity(x, y, 0.0))
        errs.append(_tg_errors(d, Q, p, 0.0)[1])
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates.min() > k + 0.5, rates


def _stage_problem(n, k, dt, seed=2, amp=3.0):
    """A stage of ARS(2,2,2) on a perturbed n x n mesh: the data of Algorithm 2
    and the monolithic solution of eqs. (imex_implicit_solve) and
    (imex_implicit_solve_constraint), by a dense least-squares solve of the
    full (Q, p, lambda) system (its null space is the constant (p, lambda))."""
    import scipy.sparse as sp
    X, C = hi.unit_square_mesh(n)
    X = hi.random_mesh_perturbation(X, n, 0.1, 1)
    d = Discretisation(X, C, k)
    par = hi.stream_function_params(seed)
    Q0 = d.l2_project_velocity(lambda x, y: amp * hi.streamfunction_velocity(par, x, y))
    st = IMEXHDG(d, dt, ars222(), 1)
    p0, l0 = st.reconstruct(Q0, 0.0)
    Qs = d.bdm_project(Q0)
    a = ars222().Aim[1, 1]
    adt = a * dt
    r = d.mass() @ Q0
    s = d.static_operators()
    A = d.mass() - adt * d.advection(Qs)
    H = sp.bmat([[A, -adt * s["Gp"], -adt * s["Gl"]], [s["Dv"], s["Tpp"], s["Tpl"]],
                 [s["Cl"], s["Elp"], s["Fll"]]]).toarray()
    x = np.linalg.lstsq(H, np.concatenate([r, np.zeros(d.nP + d.nT)]), rcond=None)[0]
    return d, (r, a, Qs, Q0, p0, l0), x[:d.nQ]


@pytest.mark.parametrize("n,k", [(3, 1), (2, 2)])
def test_p14_reading_b_converges_to_the_monolithic_stage_solve(n, k):
    """P14: with Step II read as the mixed solve of the stage operator H_{a dt}
    with the constraint residual of the iterate (reading B), the Richardson
    iterates converge to the monolithic solution of the stage equations as
    n_R grows, and the limit satisfies the constraint Gamma = 0; the printed
    Step II (reading A) settles elsewhere: it never removes the constraint
    residual of the iterate."""
    d, (r, a, Qs, Q0, p0, l0), Qm = _stage_problem(n, k, 5e-3)
    errs = {}
    for reading in ("A", "B"):
        errs[reading] = []
        for nR in (2, 8, 32):
            st = IMEXHDG(d, 5e-3, ars222(), nR, step2_reading=reading)
            Q, p, lam = st.richardson(r, a, Qs, Q0, p0, l0)
            errs[reading].append(np.linalg.norm(Q - Qm) / np.linalg.norm(Qm))
            if reading == "B" and nR == 32:
                gpsi, gmu = d.gamma(Q, p, lam)
                scale = np.linalg.norm(np.concatenate(d.gamma(Q, 0 * p, 0 * lam)))
                assert np.linalg.norm(np.concatenate([gpsi, gmu])) <= 1e-10 * scale
    eb, ea = errs["B"], errs["A"]
    assert eb[0] > eb[1] > eb[2] and eb[2] < 1e-9, eb
    assert min(ea) > 1e-3, ea          # a different fixed point
    assert abs(ea[2] - ea[1]) < 1e-3 * ea[2]  # ... which reading A does reach


def test_reading_b_step_is_a_step():
    """Reading B on whole steps: the final projection leaves Gamma(Q^{n+1}) = 0
    (P10) and the zero state stays zero (P13)."""
    X, C = hi.unit_square_mesh(3)
    d = Discretisation(X, C, 2)
    par = hi.stream_function_params(0)
    st = IMEXHDG(d, 1e-3, ars222(), 2, step2_reading="B")
    Q, p, lam = st.initial_state(lambda x, y: hi.streamfunction_velocity(par, x, y))
    Q1, p1, l1 = st.step(Q, p, lam, 0.0)
    dp, dl = st.last_final
    gpsi, gmu = d.gamma(Q1, dp, dl)
    assert np.linalg.norm(np.concatenate([gpsi, gmu])) <= 1e-11 * np.linalg.norm(d.mass() @ Q1)
    z = np.zeros(d.nQ)
    Qz, pz, lz = st.step(z, np.zeros(d.nP), np.zeros(d.nT), 0.0)
    assert np.abs(Qz).max() == 0.0 and np.abs(pz).max() == 0.0
    # The readings give different steps: the state's (p, lambda) come from the
    # pressure reconstruction, which does not make Gamma(Q, p, lambda) vanish
    # (Gamma holds tau (p - lambda) terms), and reading B removes that
    # residual in its first iteration while reading A never sees it.
    st_a = IMEXHDG(d, 1e-3, ars222(), 2)
    Qa, _, _ = st_a.step(Q, p, lam, 0.0)
    assert np.linalg.norm(np.concatenate(d.gamma(Q, p, lam))) > 1e-3 * np.linalg.norm(d.mass() @ Q)
    assert np.linalg.norm(Qa - Q1) > 1e-6 * np.linalg.norm(Q1)
