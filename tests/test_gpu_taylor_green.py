"""GPU: the paper's Taylor-Green vortex with its forcing f = -kappa exp(-kappa t) Q0
(eq. taylor_green_Q0_f, exact solution eq. exact_solution), kappa = 0.5.

* one forced configuration against the oracle, element by element;
* the convergence study of Section "Convergence" on the GPU: T = 1, n_t = n
  time steps on the n x n grid (Table "stepsizes"), IMEX Euler with k = 1,
  SSP2(3,3,2) with k = 2 and SSP3(4,3,3) with k = 3 (pairings of the
  paper's experiments), n_R = 2; the
  velocity and pressure errors must fall at least at the rate h^k the paper
  reports.
"""
import numpy as np
import pytest

import hdg_inputs as hi
from oracle.forms import Discretisation
from oracle.imex import IMEXHDG, TABLEAUX

from gpu_util import context, host, mesh, rel_l2_cells, rel_l2_trace, torch_or_skip

pytestmark = pytest.mark.gpu

KAPPA = 0.5


def _forced_context(X, C, k, scheme, nR, **kw):
    ctx = context(X, C, degree=k, imex=scheme, n_richardson=nR, rtol_trace=1e-13, rtol_velocity=1e-13, **kw)
    cp, fp = ctx.cell_points(), ctx.facet_points()
    ctx.set_forcing(hi.taylor_green_forcing(cp[..., 0], cp[..., 1], 0.0, KAPPA),
                    hi.taylor_green_forcing(fp[..., 0], fp[..., 1], 0.0, KAPPA), KAPPA)
    ctx.set_velocity_from_points(hi.taylor_green_velocity(cp[..., 0], cp[..., 1], 0.0, KAPPA))
    return ctx


@pytest.mark.parametrize("scheme,k", [("ssp2_332", 2), ("ars222", 1), ("ssp3_433", 3)])
def test_forced_steps_parity(scheme, k):
    torch_or_skip()
    X, C = mesh(4, 0.15)
    d = Discretisation(X, C, k)
    dt, nsteps = 0.125, 2
    forcing = lambda x, y, t: hi.taylor_green_forcing(x, y, t, KAPPA)
    st = IMEXHDG(d, dt, TABLEAUX[scheme](), 2, forcing=forcing)
    Q, p, lam = st.initial_state(lambda x, y: hi.taylor_green_velocity(x, y, 0.0, KAPPA))
    Q, p, lam = st.run(Q, p, lam, 0.0, nsteps)
    ctx = _forced_context(X, C, k, scheme, 2)
    ctx.advance(dt, nsteps)
    assert abs(ctx.time - nsteps * dt) < 1e-15
    got = [host(t) for t in ctx.get_state()]
    errs = (rel_l2_cells(d, got[0], Q, d.nu), rel_l2_cells(d, got[1], p, d.npp), rel_l2_trace(d, got[2], lam))
    print(f"{scheme} k={k}: rel L2 Q {errs[0]:.2e} p {errs[1]:.2e} lam {errs[2]:.2e}")
    assert max(errs) < 1e-10, errs


def _errors(d, Q, p, t):
    val, _ = d.eval_cell(Q)
    ex = hi.taylor_green_velocity(d.cx[..., 0], d.cx[..., 1], t, KAPPA)
    eq = np.sqrt(np.sum(d.cw[..., None] * (val - ex) ** 2))
    pv = np.einsum("qs,ks->kq", d.Vp, p.reshape(-1, d.npp))
    ep = np.sqrt(np.sum(d.cw * (pv - hi.taylor_green_pressure(d.cx[..., 0], d.cx[..., 1], t, KAPPA)) ** 2))
    return eq, ep


@pytest.mark.parametrize("scheme,k,ns", [("imex_euler", 1, (4, 8, 16, 32)), ("ssp2_332", 2, (4, 8, 16)),
                                         ("ssp3_433", 3, (4, 8, 16))])
def test_convergence(scheme, k, ns):
    torch_or_skip()
    T = 1.0
    errs = []
    for n in ns:
        X, C = hi.unit_square_mesh(n)
        d = Discretisation(X, C, k)
        ctx = _forced_context(X, C, k, scheme, 2)
        ctx.advance(T / n, n)
        Q, p, _ = (host(t) for t in ctx.get_state())
        errs.append(_errors(d, Q, p, T))
        ctx.close()
    errs = np.array(errs)
    rates = np.log2(errs[:-1] / errs[1:])
    print(scheme, k, "errors", errs.tolist(), "rates", rates.tolist())
    assert rates[:, 0].min() > k - 0.3, (errs, rates)
    assert rates[:, 1].min() > k - 0.3, (errs, rates)
