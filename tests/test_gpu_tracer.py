"""GPU parity of the passive DG tracer (Appendix "DG tracer advection")
through the C ABI against the oracle (oracle/tracer.py): the CG_{k+1}
projection, the transport rate, and whole IMEX steps with the tracer, on
walled and periodic perturbed meshes."""
import numpy as np
import pytest

import hdg_inputs as hi
from oracle.forms import Discretisation
from oracle.imex import IMEXHDG, TABLEAUX
from oracle.mesh import Mesh
from oracle.tracer import CGSpace, Tracer, tracer_operator

from gpu_util import context, dev, host, mesh, rel_l2_cells, torch_or_skip

pytestmark = pytest.mark.gpu


def _q0(x, y):
    return np.sin(2.0 * x + 0.3) * np.cos(1.5 * y) + 0.5


def _setup(periodic, n, k, pert, seed):
    if periodic:
        X, C, rep = hi.periodic_square_mesh(n, 2.0 * np.pi, pert, seed)
        return X, C, rep, Discretisation(Mesh(X, C, rep), None, k), hi.shear_layer_velocity
    X, C = mesh(n, pert, seed)
    par = hi.stream_function_params(seed)
    return X, C, None, Discretisation(X, C, k), lambda x, y: hi.streamfunction_velocity(par, x, y)


@pytest.mark.parametrize("periodic,n,k", [(False, 4, 1), (False, 5, 2), (True, 4, 3), (True, 3, 2)])
def test_cg_projection_and_rate(periodic, n, k):
    torch = torch_or_skip()
    X, C, rep, d, vel = _setup(periodic, n, k, 0.15, 3)
    ctx = context(X, C, vertex_rep=rep, degree=k)
    Q = np.random.default_rng(5).standard_normal(d.nQ)
    cg = CGSpace(d)
    U = cg.project(Q)
    Ug = host(ctx.cg_project(dev(torch, Q)))
    assert np.abs(Ug - U).max() <= 1e-11 * np.abs(U).max()
    q = np.random.default_rng(6).standard_normal(d.nP)
    want = Tracer(d, TABLEAUX["ars222"](), 1.0).minv(tracer_operator(d, U) @ q)
    got = host(ctx.tracer_rate(dev(torch, Q), dev(torch, q)))
    assert np.abs(got - want).max() <= 1e-10 * np.abs(want).max()


@pytest.mark.parametrize("periodic,scheme,k,dt", [(False, "ssp2_332", 2, 0.01), (True, "ssp3_433", 2, 0.02),
                                                  (False, "imex_euler", 1, 0.01)])
def test_tracer_steps(periodic, scheme, k, dt):
    torch_or_skip()
    X, C, rep, d, vel = _setup(periodic, 4, k, 0.1, 8)
    nsteps = 2
    st = IMEXHDG(d, dt, TABLEAUX[scheme](), 2)
    tr = Tracer(d, TABLEAUX[scheme](), dt)
    Q, p, lam = st.initial_state(vel)
    q = d.l2_project_pressure(_q0)
    for n in range(nsteps):
        Q, p, lam = st.step(Q, p, lam, n * dt)
        q = tr.step(q, st.last_stages)
    ctx = context(X, C, vertex_rep=rep, degree=k, imex=scheme, n_richardson=2, rtol_trace=1e-13, rtol_velocity=1e-13)
    xy = ctx.cell_points()
    ctx.set_velocity_from_points(vel(xy[..., 0], xy[..., 1]))
    ctx.set_tracer(_q0(xy[..., 0], xy[..., 1]))
    ctx.advance(dt, nsteps)
    qg = host(ctx.get_tracer())
    assert rel_l2_cells(d, qg, q, d.npp) < 1e-10
    assert rel_l2_cells(d, host(ctx.get_state()[0]), Q, d.nu) < 1e-10


def test_uniform_transport_converges_at_size():
    """At sizes the oracle does not reach: a uniform flow on the periodic
    square carries the tracer as a rigid translation; the L2 error against the
    translated profile falls under refinement (k = 2, ARS(2,2,2), CFL 0.1)."""
    torch_or_skip()
    k, T = 2, 0.5
    a = (1.0, 0.5)
    q0 = lambda x, y: np.sin(x) * np.cos(y)
    errs = []
    for n in (16, 32):
        X, C, rep = hi.periodic_square_mesh(n)
        d = Discretisation(Mesh(X, C, rep), None, k)
        nt = int(np.ceil(T / (0.1 * 2.0 * np.pi / n)))
        ctx = context(X, C, vertex_rep=rep, degree=k, imex="ars222", n_richardson=2)
        xy = ctx.cell_points()
        ctx.set_velocity_from_points(np.stack([a[0] + 0 * xy[..., 0], a[1] + 0 * xy[..., 1]], -1))
        ctx.set_tracer(q0(xy[..., 0], xy[..., 1]))
        ctx.advance(T / nt, nt)
        q = host(ctx.get_tracer())
        vals = np.einsum("qs,ks->kq", d.Vp, q.reshape(-1, d.npp))
        ex = q0(d.cx[..., 0] - a[0] * T, d.cx[..., 1] - a[1] * T)
        errs.append(np.sqrt(np.sum(d.cw * (vals - ex) ** 2)))
        ctx.close()
    rate = np.log2(errs[0] / errs[1])
    assert rate > k + 0.5, (errs, rate)
