"""Oracle pins of the passive DG tracer (Appendix "DG tracer advection").

* P_CG reproduces a field of CG_{k+1} (a global polynomial) exactly, is
  idempotent, and its output is continuous: both cells of every facet give
  the same values at the facet points, across periodic identifications too;
* a constant tracer stays constant on a periodic mesh for any velocity (the
  volume and facet terms of a(chi, 1, U) cancel exactly there);
* with a uniform velocity on the periodic square the scheme is the upwind DG
  method for linear transport, and the error against the translated exact
  profile falls at the expected rate under refinement.
"""
import numpy as np
import pytest

import hdg_inputs as hi
from oracle.forms import Discretisation
from oracle.imex import TABLEAUX
from oracle.mesh import Mesh
from oracle.tracer import CGSpace, Tracer, tracer_operator

L = 2.0 * np.pi


def _periodic(n, k, pert=0.0, seed=0):
    X, C, rep = hi.periodic_square_mesh(n, L, pert, seed)
    return Discretisation(Mesh(X, C, rep), None, k)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_cg_projection_reproduces_polynomials(k):
    X, C = hi.unit_square_mesh(4)
    X = hi.random_mesh_perturbation(X, 4, 0.2, 1)
    d = Discretisation(X, C, k)
    cg = CGSpace(d)
    Q = d.l2_project_velocity(lambda x, y: np.stack([x * x - 0.3 * y, x * y + 0.1], -1))
    assert np.abs(cg.project(Q) - Q).max() <= 1e-12


@pytest.mark.parametrize("k,periodic", [(1, False), (2, True), (3, True)])
def test_cg_projection_is_continuous_and_idempotent(k, periodic):
    if periodic:
        d = _periodic(4, k, 0.2, 3)
    else:
        X, C = hi.unit_square_mesh(4)
        d = Discretisation(hi.random_mesh_perturbation(X, 4, 0.2, 2), C, k)
    cg = CGSpace(d)
    Q = np.random.default_rng(4).standard_normal(d.nQ)
    U = cg.project(Q)
    assert np.abs(cg.project(U) - U).max() <= 1e-11 * np.abs(U).max()
    v = d.eval_cf(U)
    fc = d.mesh.facet_cells
    I = np.nonzero(d.mesh.interior)[0]
    jump = v[fc[I, 0], fc[I, 1]] - v[fc[I, 2], fc[I, 3]]
    assert np.abs(jump).max() <= 1e-11 * np.abs(v).max()
    assert np.abs(U - Q).max() > 1e-2  # a random DG field is not continuous


@pytest.mark.parametrize("k", [1, 2])
def test_constant_tracer_stays_constant_on_a_periodic_mesh(k):
    d = _periodic(4, k, 0.15, 5)
    U = CGSpace(d).project(np.random.default_rng(6).standard_normal(d.nQ))
    one = d.l2_project_pressure(lambda x, y: np.ones_like(x))
    A = tracer_operator(d, U)
    assert np.abs(A @ one).max() <= 1e-12 * abs(A).max()


def test_uniform_transport_converges():
    k, T = 1, 0.5
    a = np.array([1.0, 0.5])
    q0 = lambda x, y: np.sin(x) * np.cos(y)
    errs = []
    for n in (6, 12):
        d = _periodic(n, k)
        h = L / n
        nt = int(np.ceil(T / (0.1 * h)))
        dt = T / nt
        Q = d.l2_project_velocity(lambda x, y: np.stack([a[0] + 0 * x, a[1] + 0 * y], -1))
        tr = Tracer(d, TABLEAUX["ars222"](), dt)
        q = d.l2_project_pressure(q0)
        s = tr.tab.s
        for _ in range(nt):
            q = tr.step(q, [Q] * s)
        vals = np.einsum("qs,ks->kq", d.Vp, q.reshape(-1, d.npp))
        ex = q0(d.cx[..., 0] - a[0] * T, d.cx[..., 1] - a[1] * T)
        errs.append(np.sqrt(np.sum(d.cw * (vals - ex) ** 2)))
    rate = np.log2(errs[0] / errs[1])
    assert rate > k + 0.5, (errs, rate)
