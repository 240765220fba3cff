"""Oracle pins on doubly periodic meshes (Section "Double-layer shear flow":
periodic boundary conditions in both directions).

* topology: every facet is interior; the two sides of an identified facet
  have opposite normals, equal lengths and facet points that differ by a
  period;
* the trace operator is symmetric positive semi-definite with the constants
  as its only null space (as on the walled square);
* a uniform flow is an exact discrete steady state (it lies in the discrete
  space, its BDM projection is itself and every flux and penalty term
  vanishes), so it must survive a step to round-off; a flipped sign in the
  facet terms of the advection form breaks this;
* translation equivariance: on the uniform periodic mesh a shift of the
  data by one grid column shifts the discrete solution by one column of
  cells (a wrong identification across the boundary breaks it);
* a steady Euler solution (u = (sin x cos y, -cos x sin y)) is kept with an
  error that falls under refinement.
"""
import numpy as np
import pytest

import hdg_inputs as hi
from oracle.forms import Discretisation
from oracle.hdg import HDGSolver
from oracle.imex import IMEXHDG, ars222, ssp3_433
from oracle.mesh import Mesh

L = 2.0 * np.pi


def _disc(n, k, pert=0.0, seed=0):
    X, C, rep = hi.periodic_square_mesh(n, L, pert, seed)
    return Discretisation(Mesh(X, C, rep), None, k)


@pytest.mark.parametrize("n,pert", [(3, 0.0), (4, 0.2), (5, 0.15)])
def test_periodic_topology(n, pert):
    m = _disc(n, 1, pert).mesh
    assert m.ncells == 2 * n * n and m.nfacets == 3 * n * n
    assert m.interior.all()
    fc = m.facet_cells
    np.testing.assert_allclose(m.normal[fc[:, 0], fc[:, 1]], -m.normal[fc[:, 2], fc[:, 3]], atol=1e-14)
    np.testing.assert_allclose(m.hF_cell[fc[:, 0], fc[:, 1]], m.hF_cell[fc[:, 2], fc[:, 3]], rtol=1e-13)
    t = np.array([0.0, 0.3, 1.0])
    P = m.cell_facet_points(t)
    d = P[fc[:, 0], fc[:, 1]] - P[fc[:, 2], fc[:, 3]]  # same parameter on both sides
    shift = np.round(d / L)
    np.testing.assert_allclose(d, shift * L, atol=1e-12)
    assert np.abs(shift).max() == 1  # some facets are identified across the boundary


def test_small_periodic_mesh_is_rejected():
    with pytest.raises(ValueError):
        hi.periodic_square_mesh(2)


@pytest.mark.parametrize("k", [1, 2])
def test_periodic_trace_operator_null_space(k):
    d = _disc(3, k, 0.2)
    S = HDGSolver(d, 0.37).S
    S = S.toarray() if hasattr(S, "toarray") else np.asarray(S)
    assert np.abs(S - S.T).max() <= 1e-12 * np.abs(S).max()
    ev, V = np.linalg.eigh(S)
    tol = 1e-10 * ev[-1]
    assert ev[0] > -tol
    assert int((np.abs(ev) <= tol).sum()) == 1
    one = d.constant_trace()
    assert np.abs(S @ one).max() <= 1e-12 * np.abs(S).max() * np.abs(one).max()


@pytest.mark.parametrize("tab", [ars222, ssp3_433])
def test_uniform_flow_is_steady(tab):
    d = _disc(4, 2, 0.2, seed=3)
    st = IMEXHDG(d, 0.05, tab(), 2)
    Q0, p0, lam0 = st.initial_state(lambda x, y: np.stack([0.7 + 0 * x, -0.4 + 0 * y], -1))
    Q, p, lam = st.run(Q0, p0, lam0, 0.0, 2)
    assert np.abs(Q - Q0).max() <= 1e-12
    assert np.abs(p).max() <= 1e-11 and np.abs(lam).max() <= 1e-11


@pytest.mark.parametrize("tab,k", [(ars222, 2), (ssp3_433, 1)])
def test_translation_equivariance(tab, k):
    """On the uniform periodic mesh, shifting the initial velocity by one grid
    column shifts the discrete solution by one column of cells: the facets
    identified across the boundary act like every other facet."""
    n = 4
    d = _disc(n, k)
    h = L / n
    f = lambda x, y: hi.shear_layer_velocity(x, y, rho=0.6) + 0.3 * np.stack([np.cos(y), np.sin(2 * x)], -1)
    out = []
    for shift in (0.0, h):
        st = IMEXHDG(d, 0.05, tab(), 2)
        Q, p, lam = st.initial_state(lambda x, y: f(x - shift, y))
        Q, p, lam = st.run(Q, p, lam, 0.0, 2)
        out.append((Q.reshape(n, n, 2, -1), p.reshape(n, n, 2, -1)))  # [j][i][cell of square]
    (Q0, p0), (Q1, p1) = out
    assert np.abs(Q1 - np.roll(Q0, 1, axis=1)).max() <= 1e-11 * np.abs(Q0).max()
    assert np.abs(p1 - np.roll(p0, 1, axis=1)).max() <= 1e-10 * np.abs(p0).max()
    assert np.abs(Q1 - Q0).max() > 1e-2  # the shift is not trivial


def test_steady_vortex_error_falls():
    k, dt = 1, 0.02
    errs = []
    for n in (4, 8):
        d = _disc(n, k)
        st = IMEXHDG(d, dt, ars222(), 2)
        Q, p, lam = st.initial_state(lambda x, y: hi.steady_vortex_velocity(x, y))
        Q, p, lam = st.run(Q, p, lam, 0.0, 3)
        val, _ = d.eval_cell(Q)
        ex = hi.steady_vortex_velocity(d.cx[..., 0], d.cx[..., 1])
        errs.append(np.sqrt(np.sum(d.cw[..., None] * (val - ex) ** 2)))
    rate = np.log2(errs[0] / errs[1])
    assert rate > k - 0.3, (errs, rate)
