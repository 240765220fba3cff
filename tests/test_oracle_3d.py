"""Pins of the three-dimensional oracle (tetrahedra; CPU only).

The paper states the discretisation for d = 2 and 3 (Sections "Discontinuous
Galerkin spaces", "Hybridisation") and computes in 2D only, so nothing here is
a printed 3D number; every pin is a closed form, an exactness statement or an
invariant of the method:

* unknown counts: nu = 3 C(k+4, 3), np = C(k+3, 3), nf = C(k+2, 2); the Kuhn
  mesh of n^3 cubes has 6 n^3 cells and 12 n^3 + 6 n^2 facets, 12 n^2 of
  them on the walls;
* quadrature: the collapsed rule integrates every monomial of total degree
  <= 2n - 1 to a! b! c! / (a + b + c + 3)!, and not every one of degree 2n;
* bases: orthonormal under an independent, higher rule; they span P_m;
* mesh: conforming (every interior facet seen by two cells at the same
  physical points with opposite normals), volumes add up to 1;
* P3 (condensed = full solve), P4 (trace operator SPD, constant null space),
  P5a (patch test), P6 (Div(1, .) = 0), P7 (BDM invariants), P8 (label swap),
  the f_im energy identity and the closed form of a constant field, a
  polynomial divergence-free field, and one IMEX step (constraint, energy).
"""
import math

import numpy as np
import pytest

import hdg_inputs as hi
from oracle.forms3d import Discretisation3D
from oracle.hdg import HDGSolver, monolithic_matrix, monolithic_solve
from oracle.imex import IMEXHDG, ars233
from oracle.quadrature import triangle_rule
from oracle.tet import OrthoBasis, TetMesh, monomial_exponents, tet_rule


def _disc(n, k, pert=0.0, seed=0, cells_reversed=False):
    X, C = hi.unit_cube_mesh(n)
    if pert:
        X = hi.random_cube_perturbation(X, n, pert, seed)
    if cells_reversed:
        C = C[::-1].copy()
    return Discretisation3D(X, C, k)


# ------------------------------------------------------------ closed forms

@pytest.mark.parametrize("k", [1, 2, 3])
def test_unknown_counts(k):
    X, C = hi.unit_cube_mesh(1)
    d = Discretisation3D(X, C, k)
    assert d.nu == 3 * math.comb(k + 4, 3)
    assert d.npp == math.comb(k + 3, 3)
    assert d.nf == math.comb(k + 2, 2)
    assert d.nu + d.npp == d.Vu.shape[1] * 3 + d.Vp.shape[1]


@pytest.mark.parametrize("n", [1, 2, 3])
def test_kuhn_mesh_counts_and_conformity(n):
    X, C = hi.unit_cube_mesh(n)
    m = TetMesh(X, C)
    assert m.ncells == 6 * n**3
    assert m.nfacets == 12 * n**3 + 6 * n**2
    assert int((~m.interior).sum()) == 12 * n**2
    assert abs(m.absdet.sum() / 6.0 - 1.0) < 1e-13
    I = np.nonzero(m.interior)[0]
    fc = m.facet_cells
    assert np.allclose(m.normal[fc[I, 0], fc[I, 1]], -m.normal[fc[I, 2], fc[I, 3]], atol=1e-14)
    # every wall facet lies in a face of the cube and points out of it
    B = np.nonzero(~m.interior)[0]
    nb = m.normal[fc[B, 0], fc[B, 1]]
    assert np.allclose(np.abs(nb).max(axis=1), 1.0)
    # the kth facet is the one opposite vertex k of each of its cells
    for s in (0, 2):
        K, f = fc[I, s], fc[I, s + 1]
        opp = C[K, f]
        assert np.all(np.all(m.facets[I] != opp[:, None], axis=1))


def test_config5_sizes():
    """The 32^3 Kuhn workload at k = 2, from the closed forms."""
    n, k = 32, 2
    nc, nF = 6 * n**3, 12 * n**3 + 6 * n**2
    assert nc == 196608
    assert nF * math.comb(k + 2, 2) == 2396160
    assert nc * (3 * math.comb(k + 4, 3) + math.comb(k + 3, 3)) == 196608 * 70


@pytest.mark.parametrize("npts", [1, 2, 3, 4, 5])
def test_tet_rule_exactness(npts):
    p, w = tet_rule(npts)
    worst = 0.0
    for e in monomial_exponents(2 * npts - 1, 3):
        exact = math.factorial(e[0]) * math.factorial(e[1]) * math.factorial(e[2]) / math.factorial(sum(e) + 3)
        worst = max(worst, abs(np.sum(w * np.prod(p ** np.array(e), axis=1)) - exact))
    assert worst < 1e-15
    # and degree 2n is not integrated exactly by every monomial
    bad = 0.0
    for e in monomial_exponents(2 * npts, 3):
        if sum(e) < 2 * npts:
            continue
        exact = math.factorial(e[0]) * math.factorial(e[1]) * math.factorial(e[2]) / math.factorial(sum(e) + 3)
        bad = max(bad, abs(np.sum(w * np.prod(p ** np.array(e), axis=1)) - exact))
    assert bad > 1e-8


@pytest.mark.parametrize("m,d", [(1, 3), (3, 3), (4, 3), (2, 2), (3, 2)])
def test_orthonormal_bases(m, d):
    scale = 2.0 if d == 2 else 1.0
    B = OrthoBasis(m, d, scale=scale)
    pts, w = (tet_rule(m + 4) if d == 3 else triangle_rule(m + 4))
    V = B.eval(pts)
    assert V.shape[1] == math.comb(m + d, d)
    assert np.abs(V.T @ ((w * scale)[:, None] * V) - np.eye(V.shape[1])).max() < 1e-12
    # spans P_m: every monomial of degree <= m is reproduced from its projection
    for e in monomial_exponents(m, d):
        f = np.prod(pts ** np.array(e), axis=1)
        c = V.T @ (w * scale * f)
        assert np.abs(V @ c - f).max() < 1e-11


def test_facet_points_coincide_from_both_sides():
    d = _disc(2, 2, 0.1, 3)
    m = d.mesh
    I = np.nonzero(m.interior)[0]
    fc = m.facet_cells
    assert np.array_equal(d.cf_x[fc[I, 0], fc[I, 1]], d.cf_x[fc[I, 2], fc[I, 3]])
    # trace basis orthogonality on the physical facet: int_F mu_i mu_j = |F| delta_ij
    W = d.cf_w[fc[:, 0], fc[:, 1]]
    G = np.einsum("fq,qi,qj->fij", W, d.mu, d.mu)
    assert np.abs(G - m.area[:, None, None] * np.eye(d.nf)).max() < 1e-13


# ----------------------------------------------------------------- forms

CASES = [(2, 1, 0.0), (2, 2, 0.1), (1, 3, 0.0)]


@pytest.mark.parametrize("n,k,pert", CASES)
def test_p6_div_annihilates_constants(n, k, pert):
    d = _disc(n, k, pert)
    Q = np.random.default_rng(0).standard_normal(d.nQ)
    dq = d.div_c(Q)
    assert abs(d.constant_pressure() @ dq) < 1e-12 * np.abs(dq).sum()


@pytest.mark.parametrize("n,k,pert", CASES)
def test_p7_bdm_invariants(n, k, pert):
    d = _disc(n, k, pert)
    m = d.mesh
    Q = np.random.default_rng(1).standard_normal(d.nQ)
    Qs = d.bdm_project(Q)
    v = d.eval_cf(Qs)
    fc = m.facet_cells
    I = m.interior
    jump = np.einsum("iqc,ic->iq", v[fc[I, 0], fc[I, 1]] - v[fc[I, 2], fc[I, 3]], d.n[fc[I, 0], fc[I, 1]])
    scale = np.abs(v).max()
    assert np.abs(jump).max() < 1e-12 * scale
    wall = np.einsum("iqc,ic->iq", v[fc[~I, 0], fc[~I, 1]], d.n[fc[~I, 0], fc[~I, 1]])
    assert np.abs(wall).max() < 1e-12 * scale
    assert np.abs(d.bdm_project(Qs) - Qs).max() < 1e-11 * np.abs(Qs).max()
    _, grad = d.eval_cell(Qs)
    div = grad[..., 0, 0] + grad[..., 1, 1] + grad[..., 2, 2]
    lhs = np.einsum("kq,qs,kq->ks", d.cw, d.Vp, div).ravel()
    rhs = d.div_c(Q)
    assert np.abs(lhs - rhs).max() < 1e-11 * np.abs(rhs).max()


def test_nedelec_space_dimension():
    for k in (1, 2, 3):
        d = _disc(1, k)
        v = d.nedelec_basis(d.cx, np.arange(d.mesh.ncells))
        assert v.shape[-2] == k * (k + 2) * (k + 3) // 2
        # linearly independent on a cell
        M = np.einsum("q,qlc,qmc->lm", d.cw[0], v[0], v[0])
        ev = np.linalg.eigvalsh(M)
        assert ev[0] > 1e-10 * ev[-1]


def test_p8_label_swap_invariance():
    d0 = _disc(2, 2, 0.1, 3)
    d1 = _disc(2, 2, 0.1, 3, cells_reversed=True)
    nc = d0.mesh.ncells
    permQ = (np.arange(nc)[::-1][:, None] * d0.nu + np.arange(d0.nu)).ravel()
    permP = (np.arange(nc)[::-1][:, None] * d0.npp + np.arange(d0.npp)).ravel()
    I = d0.mesh.interior
    assert np.all(nc - 1 - d0.mesh.facet_cells[I, 0] == d1.mesh.facet_cells[I, 2])
    rng = np.random.default_rng(5)
    Q, W = rng.standard_normal(d0.nQ), rng.standard_normal(d0.nQ)
    p, lam = rng.standard_normal(d0.nP), rng.standard_normal(d0.nT)
    Qs0 = d0.bdm_project(rng.standard_normal(d0.nQ))
    Qs1 = Qs0[permQ]
    assert np.allclose(d1.bdm_project(Qs1), Qs1, atol=1e-11)
    A0, A1 = d0.advection(Qs0), d1.advection(Qs1)
    assert abs(W @ (A0 @ Q) - W[permQ] @ (A1 @ Q[permQ])) < 1e-11 * abs(W @ (A0 @ Q))
    assert np.allclose(d0.g(p, lam)[permQ], d1.g(p[permP], lam), atol=1e-12)
    g0, g1 = d0.gamma(Q, p, lam), d1.gamma(Q[permQ], p[permP], lam)
    assert np.allclose(g0[0][permP], g1[0], atol=1e-12)
    assert np.allclose(g0[1], g1[1], atol=1e-12)
    assert np.allclose(d0.div_c(Q)[permP], d1.div_c(Q[permQ]), atol=1e-12)


@pytest.mark.parametrize("n,k,pert", CASES)
def test_fim_energy_identity(n, k, pert):
    d = _disc(n, k, pert)
    m = d.mesh
    rng = np.random.default_rng(2)
    Q = rng.standard_normal(d.nQ)
    Qs = d.bdm_project(rng.standard_normal(d.nQ))
    lhs = Q @ (d.advection(Qs) @ Q)
    val, _ = d.eval_cell(Q)
    _, gs = d.eval_cell(Qs)
    divs = gs[..., 0, 0] + gs[..., 1, 1] + gs[..., 2, 2]
    vol = 0.5 * np.sum(d.cw * divs * np.sum(val * val, axis=-1))
    v, vs = d.eval_cf(Q), d.eval_cf(Qs)
    fc = m.facet_cells
    I = m.interior
    Kp, fp, Km, fm = fc[I, 0], fc[I, 1], fc[I, 2], fc[I, 3]
    n_ = d.n[Kp, fp]
    W = d.cf_w[Kp, fp]
    jq = v[Kp, fp] - v[Km, fm]
    qn = np.einsum("iqc,ic->iq", vs[Kp, fp], n_)
    up = -d.delta_up * np.sum(W * np.abs(qn) * np.sum(jq * jq, axis=-1))
    pen = -d.alpha * np.sum(W * np.einsum("iqc,ic->iq", jq, n_) ** 2 / m.hF[I][:, None])
    B = ~I
    vb = np.einsum("iqc,ic->iq", v[fc[B, 0], fc[B, 1]], d.n[fc[B, 0], fc[B, 1]])
    pen -= d.alpha * np.sum(d.cf_w[fc[B, 0], fc[B, 1]] * vb**2 / m.hF[B][:, None])
    rhs = vol + up + pen
    assert abs(lhs - rhs) < 1e-11 * (abs(vol) + abs(up) + abs(pen))
    assert up < 0 and pen < 0


@pytest.mark.parametrize("n,k", [(2, 1), (3, 2)])
def test_fim_constant_field_closed_form(n, k):
    d = _disc(n, k)
    one_x = d.l2_project_velocity(lambda x, y, z: np.stack([np.ones_like(x), 0 * x, 0 * x], -1))
    Qs = d.bdm_project(np.random.default_rng(7).standard_normal(d.nQ))
    val = one_x @ (d.advection(Qs) @ one_x)
    # only the wall penalty survives: -alpha sum over the 4 n^2 facets of the
    # two x-walls of h_F^{-1} <1>_F = -alpha 4 n^2 (h_F = <1>_F)
    assert abs(val - (-d.alpha * 4 * n * n)) < 1e-11 * n * n


@pytest.mark.parametrize("k", [2, 3])
def test_divergence_free_polynomial_field(k):
    d = _disc(2, k, 0.1)
    f = lambda x, y, z: np.stack([x * (1 - x) * (1 - 2 * y), -(1 - 2 * x) * y * (1 - y), 0 * z], -1)
    Q = d.l2_project_velocity(f)
    gp, gm = d.gamma(Q, np.zeros(d.nP), np.zeros(d.nT))
    assert np.abs(gp).max() < 1e-13 and np.abs(gm).max() < 1e-13
    assert np.abs(d.div_c(Q)).max() < 1e-13
    assert np.abs(d.bdm_project(Q) - Q).max() < 1e-12


# ---------------------------------------------------------------- the solve

def _compatible_rhs(d, seed):
    rng = np.random.default_rng(seed)
    Fw, Fpsi, Fmu = rng.standard_normal(d.nQ), rng.standard_normal(d.nP), rng.standard_normal(d.nT)
    one_p, one_t = d.constant_pressure(), d.constant_trace()
    Fpsi -= (Fpsi @ one_p - Fmu @ one_t) / (one_p @ one_p) * one_p
    return Fw, Fpsi, Fmu


@pytest.mark.parametrize("k,pert", [(1, 0.0), (2, 0.1)])
@pytest.mark.parametrize("c", [1.0, 2.9e-3])
def test_p3_condensed_equals_monolithic(k, pert, c):
    d = _disc(2, k, pert)
    Fw, Fpsi, Fmu = _compatible_rhs(d, 11)
    U, p, lam = HDGSolver(d, c).solve(Fw, Fpsi, Fmu)
    U2, p2, lam2 = monolithic_solve(d, c, Fw, Fpsi, Fmu)
    H = monolithic_matrix(d, c)
    x = np.concatenate([U, p, lam])
    b = np.concatenate([Fw, Fpsi, Fmu])
    assert np.abs(H @ x - b).max() <= 1e-13 * abs(H).max() * np.abs(x).max()
    rtol = 1e-11 if c >= 0.1 else 1e-8
    for a, ref in ((U, U2), (p, p2), (lam, lam2)):
        assert np.linalg.norm(a - ref) <= rtol * np.linalg.norm(ref)


@pytest.mark.parametrize("n,k", [(2, 1), (2, 2)])
@pytest.mark.parametrize("c", [1.0, 1e-3])
def test_p4_trace_operator_spd_with_constant_null_space(n, k, c):
    d = _disc(n, k, 0.1)
    S = HDGSolver(d, c).S.toarray()
    nrm = np.abs(S).max()
    assert np.abs(S - S.T).max() <= 1e-13 * nrm
    ev, vec = np.linalg.eigh(0.5 * (S + S.T))
    assert ev[0] >= -1e-12 * ev[-1]
    assert ev[1] > 1e-8 * ev[-1]
    z = d.constant_trace()
    z /= np.linalg.norm(z)
    assert abs(abs(vec[:, 0] @ z) - 1.0) < 1e-10
    # 7 facet blocks per row at most: the facet itself and the 3 others of each neighbour
    blocks = (np.abs(S.reshape(d.mesh.nfacets, d.nf, d.mesh.nfacets, d.nf)).sum(axis=(1, 3)) > 0).sum(axis=1)
    assert blocks.max() == 7


def _poly_p(k, seed):
    rng = np.random.default_rng(seed)
    terms = [(e, rng.standard_normal()) for e in monomial_exponents(k, 3)]

    def p(x, y, z):
        return sum(cf * x ** e[0] * y ** e[1] * z ** e[2] for e, cf in terms)

    def grad(x, y, z):
        X = (x, y, z)
        out = []
        for a in range(3):
            g = 0 * x
            for e, cf in terms:
                if e[a] == 0:
                    continue
                f = cf * e[a]
                for b in range(3):
                    f = f * X[b] ** (e[b] - (b == a))
                g = g + f
            out.append(g)
        return np.stack(out, -1)

    def lap(x, y, z):
        X = (x, y, z)
        out = 0 * x
        for e, cf in terms:
            for a in range(3):
                if e[a] > 1:
                    f = cf * e[a] * (e[a] - 1)
                    for b in range(3):
                        f = f * X[b] ** (e[b] - 2 * (b == a))
                    out = out + f
        return out

    return p, grad, lap


@pytest.mark.parametrize("k,pert", [(1, 0.1), (2, 0.0), (2, 0.12)])
@pytest.mark.parametrize("c", [1.0, 0.3])
def test_p5a_patch_test(k, pert, c):
    d = _disc(2, k, pert, seed=4)
    p, grad, lap = _poly_p(k, 9)
    Uf = lambda x, y, z: -c * grad(x, y, z)
    U_ex = d.l2_project_velocity(Uf)
    p_ex = d.l2_project_pressure(p)
    m = d.pressure_integral(p_ex) / d.domain_area()
    p_ex = p_ex - m * d.constant_pressure()
    mesh = d.mesh
    fx = mesh.facet_v0[:, None, :] + np.einsum("fda,qa->fqd", mesh.facet_E, d.fpts)
    # int_F p mu_i / int_F mu_i^2 = 2 sum_q w_q p mu_i on the reference triangle
    lam_ex = (2.0 * (p(fx[..., 0], fx[..., 1], fx[..., 2]) * d.fw[None, :]) @ d.mu).ravel() - m * d.constant_trace()
    Fpsi = np.einsum("kq,qs,kq->ks", d.cw, d.Vp, -c * lap(d.cx[..., 0], d.cx[..., 1], d.cx[..., 2])).ravel()
    Fmu = d.boundary_normal_flux(-Uf(d.cf_x[..., 0], d.cf_x[..., 1], d.cf_x[..., 2]))
    U, ph, lam = HDGSolver(d, c).solve(np.zeros(d.nQ), Fpsi, Fmu)
    assert np.abs(U - U_ex).max() < 1e-11
    assert np.abs(ph - p_ex).max() < 1e-11
    assert np.abs(lam - lam_ex).max() < 1e-11


# ---------------------------------------------------------------- one step

def test_imex_step_constraint_and_energy():
    """ARS(2,3,3) at k = 2 on the Kuhn mesh, curl of the seeded potential."""
    X, C = hi.unit_cube_mesh(2)
    d = Discretisation3D(X, C, 2)
    st = IMEXHDG(d, 2e-3, ars233(), 3)
    par = hi.vector_potential_params(0)
    Q, p, lam = st.initial_state(lambda x, y, z: hi.curl_potential_velocity(par, x, y, z))
    ke = [d.kinetic_energy(Q)]
    t = 0.0
    for _ in range(2):
        Q, p, lam = st.step(Q, p, lam, t)
        t += st.dt
        dp, dl = st.last_final
        gp, gm = d.gamma(Q, dp, dl)
        ops = d.static_operators()
        scale = max(abs(ops["Dv"]).sum(axis=1).max() * np.abs(Q).max(),
                    abs(ops["Tpl"]).sum(axis=1).max() * np.abs(dl).max())
        assert np.abs(gp).max() < 1e-12 * scale
        assert np.abs(gm).max() < 1e-12 * scale
        assert abs(d.pressure_integral(p)) < 1e-12
        ke.append(d.kinetic_energy(Q))
    assert np.all(np.diff(ke) <= 1e-12 * ke[0]), ke


def test_zero_state_stays_zero():
    d = _disc(1, 2)
    st = IMEXHDG(d, 1e-2, ars233(), 2)
    Q, p, lam = st.step(np.zeros(d.nQ), np.zeros(d.nP), np.zeros(d.nT), 0.0)
    assert not Q.any() and not p.any() and not lam.any()
