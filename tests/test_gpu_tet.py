"""GPU parity on tetrahedra (the method for d = 3): every operation of the
HDG-IMEX path through the C ABI against the CPU FP64 oracle's tetrahedral
forms, on seeded Kuhn meshes of the unit cube with perturbed interior
vertices.  FP64 bar: relative L2 <= 1e-12 for single operator
applications, <= 1e-10 for solves and whole steps.
"""
import numpy as np
import pytest

import hdg_inputs as hi
from oracle.forms3d import Discretisation3D
from oracle.hdg import HDGSolver, monolithic_matrix
from oracle.imex import IMEXHDG, ars233

from gpu_util import compatible_rhs, context, dev, host, rel_l2_cells, rel_l2_trace, torch_or_skip

pytestmark = pytest.mark.gpu

CASES = [(2, 1, 0.1), (2, 2, 0.1), (3, 2, 0.0)]


def cube(n, pert=0.0, seed=0):
    X, C = hi.unit_cube_mesh(n)
    if pert:
        X = hi.random_cube_perturbation(X, n, pert, seed)
    return X, C


@pytest.mark.parametrize("n,k,pert", CASES)
def test_points_follow_the_layout(n, k, pert):
    torch_or_skip()
    X, C = cube(n, pert)
    d = Discretisation3D(X, C, k)
    ctx = context(X, C, degree=k)
    assert (ctx.nQ, ctx.nP, ctx.nT) == (d.nQ, d.nP, d.nT)
    assert np.abs(ctx.cell_points() - d.cx).max() < 1e-14
    assert np.abs(ctx.facet_points() - d.cf_x).max() < 1e-14


@pytest.mark.parametrize("n,k,pert", CASES)
@pytest.mark.parametrize("c", [1.0, 2.9e-3])
def test_trace_operator(n, k, pert, c):
    torch = torch_or_skip()
    X, C = cube(n, pert)
    d = Discretisation3D(X, C, k)
    S = HDGSolver(d, c).S
    ctx = context(X, C, degree=k)
    x = np.random.default_rng(3).standard_normal(d.nT)
    y = host(ctx.trace_matvec(c, dev(torch, x)))
    ref = S @ x
    assert np.linalg.norm(y - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("n,k,pert", CASES)
@pytest.mark.parametrize("c", [1.0, 2.9e-3])
@pytest.mark.parametrize("solver", ["jacobi_pcg", "mg_pcg"])
def test_solve_trace(n, k, pert, c, solver):
    torch = torch_or_skip()
    X, C = cube(n, pert)
    d = Discretisation3D(X, C, k)
    Fw, Fpsi, Fmu = compatible_rhs(d, 5)
    U, p, lam = HDGSolver(d, c).solve(Fw, Fpsi, Fmu)
    ctx = context(X, C, degree=k, trace_solver=solver, rtol_trace=1e-13)
    Ug, pg, lg = (host(t) for t in ctx.solve_trace(c, dev(torch, Fw), dev(torch, Fpsi), dev(torch, Fmu)))
    H = monolithic_matrix(d, c)
    x = np.concatenate([Ug, pg, lg])
    assert np.abs(H @ x - np.concatenate([Fw, Fpsi, Fmu])).max() <= 1e-12 * abs(H).max() * np.abs(x).max()
    tol = 1e-10 if c >= 0.1 else 1e-9
    assert rel_l2_cells(d, Ug, U, d.nu) < tol
    assert rel_l2_cells(d, pg, p, d.npp) < tol
    assert rel_l2_trace(d, lg, lam) < tol


@pytest.mark.parametrize("n,k,pert", CASES)
def test_bdm_projection(n, k, pert):
    torch = torch_or_skip()
    X, C = cube(n, pert)
    d = Discretisation3D(X, C, k)
    Q = np.random.default_rng(7).standard_normal(d.nQ)
    got = host(context(X, C, degree=k).bdm_project(dev(torch, Q)))
    assert rel_l2_cells(d, got, d.bdm_project(Q), d.nu) < 1e-12


@pytest.mark.parametrize("n,k,pert", CASES)
def test_weak_divergence(n, k, pert):
    torch = torch_or_skip()
    X, C = cube(n, pert)
    d = Discretisation3D(X, C, k)
    F = np.random.default_rng(8).standard_normal(d.nQ)
    ref = d.div_c(F)
    got = host(context(X, C, degree=k).weak_divergence(dev(torch, F)))
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("n,k,pert", CASES)
def test_constraint_residual(n, k, pert):
    torch = torch_or_skip()
    X, C = cube(n, pert)
    d = Discretisation3D(X, C, k)
    rng = np.random.default_rng(4)
    Q, p, lam = rng.standard_normal(d.nQ), rng.standard_normal(d.nP), rng.standard_normal(d.nT)
    gp, gm = d.gamma(Q, p, lam)
    a, b = context(X, C, degree=k).constraint_residual(dev(torch, Q), dev(torch, p), dev(torch, lam))
    assert np.linalg.norm(host(a) - gp) <= 1e-12 * np.linalg.norm(gp)
    assert np.linalg.norm(host(b) - gm) <= 1e-12 * np.linalg.norm(gm)


@pytest.mark.parametrize("n,k,pert", CASES)
def test_momentum_residual(n, k, pert):
    torch = torch_or_skip()
    X, C = cube(n, pert)
    d = Discretisation3D(X, C, k)
    rng = np.random.default_rng(9)
    r, Q = rng.standard_normal(d.nQ), rng.standard_normal(d.nQ)
    p, lam = rng.standard_normal(d.nP), rng.standard_normal(d.nT)
    Qs = d.bdm_project(10.0 * rng.standard_normal(d.nQ))
    adt = 0.01
    ref = r - d.mass() @ Q + adt * (d.advection(Qs) @ Q + d.g(p, lam))
    got = host(context(X, C, degree=k).momentum_residual(adt, dev(torch, r), dev(torch, Qs), dev(torch, Q),
                                                         dev(torch, p), dev(torch, lam)))
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def _potential_velocity(d, seed=1):
    par = hi.vector_potential_params(seed)
    return d.l2_project_velocity(lambda x, y, z: hi.curl_potential_velocity(par, x, y, z))


@pytest.mark.parametrize("n,k,pert", CASES + [(4, 2, 0.05)])
def test_tentative_velocity(n, k, pert):
    import scipy.sparse.linalg as spla
    torch = torch_or_skip()
    X, C = cube(n, pert)
    d = Discretisation3D(X, C, k)
    Qs = d.bdm_project(_potential_velocity(d))
    rhs = np.random.default_rng(10).standard_normal(d.nQ)
    adt = 0.001
    A = (d.mass() - adt * d.advection(Qs)).tocsc()
    ref = spla.splu(A).solve(rhs)
    ctx = context(X, C, degree=k, rtol_velocity=1e-13)
    got = host(ctx.tentative_velocity(adt, dev(torch, Qs), dev(torch, rhs)))
    minv = 1.0 / d.mass().diagonal()
    assert np.linalg.norm(minv * (A @ got - rhs)) <= 1e-11 * np.linalg.norm(minv * rhs)
    assert rel_l2_cells(d, got, ref, d.nu) < 1e-10


@pytest.mark.parametrize("n,k,pert", CASES)
def test_pressure_reconstruction(n, k, pert):
    torch = torch_or_skip()
    X, C = cube(n, pert)
    d = Discretisation3D(X, C, k)
    st = IMEXHDG(d, 1e-3, ars233(), 1)
    Q = _potential_velocity(d)
    p, lam = st.reconstruct(Q, 0.0)
    pg, lg = context(X, C, degree=k, rtol_trace=1e-13).reconstruct_pressure(dev(torch, Q))
    assert rel_l2_cells(d, host(pg), p, d.npp) < 1e-10
    assert rel_l2_trace(d, host(lg), lam) < 1e-10


def _run_both(n, k, nsteps, dt, nR, pert=0.0, solver="mg_pcg", seed=0, precision="fp64", rtol_velocity=1e-13):
    X, C = cube(n, pert)
    d = Discretisation3D(X, C, k)
    par = hi.vector_potential_params(seed)
    st = IMEXHDG(d, dt, ars233(), nR)
    Q, p, lam = st.initial_state(lambda x, y, z: hi.curl_potential_velocity(par, x, y, z))
    Q, p, lam = st.run(Q, p, lam, 0.0, nsteps)
    ctx = context(X, C, degree=k, imex="ars233", n_richardson=nR, trace_solver=solver, rtol_trace=1e-13,
                  rtol_velocity=rtol_velocity, precision=precision)
    xyz = ctx.cell_points()
    ctx.set_velocity_from_points(hi.curl_potential_velocity(par, xyz[..., 0], xyz[..., 1], xyz[..., 2]))
    ctx.advance(dt, nsteps)
    return d, (Q, p, lam), tuple(host(t) for t in ctx.get_state()), ctx


@pytest.mark.parametrize("n,k,pert,solver", [(2, 1, 0.1, "jacobi_pcg"), (2, 2, 0.1, "mg_pcg"),
                                             (3, 2, 0.05, "mg_pcg")])
def test_steps(n, k, pert, solver):
    """Two ARS(2,3,3) steps with n_R = 3, element by element against the oracle."""
    torch_or_skip()
    d, ref, got, _ = _run_both(n, k, 2, 2e-3, 3, pert=pert, solver=solver)
    errs = (rel_l2_cells(d, got[0], ref[0], d.nu), rel_l2_cells(d, got[1], ref[1], d.npp),
            rel_l2_trace(d, got[2], ref[2]))
    print(f"tet n={n} k={k}: rel L2 Q {errs[0]:.2e} p {errs[1]:.2e} lam {errs[2]:.2e}")
    assert max(errs) < 1e-10, errs


def _facet_schwarz(d, Ahat, r, fp16=False):
    """sum_F R_F^T A_F^{-1} R_F r over interior facets F, A_F the block of the
    mass-scaled Step I operator on the two cells of F (entries of A_F^{-1}
    rounded to FP16 with fp16, the library's storage)."""
    nu = d.nu
    fc = d.mesh.facet_cells
    z = np.zeros_like(r)
    A = Ahat.tocsr()
    for F in np.nonzero(fc[:, 2] >= 0)[0]:
        idx = np.concatenate([fc[F, 0] * nu + np.arange(nu), fc[F, 2] * nu + np.arange(nu)])
        inv = np.linalg.inv(A[idx][:, idx].toarray())
        if fp16:
            inv = np.clip(inv, -65504.0, 65504.0).astype(np.float16).astype(np.float64)
        z[idx] += inv @ r[idx]
    return z


@pytest.mark.parametrize("n,k,pert", [(2, 1, 0.1), (2, 2, 0.1), (3, 2, 0.05)])
def test_patch_preconditioner_matches_dense(n, k, pert):
    import scipy.sparse as sp
    torch = torch_or_skip()
    X, C = cube(n, pert)
    d = Discretisation3D(X, C, k)
    Qs = 8.0 * d.bdm_project(_potential_velocity(d))
    adt = 0.002
    Ahat = sp.diags(1.0 / d.mass().diagonal()) @ (d.mass() - adt * d.advection(Qs))
    r = np.random.default_rng(5).standard_normal(d.nQ)
    ref = _facet_schwarz(d, Ahat, r, fp16=True)
    exact = _facet_schwarz(d, Ahat, r)
    got = host(context(X, C, degree=k).step1_precond(adt, dev(torch, Qs), dev(torch, r)))
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    err_exact = np.linalg.norm(got - exact) / np.linalg.norm(exact)
    print(f"tet n={n} k={k}: {err:.2e} from the FP16-rounded patch inverses, {err_exact:.2e} from the exact ones")
    assert err < 1e-5, err
    assert err_exact < 2e-3, err_exact


def test_step1_solve_with_and_without_preconditioner():
    """Both settings solve the oracle's assembled Step I system (residual
    checked with the oracle's operator; a direct 3D solve at this size would
    take the CPU minutes) to the same solution; the facet-patch
    preconditioner cuts the BiCGStab iterations several times over."""
    torch = torch_or_skip()
    X, C = cube(5, 0.05)
    d = Discretisation3D(X, C, 2)
    Qs = d.bdm_project(_potential_velocity(d, 0))
    rhs = np.random.default_rng(11).standard_normal(d.nQ)
    adt = (3.0 + 3.0 ** 0.5) / 6.0 * 1e-3
    A = (d.mass() - adt * d.advection(Qs)).tocsr()
    minv = 1.0 / d.mass().diagonal()
    its, sol = {}, {}
    for pc in (0, 1):
        ctx = context(X, C, degree=2, rtol_velocity=1e-12, step1_precond=pc)
        got = host(ctx.tentative_velocity(adt, dev(torch, Qs), dev(torch, rhs)))
        its[pc] = ctx.info()["velocity_iterations_last"]
        assert np.linalg.norm(minv * (A @ got - rhs)) <= 1e-10 * np.linalg.norm(minv * rhs)
        sol[pc] = got
        ctx.close()
    assert rel_l2_cells(d, sol[1], sol[0], d.nu) < 1e-9
    print(f"tet 6^3 k=2 Step I BiCGStab iterations: {its[0]} without, {its[1]} with the preconditioner")
    assert its[1] * 3 < its[0], its


@pytest.mark.parametrize("n,k,pert", [(2, 1, 0.1), (3, 2, 0.05)])
def test_mixed_steps(n, k, pert):
    """The mixed-precision mode on tetrahedra (Step I in FP32, stopped at
    1e-5, refined by the FP64 Richardson residual): two ARS(2,3,3) steps within
    1e-6 of the FP64 oracle."""
    torch_or_skip()
    d, ref, got, _ = _run_both(n, k, 2, 2e-3, 3, pert=pert, precision="mixed", rtol_velocity=1e-5)
    errs = (rel_l2_cells(d, got[0], ref[0], d.nu), rel_l2_cells(d, got[1], ref[1], d.npp),
            rel_l2_trace(d, got[2], ref[2]))
    print(f"tet mixed n={n} k={k}: rel L2 Q {errs[0]:.2e} p {errs[1]:.2e} lam {errs[2]:.2e}")
    assert max(errs) < 1e-6, errs
