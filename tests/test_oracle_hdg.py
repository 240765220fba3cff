"""Pins of the oracle's hybridised mixed solve (CPU only).

P3: the statically condensed solve equals a dense solve of the full
    (U, p, lambda) system on tiny meshes, for several c.
P4: the trace operator S is symmetric, positive semi-definite, and its null
    space is exactly the constant trace function.
P5a: patch test - for a global polynomial p of degree <= k, U = -c grad p,
    lambda = p on the skeleton is reproduced to round-off.
P5b: manufactured solution p = cos(pi x) cos(pi y): the pressure error
    decreases at rate ~ k+1 under mesh refinement.
"""
import numpy as np
import pytest

import hdg_inputs as hi
from oracle.forms import Discretisation
from oracle.hdg import HDGSolver, monolithic_matrix, monolithic_solve


def _disc(n, k, pert=0.0, seed=0):
    X, C = hi.unit_square_mesh(n)
    if pert:
        X = hi.random_mesh_perturbation(X, n, pert, seed)
    return Discretisation(X, C, k)


def _compatible_rhs(d, seed):
    rng = np.random.default_rng(seed)
    Fw, Fpsi, Fmu = rng.standard_normal(d.nQ), rng.standard_normal(d.nP), rng.standard_normal(d.nT)
    one_p, one_t = d.constant_pressure(), d.constant_trace()
    # the left null vector (w=0, psi=1, mu=-1) requires F_psi(1) = F_mu(1)
    Fpsi -= (Fpsi @ one_p - Fmu @ one_t) / (one_p @ one_p) * one_p
    return Fw, Fpsi, Fmu


@pytest.mark.parametrize("n,k,pert", [(2, 1, 0.0), (3, 2, 0.2), (3, 3, 0.0), (2, 4, 0.2)])
@pytest.mark.parametrize("c", [1.0, 2.9e-4])
def test_p3_condensed_equals_monolithic(n, k, pert, c):
    d = _disc(n, k, pert)
    Fw, Fpsi, Fmu = _compatible_rhs(d, 11)
    U, p, lam = HDGSolver(d, c).solve(Fw, Fpsi, Fmu)
    U2, p2, lam2 = monolithic_solve(d, c, Fw, Fpsi, Fmu)
    # backward error of the condensed solution against the full operator
    H = monolithic_matrix(d, c)
    x = np.concatenate([U, p, lam])
    b = np.concatenate([Fw, Fpsi, Fmu])
    assert np.abs(H @ x - b).max() <= 1e-13 * abs(H).max() * np.abs(x).max()
    # forward agreement; with small c the scaled system is worse conditioned
    rtol = 1e-11 if c >= 0.1 else 1e-8
    for a, ref in ((U, U2), (p, p2), (lam, lam2)):
        assert np.linalg.norm(a - ref) <= rtol * np.linalg.norm(ref)


@pytest.mark.parametrize("n,k", [(3, 1), (4, 2), (3, 3)])
@pytest.mark.parametrize("c", [1.0, 1e-3])
def test_p4_trace_operator_spd_with_constant_null_space(n, k, c):
    d = _disc(n, k, 0.15)
    S = HDGSolver(d, c).S.toarray()
    nrm = np.abs(S).max()
    assert np.abs(S - S.T).max() <= 1e-14 * nrm * 10
    ev, vec = np.linalg.eigh(0.5 * (S + S.T))
    assert ev[0] >= -1e-12 * ev[-1]
    assert ev[1] > 1e-8 * ev[-1]
    z = d.constant_trace()
    z /= np.linalg.norm(z)
    assert abs(abs(vec[:, 0] @ z) - 1.0) < 1e-10


def _poly_p(k, seed):
    rng = np.random.default_rng(seed)
    terms = [(a, dd - a, rng.standard_normal()) for dd in range(k + 1) for a in range(dd + 1)]

    def p(x, y):
        return sum(cf * x**a * y**b for a, b, cf in terms)

    def grad(x, y):
        gx = sum(cf * a * x ** max(a - 1, 0) * y**b for a, b, cf in terms if a > 0)
        gy = sum(cf * b * x**a * y ** max(b - 1, 0) for a, b, cf in terms if b > 0)
        return np.stack([gx + 0 * x, gy + 0 * x], -1)

    def lap(x, y):
        out = 0 * x
        for a, b, cf in terms:
            if a > 1:
                out = out + cf * a * (a - 1) * x ** (a - 2) * y**b
            if b > 1:
                out = out + cf * b * (b - 1) * x**a * y ** (b - 2)
        return out

    return p, grad, lap


@pytest.mark.parametrize("n,k,pert", [(3, 1, 0.2), (4, 2, 0.0), (3, 3, 0.25)])
@pytest.mark.parametrize("c", [1.0, 0.3])
def test_p5a_patch_test(n, k, pert, c):
    d = _disc(n, k, pert, seed=4)
    p, grad, lap = _poly_p(k, 9)
    Uf = lambda x, y: -c * grad(x, y)
    U_ex = d.l2_project_velocity(Uf)
    p_ex = d.l2_project_pressure(p)
    m = d.pressure_integral(p_ex) / d.domain_area()
    p_ex = p_ex - m * d.constant_pressure()
    # lambda = p on each facet (exactly representable): L2 projection on the facet
    X = d.mesh.facet_points(d.ft)
    from oracle.quadrature import gauss_legendre_01
    w = gauss_legendre_01(d.ft.size)[1]
    lam_ex = ((p(X[..., 0], X[..., 1]) * w[None, :]) @ d.mu).ravel() - m * d.constant_trace()
    Fw = np.zeros(d.nQ)
    Fpsi = np.einsum("kq,qs,kq->ks", d.cw, d.Vp, -c * lap(d.cx[..., 0], d.cx[..., 1])).ravel()
    Fmu = d.boundary_normal_flux(-Uf(d.cf_x[..., 0], d.cf_x[..., 1]))
    U, ph, lam = HDGSolver(d, c).solve(Fw, Fpsi, Fmu)
    assert np.abs(U - U_ex).max() < 1e-11
    assert np.abs(ph - p_ex).max() < 1e-11
    assert np.abs(lam - lam_ex).max() < 1e-11


def _l2_err_p(d, ph, pf):
    vals = np.einsum("qs,ks->kq", d.Vp, ph.reshape(-1, d.npp))
    return np.sqrt(np.sum(d.cw * (vals - pf(d.cx[..., 0], d.cx[..., 1])) ** 2))


@pytest.mark.parametrize("k", [1, 2])
def test_p5b_mms_pressure_rate(k):
    pf = lambda x, y: np.cos(np.pi * x) * np.cos(np.pi * y)
    errs = []
    for n in (4, 8, 16):
        d = _disc(n, k)
        Fpsi = np.einsum("kq,qs,kq->ks", d.cw, d.Vp, 2 * np.pi**2 * pf(d.cx[..., 0], d.cx[..., 1])).ravel()
        _, ph, _ = HDGSolver(d, 1.0).solve(np.zeros(d.nQ), Fpsi, np.zeros(d.nT))
        errs.append(_l2_err_p(d, ph, pf))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > k + 0.8, rates
