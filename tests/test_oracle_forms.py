"""Pins of the oracle's weak forms (CPU only).

P6: the weak divergence annihilates constants, Div(1, Q) = 0.
P7: BDM interpolant: single-valued normal component, zero on walls,
    idempotent, and (div P(Q), psi)_K = Div(psi, Q)|_K.
P8: swapping the +/- labels of the facets (by renumbering the cells) leaves
    every assembled form unchanged.
Energy identity for f_im, computed independently at quadrature points:
    f_im(Q, Q, Q*) = 1/2 (div_h Q*, |Q|^2) - delta_up sum_int <|Q*.n| |[Q]|^2>
                     - alpha sum_F h_F^{-1} <[Q.n]^2>
(central and volume terms cancel up to the divergence of Q*, which a sign or
factor error in either term would break).
Closed forms: a constant field sees only the wall penalty; a polynomial
divergence-free field with n.Q = 0 on the walls has Gamma(., Q, 0, 0) = 0,
Div(., Q) = 0 and P(Q) = Q.
"""
import numpy as np
import pytest

import hdg_inputs as hi
from oracle.forms import Discretisation


def _disc(n, k, perturb=0.0, seed=0):
    X, C = hi.unit_square_mesh(n)
    if perturb:
        X = hi.random_mesh_perturbation(X, n, perturb, seed)
    return Discretisation(X, C, k)


def _rand(d, seed=0):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(d.nQ)


CASES = [(3, 1, 0.0), (3, 2, 0.25), (4, 3, 0.2), (2, 4, 0.0)]


@pytest.mark.parametrize("n,k,pert", CASES)
def test_p6_div_annihilates_constants(n, k, pert):
    d = _disc(n, k, pert)
    Q = _rand(d)
    one = d.constant_pressure()
    assert abs(one @ d.div_c(Q)) < 1e-12 * np.abs(d.div_c(Q)).sum()


@pytest.mark.parametrize("n,k,pert", CASES)
def test_p7_bdm_invariants(n, k, pert):
    d = _disc(n, k, pert)
    m = d.mesh
    Q = _rand(d, 1)
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
    # commuting property with the weak divergence
    _, grad = d.eval_cell(Qs)
    div = grad[..., 0, 0] + grad[..., 1, 1]
    lhs = np.einsum("kq,qs,kq->ks", d.cw, d.Vp, div).ravel()
    rhs = d.div_c(Q)
    assert np.abs(lhs - rhs).max() < 1e-11 * np.abs(rhs).max()


def _permuted(n, k, pert):
    X, C = hi.unit_square_mesh(n)
    if pert:
        X = hi.random_mesh_perturbation(X, n, pert, 3)
    return Discretisation(X, C, k), Discretisation(X, C[::-1].copy(), k)


@pytest.mark.parametrize("n,k,pert", [(3, 1, 0.2), (3, 3, 0.0)])
def test_p8_label_swap_invariance(n, k, pert):
    d0, d1 = _permuted(n, k, pert)
    nc = d0.mesh.ncells
    # every interior facet really has its labels swapped
    fc0, fc1 = d0.mesh.facet_cells, d1.mesh.facet_cells
    I = d0.mesh.interior
    assert np.all(nc - 1 - fc0[I, 0] == fc1[I, 2])
    permQ = (np.arange(nc)[::-1][:, None] * d0.nu + np.arange(d0.nu)).ravel()
    permP = (np.arange(nc)[::-1][:, None] * d0.npp + np.arange(d0.npp)).ravel()
    rng = np.random.default_rng(5)
    Q, W = rng.standard_normal(d0.nQ), rng.standard_normal(d0.nQ)
    p, lam = rng.standard_normal(d0.nP), rng.standard_normal(d0.nT)
    Qs0 = d0.bdm_project(rng.standard_normal(d0.nQ))
    Qs1 = Qs0[permQ]
    assert np.allclose(d1.bdm_project(Qs1), Qs1, atol=1e-11)
    A0, A1 = d0.advection(Qs0), d1.advection(Qs1)
    assert abs(W @ (A0 @ Q) - W[permQ] @ (A1 @ Q[permQ])) < 1e-11 * abs(W @ (A0 @ Q))
    assert np.allclose((d0.g(p, lam))[permQ], d1.g(p[permP], lam), atol=1e-12)
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
    divs = gs[..., 0, 0] + gs[..., 1, 1]
    vol = 0.5 * np.sum(d.cw * divs * np.sum(val * val, axis=-1))
    v = d.eval_cf(Q)
    vs = d.eval_cf(Qs)
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


@pytest.mark.parametrize("n,k", [(3, 1), (5, 2)])
def test_fim_constant_field_closed_form(n, k):
    d = _disc(n, k)
    one_x = d.l2_project_velocity(lambda x, y: np.stack([np.ones_like(x), np.zeros_like(x)], -1))
    Qs = d.bdm_project(_rand(d, 7))
    val = one_x @ (d.advection(Qs) @ one_x)
    # only the wall penalty survives: -alpha * sum over x-walls h_F^{-1} <1> = -alpha * 2n
    assert abs(val - (-d.alpha * 2 * n)) < 1e-11 * n


@pytest.mark.parametrize("k", [2, 3])
def test_divergence_free_polynomial_field(k):
    d = _disc(4, k, 0.2)
    f = lambda x, y: np.stack([x * (1 - x) * (1 - 2 * y), -(1 - 2 * x) * y * (1 - y)], -1)
    Q = d.l2_project_velocity(f)
    gp, gm = d.gamma(Q, np.zeros(d.nP), np.zeros(d.nT))
    assert np.abs(gp).max() < 1e-13 and np.abs(gm).max() < 1e-13
    assert np.abs(d.div_c(Q)).max() < 1e-13
    assert np.abs(d.bdm_project(Q) - Q).max() < 1e-12
