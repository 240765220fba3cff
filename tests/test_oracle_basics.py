"""Pins of the oracle's quadrature, bases and function spaces (CPU only).

P1: the unknown counts of the paper's Table "stepsizes" (golden fixture).
P2: quadrature exactness against closed-form monomial integrals.
Bases: orthonormality, derivatives against central differences, and span
(the Dubiner functions of degree m span exactly the monomials of degree <= m).
"""
import math
import os

import numpy as np
import pytest

import hdg_inputs as hi
from oracle.basis import dim_p, dubiner, legendre01
from oracle.mesh import Mesh
from oracle.quadrature import cell_points_1d, facet_points, gauss_legendre_01, triangle_rule

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_dof_counts.txt")


def _table1():
    rows = []
    with open(GOLDEN) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                rows.append([int(v) for v in line.split()])
    return rows


@pytest.mark.parametrize("row", _table1(), ids=lambda r: f"n{r[0]}")
def test_p1_table1_unknown_counts(row):
    n = row[0]
    X, C = hi.unit_square_mesh(n)
    mesh = Mesh(X, C)
    assert mesh.ncells == 2 * n * n
    for k in (1, 2, 3):
        nQ = mesh.ncells * 2 * dim_p(k + 1)
        nP = mesh.ncells * dim_p(k)
        nT = mesh.nfacets * (k + 1)
        assert nQ + nP == row[k]
        assert nT == row[3 + k]


def test_mesh_topology_small():
    X, C = hi.unit_square_mesh(3)
    m = Mesh(X, C)
    assert m.nfacets == 3 * 9 + 2 * 3
    assert int((~m.interior).sum()) == 4 * 3
    # facets are sorted (lo, hi) pairs in lexicographic order
    f = m.facets
    assert np.all(f[:, 0] < f[:, 1])
    assert np.all(np.diff(f[:, 0] * 1000 + f[:, 1]) > 0)
    # outward normals: opposite on the two sides of every interior facet
    fc = m.facet_cells[m.interior]
    assert np.allclose(m.normal[fc[:, 0], fc[:, 1]], -m.normal[fc[:, 2], fc[:, 3]])
    assert np.all(m.detJ > 0)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7])
def test_p2_triangle_rule_exact(n):
    pts, w = triangle_rule(n)
    deg = 2 * n - 1
    for a in range(deg + 1):
        for b in range(deg + 1 - a):
            exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            got = np.sum(w * pts[:, 0] ** a * pts[:, 1] ** b)
            assert abs(got - exact) <= 1e-14 * max(1.0, exact) + 1e-16


def test_p2_rule_sizes_cover_integrands():
    for k in range(1, 6):
        assert 2 * cell_points_1d(k) - 1 >= 3 * k + 2
        assert 2 * facet_points(k) - 1 >= 3 * k + 3


@pytest.mark.parametrize("n", [1, 3, 6, 9])
def test_p2_gauss_legendre_01(n):
    t, w = gauss_legendre_01(n)
    for a in range(2 * n):
        assert abs(np.sum(w * t**a) - 1.0 / (a + 1)) < 1e-14


@pytest.mark.parametrize("m", [0, 1, 2, 3, 4, 5])
def test_dubiner_orthonormal_and_span(m):
    pts, w = triangle_rule(m + 1)
    V, _, _ = dubiner(m, pts[:, 0], pts[:, 1])
    assert V.shape[1] == dim_p(m)
    assert np.abs(V.T @ (w[:, None] * V) - np.eye(dim_p(m))).max() < 1e-13
    # span: monomials of degree <= m are exactly representable (least squares residual 0)
    mono = np.stack([pts[:, 0] ** a * pts[:, 1] ** b for d in range(m + 1) for a in range(d + 1)
                     for b in [d - a]], axis=1)
    coef, res, rank, _ = np.linalg.lstsq(V, mono, rcond=None)
    assert rank == dim_p(m)
    assert np.abs(V @ coef - mono).max() < 1e-12


@pytest.mark.parametrize("m", [1, 2, 4, 5])
def test_dubiner_derivatives_fd(m):
    rng = np.random.default_rng(m)
    xi = rng.uniform(0.05, 0.45, 20)
    eta = rng.uniform(0.05, 0.45, 20)
    _, Dx, Dy = dubiner(m, xi, eta)
    e = 1e-6
    fx = (dubiner(m, xi + e, eta, False) - dubiner(m, xi - e, eta, False)) / (2 * e)
    fy = (dubiner(m, xi, eta + e, False) - dubiner(m, xi, eta - e, False)) / (2 * e)
    assert np.abs(Dx - fx).max() < 1e-6
    assert np.abs(Dy - fy).max() < 1e-6


def test_legendre01_orthonormal():
    t, w = gauss_legendre_01(8)
    L = legendre01(5, t)
    assert np.abs(L.T @ (w[:, None] * L) - np.eye(6)).max() < 1e-13
    assert np.allclose(L[:, 0], 1.0)
