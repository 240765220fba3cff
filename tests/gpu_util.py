"""Shared helpers of the GPU parity tests (HIP library vs CPU oracle)."""
import numpy as np
import pytest

import hdg_inputs as hi


def torch_or_skip():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    return torch


def mesh(n, pert=0.0, seed=0):
    X, C = hi.unit_square_mesh(n)
    if pert:
        X = hi.random_mesh_perturbation(X, n, pert, seed)
    return X, C


def context(X, C, **kw):
    from paper_2410_09790_amd import hdg
    return hdg.Context(X, C, **kw)


def dev(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def rel_l2_cells(d, a, b, per_cell):
    """Relative L2 difference of cell fields in the orthonormal basis (weight det J)."""
    w = np.repeat(d.mesh.absdet, per_cell)
    num = np.sqrt(np.sum(w * (a - b) ** 2))
    den = np.sqrt(np.sum(w * b**2))
    return num / max(den, 1e-300)


def rel_l2_trace(d, a, b):
    w = np.repeat(d.mesh.hF, d.nf)
    return np.sqrt(np.sum(w * (a - b) ** 2)) / max(np.sqrt(np.sum(w * b**2)), 1e-300)


def compatible_rhs(d, seed):
    rng = np.random.default_rng(seed)
    Fw, Fpsi, Fmu = rng.standard_normal(d.nQ), rng.standard_normal(d.nP), rng.standard_normal(d.nT)
    one_p, one_t = d.constant_pressure(), d.constant_trace()
    Fpsi -= (Fpsi @ one_p - Fmu @ one_t) / (one_p @ one_p) * one_p
    return Fw, Fpsi, Fmu
