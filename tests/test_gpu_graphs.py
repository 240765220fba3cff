"""HIP-graph replay of the Krylov iteration blocks against the same blocks
launched one by one (use_graphs=0).  The replayed graph issues the same
kernels with the same arguments in the same order, so results must agree
bit for bit.  Every replay is checked, with unrelated eager device work and
host synchronisations between the replays; the graph-on runs also use a
caller-owned side stream and the legacy null stream.
"""
import numpy as np
import pytest

import hdg_inputs as hi
from oracle.forms import Discretisation
from oracle.hdg import HDGSolver

from gpu_util import compatible_rhs, context, dev, host, mesh, rel_l2_cells, torch_or_skip

pytestmark = pytest.mark.gpu


def _eager_noise(torch):
    a = torch.randn(257, 263, dtype=torch.float64, device="cuda")
    (a @ a.T).sum().item()
    torch.zeros(1 << 16, device="cuda").add_(1.0)
    torch.cuda.synchronize()


def _pair(X, C, stream=None, **kw):
    on = context(X, C, stream=stream, use_graphs=1, **kw)
    off = context(X, C, use_graphs=0, **kw)
    return on, off


@pytest.mark.parametrize("side_stream", [False, True])
def test_advance_replays_match_eager(side_stream):
    torch = torch_or_skip()
    X, C = mesh(10, 0.15)
    stream = torch.cuda.Stream() if side_stream else None
    kw = dict(degree=2, imex="ars222", n_richardson=2, rtol_trace=1e-13, rtol_velocity=1e-13)
    on, off = _pair(X, C, stream, **kw)
    par = hi.stream_function_params(1)
    for ctx in (on, off):
        xy = ctx.cell_points()
        ctx.set_velocity_from_points(hi.streamfunction_velocity(par, xy[..., 0], xy[..., 1]))
    if stream is not None:
        stream.synchronize()
    for step in range(4):
        on.advance(2e-3, 1)
        off.advance(2e-3, 1)
        if stream is not None:
            stream.synchronize()
        a = [host(t) for t in on.get_state()]
        b = [host(t) for t in off.get_state()]
        for x, y in zip(a, b):
            assert np.array_equal(x, y), f"replay {step}: max diff {np.abs(x - y).max():.3e}"
        _eager_noise(torch)
    io, ie = on.info(), off.info()
    for key in ("pcg_iterations_total", "velocity_iterations_total", "bicgstab_restarts"):
        assert io[key] == ie[key], key


def test_solve_trace_replays_match_eager_and_oracle():
    torch = torch_or_skip()
    X, C = mesh(6, 0.2)
    k, c = 3, 2.9e-2
    d = Discretisation(X, C, k)
    on, off = _pair(X, C, degree=k, rtol_trace=1e-13)
    for seed in range(4):
        Fw, Fpsi, Fmu = compatible_rhs(d, 20 + seed)
        args = [dev(torch, v) for v in (Fw, Fpsi, Fmu)]
        r_on = [host(t) for t in on.solve_trace(c, *args)]
        r_off = [host(t) for t in off.solve_trace(c, *args)]
        for x, y in zip(r_on, r_off):
            assert np.array_equal(x, y), f"rhs {seed}"
        if seed == 0:
            U, p, lam = HDGSolver(d, c).solve(Fw, Fpsi, Fmu)
            assert rel_l2_cells(d, r_on[0], U, d.nu) < 1e-9
        _eager_noise(torch)


def test_tentative_velocity_replays_per_time_step():
    """Step I blocks are captured per adt; alternating adt values reuse them."""
    torch = torch_or_skip()
    X, C = mesh(8, 0.1)
    k = 2
    on, off = _pair(X, C, degree=k, rtol_velocity=1e-13)
    d = Discretisation(X, C, k)
    rng = np.random.default_rng(7)
    par = hi.stream_function_params(2)
    xy = on.cell_points()
    on.set_velocity_from_points(hi.streamfunction_velocity(par, xy[..., 0], xy[..., 1]))
    Qs = on.get_state()[0]
    for i, adt in enumerate([1e-3, 4e-3, 1e-3, 4e-3, 2.5e-3]):
        rhs = dev(torch, rng.standard_normal(d.nQ))
        a = host(on.tentative_velocity(adt, Qs, rhs))
        b = host(off.tentative_velocity(adt, Qs, rhs))
        assert np.array_equal(a, b), f"call {i} (adt {adt})"
        _eager_noise(torch)
