"""Launch shapes of the Step I operator (threads per workgroup 64, 128, 256;
XCD order on and off) against the oracle and against each other.

The operator computes every cell the same way in every shape; only the
partial sums of the Krylov inner products follow the workgroups, so shapes
agree to rounding and one shape repeats its bits.  The 13 x 13 mesh (338
cells, 676 operator threads) leaves a ragged last workgroup in every shape.
"""
import numpy as np
import pytest

import hdg_inputs as hi
from oracle.forms import Discretisation
from oracle.imex import IMEXHDG, ars222

from gpu_util import context, host, mesh, rel_l2_cells, rel_l2_trace, torch_or_skip

pytestmark = pytest.mark.gpu

SHAPES = [(b, x) for b in (64, 128, 256) for x in (1, 0)]


def _run(X, C, k, shape, vel, nsteps, dt, precision="fp64"):
    ctx = context(X, C, degree=k, imex="ars222", n_richardson=2, rtol_trace=1e-13, rtol_velocity=1e-13,
                  step1_block=shape[0], step1_xcd=shape[1], precision=precision)
    assert (ctx.info()["step1_block"], ctx.info()["step1_xcd"]) == shape
    xy = ctx.cell_points()
    ctx.set_velocity_from_points(vel(xy[..., 0], xy[..., 1]))
    ctx.advance(dt, nsteps)
    out = [host(t) for t in ctx.get_state()]
    ctx.close()
    return out


@pytest.mark.parametrize("k", [1, 3])
def test_every_shape_matches_the_oracle(k):
    torch_or_skip()
    X, C = mesh(13, 0.15, seed=3)
    par = hi.stream_function_params(5)
    vel = lambda x, y: hi.streamfunction_velocity(par, x, y)
    d = Discretisation(X, C, k)
    st = IMEXHDG(d, 2e-3, ars222(), 2)
    Q, p, lam = st.initial_state(vel)
    Q, p, lam = st.run(Q, p, lam, 0.0, 2)
    runs = {s: _run(X, C, k, s, vel, 2, 2e-3) for s in SHAPES}
    for s, (gq, gp, gl) in runs.items():
        assert rel_l2_cells(d, gq, Q, d.nu) < 1e-10, s
        assert rel_l2_cells(d, gp, p, d.npp) < 1e-9, s
        assert rel_l2_trace(d, gl, lam) < 1e-9, s
    ref = runs[(256, 1)]
    for s, got in runs.items():
        for a, b in zip(got, ref):
            assert np.linalg.norm(a - b) <= 1e-11 * np.linalg.norm(b), s


def test_a_shape_repeats_its_bits_in_both_precisions():
    torch_or_skip()
    X, C = mesh(13, 0.1, seed=4)
    par = hi.stream_function_params(2)
    vel = lambda x, y: hi.streamfunction_velocity(par, x, y)
    for prec in ("fp64", "mixed"):
        a = _run(X, C, 2, (64, 0), vel, 2, 2e-3, prec)
        b = _run(X, C, 2, (64, 0), vel, 2, 2e-3, prec)
        for x, y in zip(a, b):
            assert np.array_equal(x, y), prec


def test_the_binding_applies_the_tuned_table():
    torch_or_skip()
    from paper_2410_09790_amd import hdg
    X, C = mesh(8)
    for k in (1, 4):
        want = hdg.tuned_launch(k, C.shape[0]) or {"step1_block": 256, "step1_xcd": 1}
        ctx = context(X, C, degree=k)
        info = ctx.info()
        assert (info["step1_block"], info["step1_xcd"]) == (want["step1_block"], want["step1_xcd"])
        ctx.close()
