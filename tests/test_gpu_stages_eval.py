"""Stage-granular stepping (hdg_advance_stages) and the basis-free export
(hdg_eval_points) through the C ABI.

* any chunking of the implicit stages gives the state of hdg_advance bit for
  bit, across step boundaries, and the call sequence is guarded;
* point values of the GPU state at arbitrary reference points agree with the
  oracle's evaluation of the same coefficients in its own basis code.
"""
import numpy as np
import pytest

import hdg_inputs as hi
from oracle.basis import dubiner

from gpu_util import context, host, mesh, torch_or_skip

pytestmark = pytest.mark.gpu


def _ctx(X, C, k, imex, rep=None):
    ctx = context(X, C, vertex_rep=rep, degree=k, imex=imex, n_richardson=2, rtol_trace=1e-12, rtol_velocity=1e-11)
    xy = ctx.cell_points()
    par = hi.stream_function_params(5)
    ctx.set_velocity_from_points(hi.streamfunction_velocity(par, xy[..., 0], xy[..., 1]))
    return ctx


@pytest.mark.parametrize("imex,stages,chunks", [("ars222", 2, [1, 1, 1, 1, 1, 1]), ("ssp3_433", 3, [2, 3, 1, 3]),
                                                ("ssp2_332", 3, [5, 4])])
def test_stage_chunks_match_whole_steps(imex, stages, chunks):
    torch_or_skip()
    from paper_2410_09790_amd import hdg
    X, C = mesh(6, 0.15)
    dt = 2e-3
    nsteps = sum(chunks) // stages
    ref = _ctx(X, C, 2, imex)
    ref.advance(dt, nsteps)
    want = [host(t) for t in ref.get_state()]
    ctx = _ctx(X, C, 2, imex)
    done = 0
    for c in chunks:
        ctx.advance_stages(dt, c)
        done += c
        assert ctx.pending_stage == (done % stages) + 1 if done % stages else ctx.pending_stage == 0
    assert ctx.pending_stage == 0
    got = [host(t) for t in ctx.get_state()]
    for x, y in zip(got, want):
        assert np.array_equal(x, y)
    assert abs(ctx.time - ref.time) < 1e-15
    # guards: another dt mid-step, hdg_advance mid-step; set_state abandons the step
    ctx.advance_stages(dt, 1)
    with pytest.raises(hdg.HDGError):
        ctx.advance_stages(2 * dt, 1)
    with pytest.raises(hdg.HDGError):
        ctx.advance(dt, 1)
    Q, p, lam = ctx.get_state()
    for x, y in zip([host(Q), host(p), host(lam)], want):
        assert np.array_equal(x, y)  # unchanged while the step is in progress
    ctx.set_state(Q, p, lam)
    assert ctx.pending_stage == 0
    ctx.advance(dt, 1)


@pytest.mark.parametrize("k,periodic", [(1, False), (3, False), (2, True)])
def test_eval_points_against_the_oracle_basis(k, periodic):
    torch_or_skip()
    if periodic:
        X, C, rep = hi.periodic_square_mesh(4, amplitude=0.1, seed=2)
    else:
        (X, C), rep = mesh(5, 0.2), None
    ctx = _ctx(X, C, k, "ars222", rep)
    ctx.advance(1e-3, 1)
    Q, p, _ = (host(t) for t in ctx.get_state())
    rng = np.random.default_rng(11)
    pts = rng.uniform(0.0, 1.0, size=(37, 2))
    pts[:, 1] *= 1.0 - pts[:, 0]  # inside the reference triangle
    pts = np.vstack([pts, [[0.0, 0.0], [1.0, 0.0], [0.0, 1.0], [1.2, -0.1]]])  # vertices, one outside
    Qo, po = (host(t) for t in ctx.eval_points(pts))
    Vu = dubiner(k + 1, pts[:, 0], pts[:, 1], derivatives=False)
    Vp = dubiner(k, pts[:, 0], pts[:, 1], derivatives=False)
    ns, npp = Vu.shape[1], Vp.shape[1]
    Qc = Q.reshape(-1, 2, ns)
    want_Q = np.einsum("qs,kcs->kqc", Vu, Qc)
    want_p = np.einsum("qs,ks->kq", Vp, p.reshape(-1, npp))
    assert np.abs(Qo - want_Q).max() <= 1e-13 * np.abs(want_Q).max()
    assert np.abs(po - want_p).max() <= 1e-13 * np.abs(want_p).max()
