"""Batching and serving of independent instances on one GPU.

* hdg_batch_advance: each member's result is bit for bit that of the same
  context advanced alone;
* hdg_footprint_bytes: the host-side estimate bounds what a context really
  holds after a step (and is not far above it);
* the continuous-batching loop (paper_2410_09790_amd.serve): jobs of mixed
  size and degree admitted by footprint overlap on the device, never exceed
  the memory budget, and each result is the same alone and in the mix.
"""
import time

import numpy as np
import pytest

import hdg_inputs as hi

from gpu_util import context, host, mesh, torch_or_skip

pytestmark = pytest.mark.gpu


def _sf(seed):
    par = hi.stream_function_params(seed)
    return lambda x, y: hi.streamfunction_velocity(par, x, y)


CASES = [(6, 1, 0), (9, 2, 1), (5, 3, 2), (12, 1, 3)]


def _make(torch, n, k, seed, stream=None):
    X, C = mesh(n, 0.1, seed)
    ctx = context(X, C, stream=stream, degree=k, imex="ars222", n_richardson=3, rtol_trace=1e-12,
                  rtol_velocity=1e-11)
    xy = ctx.cell_points()
    ctx.set_velocity_from_points(_sf(seed)(xy[..., 0], xy[..., 1]))
    return ctx


def test_batch_matches_members_alone():
    torch = torch_or_skip()
    from paper_2410_09790_amd import hdg
    alone = []
    for n, k, seed in CASES:
        ctx = _make(torch, n, k, seed)
        ctx.advance(1e-3, 3)
        alone.append([host(t) for t in ctx.get_state()])
        ctx.close()
    streams = [torch.cuda.Stream() for _ in CASES]
    ctxs = [_make(torch, n, k, seed, s) for (n, k, seed), s in zip(CASES, streams)]
    b = hdg.Batch(ctxs)
    status = b.advance(1e-3, 3)
    assert (status == 0).all()
    for ctx, ref in zip(ctxs, alone):
        got = [host(t) for t in ctx.get_state()]
        for x, y in zip(got, ref):
            assert np.array_equal(x, y)
    b.close()
    with pytest.raises(hdg.HDGError):
        hdg.Batch([ctxs[0], ctxs[0]])
    for c in ctxs:
        c.close()


@pytest.mark.parametrize("n,k,imex,kw", [(16, 1, "ars222", {}), (24, 3, "ars222", {}),
                                          (20, 4, "ars222", {"precision": "mixed"}),
                                          (12, 2, "ssp3_433", {"periodic": True}),
                                          (10, 2, "ars222", {"trace_solver": "jacobi_pcg"})])
def test_footprint_bounds_the_device_memory(n, k, imex, kw):
    torch_or_skip()
    from paper_2410_09790_amd import hdg
    kw = dict(kw)
    rep = None
    if kw.pop("periodic", False):
        X, C, rep = hi.periodic_square_mesh(n)
        vel, dt = hi.shear_layer_velocity, 0.04
    else:
        X, C = mesh(n, 0.1)
        vel, dt = _sf(0), 1e-3
    fp = hdg.footprint_bytes(X, C, dt, vertex_rep=rep, degree=k, imex=imex, **kw)
    ctx = context(X, C, vertex_rep=rep, degree=k, imex=imex, **kw)
    xy = ctx.cell_points()
    ctx.set_velocity_from_points(vel(xy[..., 0], xy[..., 1]))
    ctx.advance(dt, 1)
    info = ctx.info()
    ctx.close()
    actual = info["device_bytes"] + info["device_transient_bytes"]
    assert actual <= fp <= 1.3 * actual, (fp, actual)


def test_serving_same_alone_and_in_the_mix():
    torch = torch_or_skip()
    from paper_2410_09790_amd import serve
    jobs = []
    for j, (n, k) in enumerate([(8, 1), (14, 2), (6, 3), (10, 1), (12, 2), (5, 4), (9, 3), (16, 1)]):
        X, C = mesh(n, 0.1, j)
        jobs.append(serve.Job(X, C, _sf(j), 1e-3, 3, dict(degree=k, imex="ars222", n_richardson=3,
                                                          rtol_trace=1e-12, rtol_velocity=1e-11), name=f"j{j}"))
    alone = [serve.run_alone(job)[1] for job in jobs]
    from paper_2410_09790_amd import hdg
    fps = sorted(hdg.footprint_bytes(job.coords, job.cells, job.dt, **job.params) for job in jobs)
    budget = sum(fps[-3:])  # room for about three of the largest at once
    srv = serve.Server(budget, workers=3, slots=4)
    for job in jobs:
        srv.submit(job)
    srv.drain(timeout=120)
    assert srv.max_in_use <= budget
    assert srv.max_active >= 2  # jobs overlapped
    for res, ref in zip(srv.results, alone):
        assert res.error is None, res.error
        for x, y in zip(res.state, ref):
            assert np.array_equal(x, y), res.job.name
    big = serve.Job(*mesh(16), _sf(0), 1e-3, 1, dict(degree=4))
    small = serve.Server(fps[0] // 2, workers=1, slots=1)
    r = small.submit(big)
    assert r.error is not None and "budget" in r.error
    small.drain(timeout=10)


def test_short_job_overtakes_a_long_one():
    """Stage-granular shortest-remaining-work: a short job submitted while a
    long one runs on the only worker finishes first, and both equal their
    lone runs bit for bit."""
    torch_or_skip()
    from paper_2410_09790_amd import serve
    X, C = mesh(16, 0.1, 1)
    long_job = serve.Job(X, C, _sf(1), 1e-3, 12, dict(degree=3, imex="ars222", n_richardson=3), name="long")
    Xs, Cs = mesh(4, 0.1, 2)
    short_job = serve.Job(Xs, Cs, _sf(2), 1e-3, 2, dict(degree=1, imex="ars222", n_richardson=3), name="short")
    alone = [serve.run_alone(j)[1] for j in (long_job, short_job)]
    srv = serve.Server(8 << 30, workers=1, slots=4)
    r_long = srv.submit(long_job)
    while r_long.start == 0.0:  # the long job is on the worker
        time.sleep(0.01)
    r_short = srv.submit(short_job)
    srv.drain(timeout=120)
    assert r_short.end < r_long.end
    for res, ref in zip((r_long, r_short), alone):
        assert res.error is None, res.error
        for x, y in zip(res.state, ref):
            assert np.array_equal(x, y), res.job.name


def test_batch_of_mixed_features():
    """A batch mixing a walled degree-4 member, a periodic shear-layer member
    with SSP3(4,3,3) and a member carrying a tracer: each equals its lone run."""
    torch = torch_or_skip()
    from paper_2410_09790_amd import hdg

    def members(streams):
        X, C = mesh(5, 0.1, 2)
        a = context(X, C, stream=streams[0], degree=4, imex="ars222", n_richardson=2)
        xy = a.cell_points()
        a.set_velocity_from_points(_sf(2)(xy[..., 0], xy[..., 1]))
        Xp, Cp, rep = hi.periodic_square_mesh(6)
        b = context(Xp, Cp, stream=streams[1], vertex_rep=rep, degree=2, imex="ssp3_433", n_richardson=2)
        xy = b.cell_points()
        b.set_velocity_from_points(hi.shear_layer_velocity(xy[..., 0], xy[..., 1]))
        X3, C3 = mesh(6, 0.1, 3)
        c = context(X3, C3, stream=streams[2], degree=2, imex="ssp2_332", n_richardson=2)
        xy = c.cell_points()
        c.set_velocity_from_points(_sf(3)(xy[..., 0], xy[..., 1]))
        c.set_tracer(np.sin(3.0 * xy[..., 0]) * np.cos(2.0 * xy[..., 1]))
        return [a, b, c]

    dts = [1e-3, 0.04, 5e-3]
    alone = members([None, None, None])
    for ctx, dt in zip(alone, dts):
        ctx.advance(dt, 2)
    ref = [[host(t) for t in ctx.get_state()] for ctx in alone]
    ref_q = host(alone[2].get_tracer())
    streams = [torch.cuda.Stream() for _ in range(3)]
    mixed = members(streams)
    b = hdg.Batch(mixed)
    assert (b.advance(dts, 2) == 0).all()
    for ctx, want in zip(mixed, ref):
        for x, y in zip([host(t) for t in ctx.get_state()], want):
            assert np.array_equal(x, y)
    assert np.array_equal(host(mixed[2].get_tracer()), ref_q)
    b.close()
