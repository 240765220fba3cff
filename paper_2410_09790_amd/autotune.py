"""Autotuner of the Step I operator's launch shape on the current GPU.

The shape is the number of threads per workgroup (64, 128 or 256; two threads
per cell) and the workgroup-to-XCD order (contiguous eighths of the cells per
XCD, or the hardware's round-robin order).  Smaller workgroups spread a small
mesh over more compute units; they also give the Krylov reductions more
partial sums to read, so the figure of merit is wall time per BiCGStab
iteration of a whole Step I solve (Algorithm 2, Step I), the vector updates
and the host's convergence checks included.

For every degree k = 1..4 and walled n x n split-square mesh of a size list,
one context per candidate shape solves the same systems (the state's own
velocity as Q* and as right-hand side, a_ii dt of ARS(2,2,2) at dt = 1e-3);
the candidates are timed in turn, forwards and then backwards, and each keeps
its best time.  The fastest shape per (k, n) goes to a JSON table that the
binding reads (hdg.tuned_launch):

    python -m paper_2410_09790_amd.autotune --out launch_table.json
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import hdg

SHAPES = [(b, x) for b in (256, 128, 64) for x in (1, 0)]
ARS222_GAMMA = 1.0 - 1.0 / np.sqrt(2.0)


def velocity(x, y):
    """A divergence-free field tangent to the walls of the unit square."""
    s, pi = np.sin, np.pi
    return np.stack([s(pi * x) ** 2 * s(2 * pi * y), -s(2 * pi * x) * s(pi * y) ** 2], axis=-1)


def _time_solves(ctx, Q, adt, min_seconds):
    import torch
    torch.cuda.synchronize()
    el, its, n = 0.0, 0, 0
    while n < 2 or el < min_seconds:
        t0 = time.perf_counter()
        ctx.tentative_velocity(adt, Q, Q)
        torch.cuda.synchronize()
        el += time.perf_counter() - t0
        its += ctx.info()["velocity_iterations_last"][-1]
        n += 1
    return el / max(its, 1)


def tune_one(n: int, k: int, dt: float = 1e-3, min_seconds: float = 0.25, log=print):
    coords, cells, _ = hdg.mesh_square(n)
    adt = ARS222_GAMMA * dt
    ctxs, Qs = {}, {}
    try:
        for shape in SHAPES:
            ctx = hdg.Context(coords, cells, degree=k, step1_block=shape[0], step1_xcd=shape[1],
                              rtol_velocity=1e-8, max_it_velocity=20000)
            ctxs[shape] = ctx
            xy = ctx.cell_points()
            ctx.set_velocity_from_points(velocity(xy[..., 0], xy[..., 1]))
            Qs[shape] = ctx.get_state()[0]
            ctx.tentative_velocity(adt, Qs[shape], Qs[shape])  # graph capture, first touches
        best = {s: np.inf for s in SHAPES}
        for order in (SHAPES, SHAPES[::-1]):
            for shape in order:
                best[shape] = min(best[shape], _time_solves(ctxs[shape], Qs[shape], adt, min_seconds))
    finally:
        for ctx in ctxs.values():
            ctx.close()
    win = min(SHAPES, key=lambda s: best[s])
    row = {"degree": k, "n": n, "ncells": 2 * n * n, "step1_block": win[0], "step1_xcd": win[1],
           "us_per_iteration": {f"{b}/{x}": round(best[(b, x)] * 1e6, 2) for b, x in SHAPES}}
    log(f"k={k} n={n}: best {win[0]} threads, xcd {win[1]}; "
        + ", ".join(f"{key} {v:.1f} us" for key, v in row["us_per_iteration"].items()))
    return row


def main(argv=None):
    import torch
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", default=hdg.LAUNCH_TABLE)
    ap.add_argument("--sizes", default="16,32,64,128,256")
    ap.add_argument("--degrees", default="1,2,3,4")
    ap.add_argument("--min-seconds", type=float, default=0.25)
    a = ap.parse_args(argv)
    entries = []
    for k in [int(v) for v in a.degrees.split(",")]:
        for n in [int(v) for v in a.sizes.split(",")]:
            entries.append(tune_one(n, k, min_seconds=a.min_seconds, log=lambda s: print(s, flush=True)))
    table = {"device": torch.cuda.get_device_name(0), "measure": "wall seconds per BiCGStab iteration of a "
             "Step I solve, best of two passes", "candidates": [f"{b}/{x}" for b, x in SHAPES],
             "entries": entries}
    with open(a.out, "w") as f:
        json.dump(table, f, indent=1)
    print(f"wrote {a.out}", flush=True)


if __name__ == "__main__":
    main()
