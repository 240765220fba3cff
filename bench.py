#!/usr/bin/env python3
"""Throughput benchmark of the HDG-IMEX step on one MI355X.

Workload: the 256 x 256 unit square cut into 131072 triangles, pressure/trace
degree k = 3 (velocity degree 4), stream-function initial velocity of seed 0,
zero forcing, ARS(2,2,2) IMEX, dt = 1e-3, 3 Richardson iterations, trace
systems solved by PCG with the P1-coarse-space multigrid, FP64.

A step is one IMEX-HDG time step (Algorithm 1): two implicit stages of three
Richardson iterations each (residual, tentative-velocity solve, weak
divergence, hybridised mixed solve, update), the BDM interpolant per stage,
the final projection and the pressure reconstruction.

Metric: trace DOF-IMEX-stages per second = N_trace * (s-1) * steps / wall time,
with the state resident on the device before the timed region starts.

The line also carries "mixed": the same workload with the per-stage Step I
cell matrices stored in FP32 and the Step I solves stopped at 1e-5 (FP64
arithmetic, trace solves and Richardson residual, the Richardson loop acting
as iterative refinement), its throughput and the relative L2 difference of
its final state from the FP64 run's.

"latency" gives p50/p99 per-call latencies of hdg_advance (one step) and
hdg_solve_trace on the small 16 x 16, k = 1 workload.

Output: one JSON line on stdout (everything else goes to stderr).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WORKLOAD = {"workload": "unit_square_256x256_k3_ars222", "n": 256, "k": 3, "seed": 0, "scheme": "ars222",
            "dt": 1e-3, "n_richardson": 3, "trace_solver": "mg_pcg", "precision": "fp64",
            # the Step I preconditioner rebuilt once per step (the two implicit
            # stages of ARS(2,2,2) have the same a_ii dt); a solver setting:
            # it changes iteration counts, not the solution
            "step1_precond_lag": 2,
            # the paper's solver tolerances: trace system 1e-12, tentative velocity 1e-10
            "rtol_trace": 1e-12, "rtol_velocity": 1e-10}

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
CSRC = os.path.join(ROOT, "paper_2410_09790_amd", "csrc")
# HBM bytes per launch from the FETCH_SIZE / WRITE_SIZE counter passes (each
# scaled by the counts of a 256 MiB copy), valid only for the kernel code
# they were taken on: the sha256 prefix of the listed functions' source text
# (the kernel and the device functions it calls), so an edit elsewhere in the
# file leaves a record valid and an edit of the kernel voids it
MEASURED_TRAFFIC = {
    "apply_step1_operator": {"src": "step1.hip", "funcs": ["pair_swap", "tile_idx", "step1_core", "xcd_block",
                                                           "stage_fbu", "k_apply_soa"],
                             "sha256": "7c4357a97939b50c", "bytes_per_launch": 244.8e6},
    "step1_precond_apply": {"src": "step1.hip", "funcs": ["PcWood", "k_pc_pass1", "k_pc_pass2"],
                            "sha256": "2f89933d19e0075e", "bytes_per_launch": 1085.9e6},
    "trace_spmv": {"src": "kernels.hip", "funcs": ["k_spmv"], "sha256": "96d7545c27858460", "bytes_per_launch": 159.1e6},
    "trace_spmv_512": {"src": "kernels.hip", "funcs": ["k_spmv"], "sha256": "96d7545c27858460", "bytes_per_launch": 627.3e6},
    # tetrahedra, 32^3 Kuhn cubes, k = 2
    "trace_spmv_tet": {"src": "kernels.hip", "funcs": ["TetRowsShape", "tet_gather", "k_spmv_tet"],
                       "sha256": "4233bb038e2c001c", "bytes_per_launch": 915.8e6},
    "apply_step1_operator_tet": {"src": "kernels3.hip", "funcs": ["wave_sum", "Apply3Shape", "k3_apply"],
                                 "sha256": "2f38edc18632650d", "bytes_per_launch": 1306.9e6},
    "step1_precond_apply_tet": {"src": "kernels3.hip", "funcs": ["PcLayout3", "PcApplyShape3", "k3_pc_apply"],
                                "sha256": "05c242fd8b89e85b", "bytes_per_launch": 12485.2e6},
}
FP64_PEAK_TFLOPS = 78.6      # MI355X FP64 vector
MIXED_RTOL_VELOCITY = 1e-5  # Step I tolerance of the mixed-precision run
PROFILE_EVERY = 15           # event-time one launch in 15 of each kernel class (odd: launches alternate)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_cost(kernel: str, k: int, nc: int, nF: int, nF_int: int | None = None):
    """(bytes, flops) that one launch of `kernel` must move / execute at minimum.

    apply_step1_operator (mass-scaled Step I operator on structure-of-arrays
    vectors; the event class covers its two BiCGStab launches, v = A p with
    rh.v and t = A s with four inner products, which move the same data): per
    cell the advecting field at the nq_cell cell points (2 doubles each),
    3 nq_facet upwind weights, det J and the three normals (7 doubles),
    9 int32 connectivity entries, and 3 velocity vectors of 2 ns doubles
    (input, rh, output).  Flops: per cell and component, per cell point
    3 ns + 2 FMA (the reference gradient, its product with the field, the
    test sum), and per facet point 3 ns FMA (own trace, neighbour trace,
    projection) plus ~10 for the jump and flux.
    trace_spmv (facet-block ELL, FP64): per facet row 5 blocks of (k+1)^2
    values, 5 int32 column ids, reads x and writes y ((k+1) doubles each).
    step1_precond_apply (facet-patch Schwarz of the Step I operator in
    Woodbury form, two launches per application; m = 2 (k+2) trace
    coefficients of a cell on a facet, nu = 2 ns): per cell the FP16 rows
    of the first pass (A_e^{-1} and the three rotated trace maps G_f, nu + 3m
    rows of nu) and of H (nu x 3m), the input and output vectors (nu doubles
    each), the first-pass results (nu + 3m doubles) written once and read
    once, 3 int32 neighbour entries; per interior facet the two cells' rows
    of the FP16 correction (2 x m x 2m) and two FP32 scales.  Flops: the two
    matrix passes and three m x 2m products per cell.  nF_int: the interior
    facets (default nF).
    """
    ns = (k + 2) * (k + 3) // 2
    nqf = (3 * k + 5) // 2
    nf = k + 1
    nu = 2 * ns
    if kernel == "apply_step1_operator":
        nqc = ((3 * k + 4) // 2) ** 2
        nbytes = nc * (8 * (2 * nqc + 3 * nqf + 7 + 3 * 2 * ns) + 4 * 9)
        flops = nc * 2 * (nqc * (6 * ns + 4) + 3 * nqf * (6 * ns + 10) + 2 * ns)
        return nbytes, flops
    if kernel == "step1_precond_apply":
        ni = nF if nF_int is None else nF_int
        mt = 2 * (k + 2)
        r1 = nu + 3 * mt
        nbytes = nc * (2 * r1 * nu + 2 * nu * 3 * mt + 2 * 8 * nu + 2 * 8 * r1 + 4 * 3) + ni * (4 * mt * mt * 2 + 2 * 4)
        flops = nc * (2 * r1 * nu + 2 * nu * 3 * mt + 2 * 6 * mt * mt)
        return nbytes, flops
    if kernel == "trace_spmv":
        nbytes = nF * (8 * 5 * nf * nf + 4 * 5 + 8 * 2 * nf)
        flops = nF * 2 * 5 * nf * nf
        return nbytes, flops
    return None, None


def algorithmic_cost_tet(kernel: str, k: int, nc: int, nF: int, nF_int: int | None = None):
    """(bytes, flops) per launch on tetrahedra (ns = (k+2)(k+3)(k+4)/6 per
    velocity component, nf = (k+1)(k+2)/2 per facet, nq = ceil((3k+4)/2)^2
    facet points).  trace_spmv: per facet row 7 blocks of nf^2 values (the
    three of a wall facet's missing neighbour included: the ELL kernel reads
    them), 7 int32 column ids, x read and y written.  apply_step1_operator:
    per cell the ns x ns volume matrix, 4 nq upwind weights, det J and the
    four normals (13 doubles), 16 int32 connectivity entries, the input,
    output and inner-product vectors (3 x 3 ns doubles); flops: per
    component 2 ns^2 for the volume term and per facet point 2 (3 ns) for
    each of the own trace, the neighbour trace and the test sum.
    step1_precond_apply: per interior facet (nF_int) the FP16 inverse of its
    2 nu x 2 nu patch block (nu = 3 ns), read as two halves by its two cells,
    plus per cell the input and output vectors (nu doubles each) and 4 int32
    neighbour ids.  step1_precond_build (the class covers the cell blocks and
    the patch inversions, once per step): per cell its nu x nu FP64 block
    written and read back, per interior facet the FP16 inverse written;
    flops: 2 (2 nu)^3 per interior facet for the inversion (the matrix cores
    run the rank-4 updates on the block padded to a multiple of 16)."""
    ns = (k + 2) * (k + 3) * (k + 4) // 6
    nf = (k + 1) * (k + 2) // 2
    nq = ((3 * k + 5) // 2) ** 2
    if kernel == "trace_spmv":
        return nF * (8 * 7 * nf * nf + 4 * 7 + 8 * 2 * nf), nF * 2 * 7 * nf * nf
    if kernel == "apply_step1_operator":
        nbytes = nc * (8 * (ns * ns + 4 * nq + 13 + 3 * 3 * ns) + 4 * 16)
        flops = nc * (3 * 2 * ns * ns + 4 * nq * (3 * 2 * 3 * ns + 15))
        return nbytes, flops
    if kernel == "step1_precond_apply":
        nu = 3 * ns
        ni = nF if nF_int is None else nF_int
        return ni * (2 * nu) ** 2 * 2 + nc * (2 * 8 * nu + 4 * 4), ni * 2 * (2 * nu) ** 2
    if kernel == "step1_precond_build":
        nu = 3 * ns
        ni = nF if nF_int is None else nF_int
        return nc * 2 * 8 * nu * nu + ni * (2 * nu) ** 2 * 2, ni * 2 * (2 * nu) ** 3
    return None, None


def method_bytes(kernel: str, k: int, nc: int):
    """Bytes per launch of the Step I operator if it read only what the method
    itself defines per cell: the input, output and inner-product vectors
    (3 x 2 ns doubles), Q* (2 ns doubles), det J and the three normals
    (7 doubles) and 9 int32 connectivity entries; the per-stage field at the
    cell points and upwind weights the kernel streams are a design choice on
    top."""
    if kernel != "apply_step1_operator":
        return None
    ns = (k + 2) * (k + 3) // 2
    return nc * (8 * (4 * 2 * ns + 7) + 4 * 9)


def function_source(text: str, name: str) -> str:
    """Source text of the function or struct `name` (its declaration line
    through the brace that closes its body, template line included)."""
    import re
    m = re.search(r"^[^\n]*\b(?:struct\s+)?" + re.escape(name) + r"\b[^;\n]*(?:\(|\{|$)", text, re.M)
    while m is not None:
        start = text.rfind("\n", 0, m.start()) + 1
        line = text[start:text.find("\n", m.start())]
        if not line.lstrip().startswith(("//", "return", "if", "for")) and ("(" in line or "struct" in line):
            break
        m = re.search(r"^[^\n]*\b" + re.escape(name) + r"\b[^;\n]*(?:\(|\{|$)", text[m.end():], re.M)
        if m is None:
            break
        m = re.search(re.escape(m.group(0)), text)
    if m is None:
        raise KeyError(name)
    start = text.rfind("\n", 0, m.start()) + 1
    prev = text.rfind("\n", 0, start - 1) + 1
    if text[prev:start].lstrip().startswith("template"):
        start = prev
    i = text.index("{", m.start())
    depth = 0
    for j in range(i, len(text)):
        if text[j] == "{":
            depth += 1
        elif text[j] == "}":
            depth -= 1
            if depth == 0:
                return text[start:j + 1]
    raise ValueError(name)


def kernel_sha(rec: dict) -> str:
    import hashlib
    with open(os.path.join(CSRC, rec["src"])) as fh:
        text = fh.read()
    h = hashlib.sha256()
    for name in rec["funcs"]:
        h.update(function_source(text, name).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    rec = MEASURED_TRAFFIC.get(kernel)
    if rec is None:
        return None
    try:
        sha = kernel_sha(rec)
    except KeyError:  # a listed function no longer exists: the record is void
        return None
    return rec["bytes_per_launch"] if sha == rec["sha256"] else None


def cpu_baseline():
    """The oracle (NumPy/SciPy, FP64) on a bounded sample: one step of the same
    scheme, degree, dt, n_R and seed on the 32 x 32 mesh, timed once with the
    BLAS thread pools at one thread and once at their default size (all the
    cores the process may use).  The value is the sample's own throughput in
    trace DOF-stages/s (the better of the two), not an extrapolation to the
    256 x 256 mesh: the oracle's direct solves grow faster than the mesh."""
    from threadpoolctl import threadpool_info, threadpool_limits

    import numpy as np

    import hdg_inputs as hi
    from oracle.forms import Discretisation
    from oracle.imex import IMEXHDG, ars222
    n = 32
    X, C = hi.unit_square_mesh(n)
    par = hi.stream_function_params(WORKLOAD["seed"])
    runs = {}
    for label, limit in (("one_thread", 1), ("all_threads", None)):
        with threadpool_limits(limits=limit):
            threads = max([pool.get("num_threads", 1) for pool in threadpool_info()] or [1])
            d = Discretisation(X, C, WORKLOAD["k"])
            st = IMEXHDG(d, WORKLOAD["dt"], ars222(), WORKLOAD["n_richardson"])
            Q, p, lam = st.initial_state(lambda x, y: hi.streamfunction_velocity(par, x, y))
            t0 = time.perf_counter()
            Q, p, lam = st.step(Q, p, lam, 0.0)
            el = time.perf_counter() - t0
        assert np.all(np.isfinite(Q))
        runs[label] = {"threads": threads, "seconds": round(el, 2), "value": d.nT * (ars222().s - 1) / el}
        log(f"cpu baseline ({label}, {threads} threads): {el:.1f} s for one step")
    best = max(runs, key=lambda r: runs[r]["value"])
    return {"value": runs[best]["value"], "unit": "trace-DOF-stages/s", "cores": runs[best]["threads"],
            "kind": "oracle",
            "sample": f"one ARS(2,2,2) step, k=3, dt=1e-3, n_R=3, seed 0 on the 32x32 mesh ({d.nT} trace DOFs, "
                      "SuperLU direct solves); the value is this sample's own throughput, not extrapolated to "
                      "the 256x256 mesh",
            "runs": runs, "nproc": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}


def trace_operator_run(hdg, hi, torch, n: int = 512, k: int = 3, calls: int = 40):
    """The assembled trace operator (the SpMV of every PCG iteration) on a mesh
    whose operator does not fit the 256 MB last-level cache: 512 x 512, k = 3
    (inside the serving recipe's range), c = gamma dt.  Each of `calls`
    applications is event-timed; algorithmic bytes as in algorithmic_cost."""
    import numpy as np
    X, C = hi.unit_square_mesh(n)
    ctx = hdg.Context(X, C, degree=k, trace_solver="jacobi_pcg", step1_precond=0)
    c = (1.0 - 2.0 ** -0.5) * 1e-3
    x = torch.as_tensor(np.random.default_rng(3).standard_normal(ctx.nT)).cuda()
    ctx.trace_matvec(c, x)  # builds the operator
    ctx.trace_matvec(c, x)
    ctx.profile(1)
    for _ in range(calls):
        ctx.trace_matvec(c, x)
    kv = ctx.info()["kernels"]["trace_spmv"]
    ctx.profile(0)
    nbytes, _ = algorithmic_cost("trace_spmv", k, ctx.ncells, ctx.nfacets)
    avg = kv["ms"] / kv["timed"] * 1e-3
    gbs = nbytes / avg / 1e9
    out = {"workload": f"unit_square_{n}x{n}_k{k} trace operator, c = gamma dt ({ctx.nT} trace DOFs, "
                       f"{nbytes / 1e6:.1f} MB per application, FP64)",
           "avg_launch_us": round(avg * 1e6, 2), "launches": kv["timed"], "algorithmic_bytes_per_launch": nbytes,
           "achieved_GBps": round(gbs, 1), "peak": HBM_PEAK_GBS, "frac": round(gbs / HBM_PEAK_GBS, 4),
           "traffic": MEASURED_TRAFFIC.get("trace_spmv_512", {}).get("bytes_per_launch")
           if measured_traffic("trace_spmv_512") else None}
    log(f"trace operator {n}x{n} k={k}: {avg * 1e6:.1f} us per application, {gbs:.0f} GB/s "
        f"({gbs / HBM_PEAK_GBS:.3f} of peak)")
    ctx.close()
    return out


TET_WORKLOAD = {"n": 32, "k": 2, "seed": 0, "scheme": "ars233", "dt": 1e-3, "n_richardson": 3,
                "trace_solver": "mg_pcg", "rtol_trace": 1e-12, "rtol_velocity": 1e-10}


def tet_run(hdg, hi, torch, n: int, steps: int, warmup: int, trace_calls: int = 20, pc_lag: int = 2,
            mixed: bool = False):
    """The three-dimensional workload: the unit cube in n^3 Kuhn cubes (6 n^3
    tetrahedra), k = 2, the curl of the seeded vector potential, ARS(2,3,3),
    dt = 1e-3, n_R = 3, MG-PCG, the paper's tolerances, FP64, the Step I
    preconditioner rebuilt once per step (pc_lag stages; the two stages of
    a step have the same adt).  Reports trace
    DOF-stages/s over `steps` timed steps, the kernel classes with their
    rooflines, and the assembled trace operator (c = gamma dt) applied
    `trace_calls` times with event timing (out of the last-level cache at
    n = 32).  mixed: also the mixed-precision mode (Step I in FP32 stopped at
    MIXED_RTOL_VELOCITY, FP64 Richardson residual and trace solves) and the
    FP64 path at that Step I tolerance, each against the FP64 state."""
    import numpy as np
    w = TET_WORKLOAD
    k = w["k"]
    X, C = hi.unit_cube_mesh(n)
    t0 = time.perf_counter()
    ctx = hdg.Context(X, C, degree=k, imex=w["scheme"], n_richardson=w["n_richardson"],
                      trace_solver=w["trace_solver"], rtol_trace=w["rtol_trace"], rtol_velocity=w["rtol_velocity"],
                      step1_precond_lag=pc_lag)
    par = hi.vector_potential_params(w["seed"])
    xyz = ctx.cell_points()
    ctx.set_velocity_from_points(hi.curl_potential_velocity(par, xyz[..., 0], xyz[..., 1], xyz[..., 2]))
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    log(f"tet {n}^3: setup {setup:.2f} s, {ctx.ncells} cells, {ctx.nT} trace DOFs, {ctx.nQ} velocity DOFs")
    t0 = time.perf_counter()
    ctx.advance(w["dt"], warmup)
    torch.cuda.synchronize()
    log(f"tet {n}^3: warmup {warmup} step(s) {time.perf_counter() - t0:.2f} s")
    before = ctx.info()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.advance(w["dt"], steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    info = ctx.info()
    ref = tuple(t_.clone() for t_ in ctx.get_state()) if mixed else None  # the mixed runs' reference
    # kernel timing in one more step (event timing replays no graphs)
    ctx.profile(PROFILE_EVERY)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.advance(w["dt"], 1)
    torch.cuda.synchronize()
    el_prof = time.perf_counter() - t1
    kinfo = ctx.info().get("kernels", {})
    ctx.profile(0)
    Q, _, _ = ctx.get_state()
    assert bool(torch.isfinite(Q).all()), "non-finite velocity"
    stages = 2  # ARS(2,3,3): two implicit stages per step
    value = ctx.nT * stages * steps / el
    d = {key: info[key] - before[key] for key in ("pcg_iterations_total", "trace_solves", "velocity_iterations_total",
                                                   "velocity_solves", "bicgstab_restarts", "pcg_floor_stops")}
    log(f"tet {n}^3: {steps} steps {el:.3f} s, {1e3 * el / steps:.1f} ms/step, {value:.4g} trace DOF-stages/s; "
        f"PCG {d['pcg_iterations_total']} its / {d['trace_solves']} solves, Step I "
        f"{d['velocity_iterations_total']} its / {d['velocity_solves']} solves")
    kernels = {}
    for name, kv in kinfo.items():
        if not kv.get("timed"):
            continue
        avg = kv["ms"] / kv["timed"] * 1e-3
        rec = {"avg_launch_us": round(avg * 1e6, 2), "launches": kv["launches"],
               "share_of_step": round(avg * kv["launches"] / el_prof, 3)}
        nb, fl = algorithmic_cost_tet(name, k, ctx.ncells, ctx.nfacets, ctx.nfacets - 12 * n * n)
        if n == 32 and measured_traffic(name + "_tet") is not None:
            rec["traffic"] = measured_traffic(name + "_tet")
        if nb is not None:
            rec.update({"algorithmic_bytes_per_launch": nb, "achieved_GBps": round(nb / avg / 1e9, 1),
                        "frac_hbm": round(nb / avg / 1e9 / HBM_PEAK_GBS, 4), "algorithmic_flops_per_launch": fl,
                        "achieved_TFLOPs": round(fl / avg / 1e12, 3),
                        "frac_fp64": round(fl / avg / 1e12 / FP64_PEAK_TFLOPS, 4)})
        kernels[name] = rec
        log(f"  tet {name:24s} {kv['launches']:7d} launches {avg * 1e6:9.1f} us/launch, "
            f"{rec['share_of_step']:.3f} of the step")
    # the assembled trace operator alone (c = gamma dt), event-timed
    c = (3.0 + 3.0 ** 0.5) / 6.0 * w["dt"]
    x = torch.as_tensor(np.random.default_rng(3).standard_normal(ctx.nT)).cuda()
    ctx.trace_matvec(c, x)
    ctx.profile(1)
    for _ in range(trace_calls):
        ctx.trace_matvec(c, x)
    kv = ctx.info()["kernels"]["trace_spmv"]
    ctx.profile(0)
    avg = kv["ms"] / kv["timed"] * 1e-3
    nb, _ = algorithmic_cost_tet("trace_spmv", k, ctx.ncells, ctx.nfacets)
    gbs = nb / avg / 1e9
    trace = {"avg_launch_us": round(avg * 1e6, 2), "launches": kv["timed"], "algorithmic_bytes_per_launch": nb,
             "achieved_GBps": round(gbs, 1), "peak": HBM_PEAK_GBS, "frac": round(gbs / HBM_PEAK_GBS, 4),
             "traffic": measured_traffic("trace_spmv_tet") if n == 32 else None}
    log(f"tet {n}^3 trace operator: {avg * 1e6:.1f} us per application, {nb / 1e6:.1f} MB, {gbs:.0f} GB/s "
        f"({gbs / HBM_PEAK_GBS:.3f} of peak)")
    mixed_out = None
    if mixed:
        mixed_out = {}
        for label, prec in (("mixed", "mixed"), ("fp64_same_rtol", "fp64")):
            c2 = hdg.Context(X, C, degree=k, imex=w["scheme"], n_richardson=w["n_richardson"],
                             trace_solver=w["trace_solver"], rtol_trace=w["rtol_trace"],
                             rtol_velocity=MIXED_RTOL_VELOCITY, precision=prec, step1_precond_lag=pc_lag)
            c2.set_velocity_from_points(hi.curl_potential_velocity(par, xyz[..., 0], xyz[..., 1], xyz[..., 2]))
            c2.advance(w["dt"], warmup)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            c2.advance(w["dt"], steps)
            torch.cuda.synchronize()
            el2 = time.perf_counter() - t1
            diffs = {nm: float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
                     for nm, a, b in zip(("Q", "p", "lambda"), c2.get_state(), ref)}
            mixed_out[label] = {"ms_per_step": 1e3 * el2 / steps, "value": c2.nT * stages * steps / el2,
                                "rtol_velocity": MIXED_RTOL_VELOCITY, "rel_l2_diff_vs_fp64": diffs}
            log(f"tet {n}^3 {label}: {1e3 * el2 / steps:.1f} ms/step, rel. L2 diff vs FP64 {diffs}")
            c2.close()
        mixed_out["speedup_vs_fp64"] = round(mixed_out["mixed"]["value"] / value, 3)
        mixed_out["speedup_precision_only"] = round(mixed_out["mixed"]["value"] /
                                                    mixed_out["fp64_same_rtol"]["value"], 3)
    out = {"workload": f"unit_cube_{n}^3_kuhn_k{k}_ars233 ({ctx.ncells} tetrahedra, {ctx.nT} trace DOFs)",
           "metric": "trace DOF-IMEX-stages/sec (FP64)", "value": value, "unit": "trace-DOF-stages/s",
           "steps": steps, "warmup": warmup, "ms_per_step": 1e3 * el / steps, "setup_s": round(setup, 2),
           "dt": w["dt"], "n_richardson": w["n_richardson"], "rtol_trace": w["rtol_trace"],
           "rtol_velocity": w["rtol_velocity"], "step1_precond_lag": pc_lag,
           "pcg_iterations_per_solve": round(d["pcg_iterations_total"] / max(d["trace_solves"], 1), 1),
           "velocity_iterations_per_solve": round(d["velocity_iterations_total"] / max(d["velocity_solves"], 1), 1),
           "bicgstab_restarts": d["bicgstab_restarts"], "pcg_floor_stops": d["pcg_floor_stops"],
           "kernels": kernels, "trace_operator": trace, "mixed": mixed_out}
    ctx.close()
    return out


def mixed_run(hdg, hi, torch, w, X, C, args, ref_state):
    """The same workload in the mixed-precision mode: the Step I solve in FP32
    (vectors, cell data, arithmetic) stopped at MIXED_RTOL_VELOCITY, the FP64
    Richardson residual refining each stage, FP64 trace solves.  Reports the
    throughput and the relative L2 difference of the final state from the
    FP64 run above (ref_state: its state after the same warm-up and timed
    steps from the same initial state), and the FP64 path at the same Step I tolerance (the
    equal-tolerance baseline, so that the ratio measures the precision
    alone)."""
    mctx = hdg.Context(X, C, degree=w["k"], imex=w["scheme"], n_richardson=w["n_richardson"],
                       trace_solver=w["trace_solver"], rtol_trace=w["rtol_trace"],
                       rtol_velocity=MIXED_RTOL_VELOCITY, precision="mixed",
                       step1_precond_lag=w["step1_precond_lag"])
    par = hi.stream_function_params(w["seed"])
    xy = mctx.cell_points()
    mctx.set_velocity_from_points(hi.streamfunction_velocity(par, xy[..., 0], xy[..., 1]))
    mctx.advance(w["dt"], args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mctx.advance(w["dt"], args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    # uniform mesh: equal det J in every cell, so 2-norms are L2 norms
    diffs = {}
    for name, a, b in zip(("Q", "p", "lambda"), mctx.get_state(), ref_state):
        diffs[name] = float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
    value = mctx.nT * 2 * args.steps / el
    mctx_nT = mctx.nT
    log(f"mixed: {args.steps} steps {el:.3f} s, {1e3 * el / args.steps:.1f} ms/step, rel. L2 diff vs FP64 {diffs}")
    mctx.close()
    # the equal-tolerance FP64 leg: FP64 storage with the same Step I rtol, so
    # that the ratio measures the precision alone
    fctx = hdg.Context(X, C, degree=w["k"], imex=w["scheme"], n_richardson=w["n_richardson"],
                       trace_solver=w["trace_solver"], rtol_trace=w["rtol_trace"],
                       rtol_velocity=MIXED_RTOL_VELOCITY, precision="fp64",
                       step1_precond_lag=w["step1_precond_lag"])
    fctx.set_velocity_from_points(hi.streamfunction_velocity(par, xy[..., 0], xy[..., 1]))
    fctx.advance(w["dt"], args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fctx.advance(w["dt"], args.steps)
    torch.cuda.synchronize()
    el64 = time.perf_counter() - t0
    diffs64 = {}
    for name, a, b in zip(("Q", "p", "lambda"), fctx.get_state(), ref_state):
        diffs64[name] = float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
    fctx.close()
    value64 = mctx_nT * 2 * args.steps / el64
    log(f"FP64 at the mixed run's Step I rtol: {1e3 * el64 / args.steps:.1f} ms/step, diff vs FP64 {diffs64}")
    return {"value": value, "ms_per_step": 1e3 * el / args.steps,
            "precision": f"Step I in FP32 (Krylov vectors, cell matrices, upwind weights, arithmetic; FP64 inner "
                         f"products) stopped at rtol {MIXED_RTOL_VELOCITY:g}; FP64 Richardson residual (which refines "
                         "each stage), trace solves, increment-form final projection and pressure reconstruction; "
                         "the Step I preconditioner is FP16-stored in both modes",
            "rel_l2_diff_vs_fp64": diffs, "speedup_vs_fp64": None,
            "fp64_same_rtol": {"value": value64, "ms_per_step": 1e3 * el64 / args.steps,
                               "rel_l2_diff_vs_fp64": diffs64},
            "speedup_precision_only": round(value / value64, 3)}


def latency_run(hdg, hi, torch, ncalls: int = 100):
    """Per-call latency distributions on the small parity workload (16 x 16
    mesh, k = 1, ARS(2,2,2), dt = 1e-3, n_R = 3, facet-block-Jacobi PCG at
    1e-12, Step I at 1e-10, FP64): hdg_advance of one step, and
    hdg_solve_trace with c = gamma dt on seeded data, each call synchronous,
    after 5 warm-up calls."""
    import numpy as np
    X, C = hi.unit_square_mesh(16)
    ctx = hdg.Context(X, C, degree=1, imex="ars222", n_richardson=3, trace_solver="jacobi_pcg", rtol_trace=1e-12,
                      rtol_velocity=1e-10)
    par = hi.stream_function_params(0)
    xy = ctx.cell_points()
    ctx.set_velocity_from_points(hi.streamfunction_velocity(par, xy[..., 0], xy[..., 1]))

    def dist(fn):
        for _ in range(5):
            fn()
        ts = []
        for _ in range(ncalls):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(1e3 * (time.perf_counter() - t0))
        ts = np.array(ts)
        return {"p50": round(float(np.percentile(ts, 50)), 3), "p99": round(float(np.percentile(ts, 99)), 3),
                "mean": round(float(ts.mean()), 3), "calls": ncalls}

    adv = dist(lambda: ctx.advance(1e-3, 1))
    rng = np.random.default_rng(7)
    Fpsi = torch.as_tensor(rng.standard_normal(ctx.nP)).cuda()
    Fmu = torch.as_tensor(rng.standard_normal(ctx.nT)).cuda()
    c = (1.0 - 2.0 ** -0.5) * 1e-3
    tr = dist(lambda: ctx.solve_trace(c, None, Fpsi, Fmu))
    ctx.close()
    log(f"latency (16x16, k=1): advance one step p50 {adv['p50']} ms p99 {adv['p99']} ms; "
        f"solve_trace p50 {tr['p50']} ms p99 {tr['p99']} ms")
    return {"workload": "unit_square_16x16_k1_ars222 (512 cells, 1600 trace DOFs), FP64, facet-block-Jacobi PCG",
            "advance_one_step_ms": adv, "solve_trace_ms": tr}


def shear_layer_run(hdg, hi, torch, nsteps: int = 5):
    """The paper's double-layer shear flow (Section "Double-layer shear flow")
    at its largest tabulated size: [0, 2 pi]^2 periodic, 64 x 64 squares,
    k = 3, SSP3(4,3,3), dt = 0.04, n_R = 2, the paper's tolerances (trace
    1e-12, Step I 1e-10), FP64; one warm-up step, then nsteps timed steps
    with the state resident on the device."""
    import numpy as np
    n, k, dt = 64, 3, 0.04
    X, C, rep = hi.periodic_square_mesh(n)
    ctx = hdg.Context(X, C, vertex_rep=rep, degree=k, imex="ssp3_433", n_richardson=2, rtol_trace=1e-12,
                      rtol_velocity=1e-10)
    xy = ctx.cell_points()
    ctx.set_velocity_from_points(hi.shear_layer_velocity(xy[..., 0], xy[..., 1]))
    ctx.advance(dt, 1)
    torch.cuda.synchronize()
    i0 = ctx.info()
    t0 = time.perf_counter()
    ctx.advance(dt, nsteps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    i1 = ctx.info()
    Q = ctx.get_state()[0].cpu().numpy().reshape(ctx.ncells, -1)
    det = (L_SHEAR / n) ** 2  # det J of every cell of the uniform mesh; the velocity mass matrix is det J times I
    ke = 0.5 * det * float(np.sum(Q * Q))
    nT = ctx.nT
    ctx.close()
    stages = 3  # implicit stages of SSP3(4,3,3)
    its = {key: i1[key] - i0[key] for key in ("pcg_iterations_total", "trace_solves", "velocity_iterations_total",
                                              "velocity_solves")}
    log(f"shear layer (64x64 periodic, k=3, SSP3(4,3,3)): {1e3 * el / nsteps:.1f} ms/step over {nsteps} steps; {its}")
    return {"workload": "periodic_2pi_64x64_k3_ssp3_433 (8192 cells, 49152 trace DOFs), dt=0.04, n_R=2, FP64",
            "ms_per_step": 1e3 * el / nsteps, "steps": nsteps, "value": nT * stages * nsteps / el,
            "unit": "trace-DOF-stages/s", "kinetic_energy_after": ke, "iterations": its,
            "paper_s_per_step": 52.16,
            "paper_note": "the paper's shear-layer table, SSP3(4,3,3), k=3, 64x64: 52.16 s per step on its "
                          "own (CPU) hardware; context, not a target"}


L_SHEAR = 2.0 * 3.141592653589793


def batched_run(hdg, hi, torch, ninst: int = 4, steps: int = 1):
    """A bounded sample of the batched workload: instances j = 0..ninst-1 with
    n = integers(32, 257), k = integers(1, 5) drawn from default_rng(j) and
    the seed-j stream-function data; ARS(2,2,2), dt = 1e-3, n_R = 3, MG-PCG,
    the paper's tolerances.  One untimed warm-up step (operator builds, graph
    capture), then `steps` timed steps of every instance one after another
    (FP64), `steps` timed steps of all of them as one hdg_batch on distinct
    streams (FP64), and the same with FP32 cell-matrix storage (Step I rtol
    1e-5).  The mixed states after 1 + steps steps are compared with the FP64
    states after as many."""
    import numpy as np
    specs = []
    for j in range(ninst):
        n, k, par = hi.batched_instance(j)
        specs.append((par, n, k))

    def make(n, k, par, stream, **kw):
        X, C = hi.unit_square_mesh(n)
        ctx = hdg.Context(X, C, stream=stream, degree=k, imex="ars222", n_richardson=3, rtol_trace=1e-12, **kw)
        xy = ctx.cell_points()
        ctx.set_velocity_from_points(hi.streamfunction_velocity(par, xy[..., 0], xy[..., 1]))
        return ctx

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    dt = 1e-3
    streams = [torch.cuda.Stream() for _ in specs]
    f64 = []
    for (par, n, k), s in zip(specs, streams):
        f64.append(make(n, k, par, s, rtol_velocity=1e-10))
        if len(f64) % 8 == 0:
            log(f"batched: {len(f64)} of {len(specs)} FP64 instances set up")
    work = sum(c.nT * 2 for c in f64) * steps  # trace DOF-stages of `steps` steps of every instance
    bf = hdg.Batch(f64)
    bf.advance(dt, 1)  # warm-up
    log("batched: FP64 warm-up step done")

    def one_by_one():
        for i, c in enumerate(f64):
            c.advance(dt, steps)
            if (i + 1) % 8 == 0:
                log(f"batched: {i + 1} of {len(f64)} instances advanced one at a time")

    t_seq = timed(one_by_one)
    ref = [tuple(t.cpu().numpy() for t in c.get_state()) for c in f64]
    def batch_steps(b, what):
        for i in range(steps):  # one step per call: a progress line per step
            b.advance(dt, 1)
            if steps > 1:
                log(f"batched: {what} step {i + 1} of {steps}")

    t_bat = timed(lambda: batch_steps(bf, "FP64"))
    log(f"batched: FP64 one at a time {t_seq:.1f} s, as one batch {t_bat:.1f} s")
    bf.close()
    for c in f64:
        c.close()
    mstreams = [torch.cuda.Stream() for _ in specs]
    mx = [make(n, k, par, s, rtol_velocity=MIXED_RTOL_VELOCITY, precision="mixed")
          for (par, n, k), s in zip(specs, mstreams)]
    bm = hdg.Batch(mx)
    bm.advance(dt, 1)  # warm-up
    log("batched: mixed warm-up step done")
    t_mix = timed(lambda: batch_steps(bm, "mixed"))
    diff = 0.0
    for c, (Q, p, lam) in zip(mx, ref):
        Qm, pm, lm = (t.cpu().numpy() for t in c.get_state())
        diff = max(diff, float(np.linalg.norm(Qm - Q) / np.linalg.norm(Q)),
                   float(np.linalg.norm(pm - p) / np.linalg.norm(p)), float(np.linalg.norm(lm - lam) / np.linalg.norm(lam)))
    bm.close()
    for c in mx:
        c.close()
    out = {"workload": "batched sample: instances " + ", ".join(f"{n}x{n} k={k}" for _, n, k in specs) +
                       " (draws j = 0..%d of the batched recipe), ARS(2,2,2), dt=1e-3, n_R=3, %d timed step(s) each"
                       % (ninst - 1, steps),
           "unit": "trace-DOF-stages/s",
           "fp64_one_at_a_time": work / t_seq, "fp64_batched": work / t_bat, "mixed_batched": work / t_mix,
           "mixed_max_rel_l2_diff_vs_fp64": diff,
           "seconds": {"fp64_one_at_a_time": t_seq, "fp64_batched": t_bat, "mixed_batched": t_mix}}
    log(f"batched: one-at-a-time FP64 {work / t_seq:.4g}, batched FP64 {work / t_bat:.4g}, batched mixed "
        f"{work / t_mix:.4g} trace-DOF-stages/s; mixed vs FP64 {diff:.2e}")
    return out


def serving_run(hdg, hi, torch, njobs: int = 16, nmax: int = 48, steps: int = 10, rhos=(0.5, 0.8),
                workers=(1, 2)):
    """A sample of the serving workload: jobs j = 0..njobs-1 with
    n = round(exp(U(ln 16, ln 512))) (clipped to nmax when nmax < 512) and
    k = integers(1, 5) from default_rng(10000 + j), `steps` ARS(2,2,2) steps
    each (dt = 1e-3, n_R = 3, Jacobi-PCG below 32 x 32, else MG-PCG; FP64 at
    the paper's tolerances).  Each job first runs alone (service time and
    reference state); then, for each offered load rho, the jobs arrive with
    exponential gaps from default_rng(999) at rate rho / mean alone time, and
    are run twice under the same arrivals: one at a time in arrival order
    (FIFO, measured) and by the stage-granular shortest-remaining-work server
    (admission by footprint) with each worker-thread count in `workers`.
    Latency = arrival to completion."""
    import threading
    import numpy as np
    from paper_2410_09790_amd import serve
    jobs = []
    for j in range(njobs):
        n, k, par = hi.serving_job(j)
        n = min(n, nmax)
        X, C = hi.unit_square_mesh(n)
        solver = "jacobi_pcg" if n < 32 else "mg_pcg"
        vel = (lambda par_: lambda x, y: hi.streamfunction_velocity(par_, x, y))(par)
        jobs.append(serve.Job(X, C, vel, 1e-3, steps,
                              dict(degree=k, imex="ars222", n_richardson=3, trace_solver=solver, rtol_trace=1e-12,
                                   rtol_velocity=1e-10), name=f"{n}x{n} k={k}"))
    alone = []
    for i, job in enumerate(jobs):
        alone.append(serve.run_alone(job))
        log(f"serving: job {i} ({job.name}) alone {alone[-1][0]:.2f} s")
    service = np.array([a[0] for a in alone])
    work = sum(a[2] * steps * 2 for a in alone)
    out = {"workload": f"serving sample: jobs 0..{njobs - 1} of the serving recipe" +
                       (f", n clipped to {nmax}" if nmax < 512 else " (n not clipped)") +
                       f", {steps} ARS(2,2,2) steps each, Poisson arrivals at offered load rho (arrival rate x mean "
                       f"alone service time); FP64, paper tolerances",
           "jobs": [j.name for j in jobs], "alone_s": [round(float(x), 3) for x in service],
           "unit": "trace-DOF-stages/s", "server": "stage-granular shortest remaining work",
           "loads": {}}
    for rho in rhos:
        arrivals = hi.serving_arrivals(service.mean() / rho, njobs)
        fifo = serve.run_fifo(jobs, arrivals,
                              progress=lambda i, r: log(f"serving rho={rho}: FIFO job {i - 1} done at {r[2]:.1f} s"))
        fifo_lat = [e - a for a, _, e in fifo]
        fifo_span = max(e for _, _, e in fifo) - arrivals[0]
        log(f"serving rho={rho}: FIFO p50/p99 {serve.percentiles(fifo_lat)} s")
        load = {"fifo_one_at_a_time_measured": {"latency_s": serve.percentiles(fifo_lat),
                                                "mean_latency_s": float(np.mean(fifo_lat)),
                                                "throughput": work / fifo_span}}
        for nw in workers:
            srv = serve.Server(64 << 30, workers=nw,
                               on_done=lambda r, nw=nw: log(f"serving rho={rho}, {nw} workers: job "
                                                            f"{srv.results.index(r)} done at {r.end:.1f} s"))

            def feed():
                t0 = srv.now()
                for a_j, job in zip(arrivals, jobs):
                    wait = a_j - (srv.now() - t0)
                    if wait > 0:
                        time.sleep(wait)
                    srv.submit(job)

            th = threading.Thread(target=feed)
            th.start()
            th.join()
            srv.drain()
            res = srv.results
            same = all(r.error is None and all(np.array_equal(x, y) for x, y in zip(r.state, a[1]))
                       for r, a in zip(res, alone))
            lat = [r.latency for r in res]
            makespan = max(r.end for r in res) - min(r.arrival for r in res)
            load[f"served_{nw}_workers"] = {"policies": srv.policies,
                "latency_s": serve.percentiles(lat), "mean_latency_s": float(np.mean(lat)),
                "throughput": work / makespan, "max_active": srv.max_active, "max_in_use_bytes": srv.max_in_use,
                "results_identical_to_alone": bool(same)}
            log(f"serving rho={rho}, {nw} workers: served p50/p99 {serve.percentiles(lat)} s, mean "
                f"{np.mean(lat):.3f} s, throughput {work / makespan:.4g}; FIFO {serve.percentiles(fifo_lat)} s, mean "
                f"{np.mean(fifo_lat):.3f} s, {work / fifo_span:.4g}; identical to alone: {same}")
        out["loads"][str(rho)] = load
    return out


def copy_bandwidth(torch, mib: int = 2048, reps: int = 5) -> float:
    """GB/s (bytes read + written) of a plain device-to-device copy of mib MiB,
    larger than the last-level cache: what a streaming kernel reaches on this
    device, reported beside the published peak."""
    src = torch.ones(mib * (1 << 20) // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    gbs = 2.0 * src.numel() * 8 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=WORKLOAD["n"], help="mesh size (experiments only)")
    ap.add_argument("--k", type=int, default=WORKLOAD["k"], help="degree (experiments only)")
    ap.add_argument("--pc-lag", type=int, default=WORKLOAD["step1_precond_lag"],
                    help="stages between rebuilds of the Step I preconditioner")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="do not time kernels with events")
    ap.add_argument("--profile-steps", type=int, default=2,
                    help="steps run after the timed ones with per-kernel event timing")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision run")
    ap.add_argument("--no-latency", action="store_true", help="skip the per-call latency distributions")
    ap.add_argument("--no-shear", action="store_true", help="skip the periodic shear-layer run")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-instances sample")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving sample")
    ap.add_argument("--no-trace-op", action="store_true", help="skip the out-of-cache trace-operator leg")
    ap.add_argument("--no-tet", action="store_true", help="skip the three-dimensional (tetrahedra) leg")
    ap.add_argument("--tet-n", type=int, default=TET_WORKLOAD["n"], help="cubes per side of the 3D leg")
    ap.add_argument("--tet-steps", type=int, default=2, help="timed steps of the 3D leg (workload: 10)")
    ap.add_argument("--tet-only", action="store_true", help="run only the three-dimensional leg")
    ap.add_argument("--tet-mixed", action="store_true",
                    help="3D leg: also the mixed-precision mode and FP64 at its Step I tolerance")
    ap.add_argument("--tet-pc-lag", type=int, default=2,
                    help="stages between rebuilds of the 3D leg's Step I preconditioner (2: once per step)")
    ap.add_argument("--batched-instances", type=int, default=4, help="instances of the batched sample (recipe: 64)")
    ap.add_argument("--batched-steps", type=int, default=1, help="timed steps of the batched sample (recipe: 10)")
    ap.add_argument("--serving-jobs", type=int, default=16, help="jobs of the serving sample (recipe: 200)")
    ap.add_argument("--serving-nmax", type=int, default=48, help="mesh size cap of the serving sample (recipe: 512)")
    ap.add_argument("--serving-rho", type=float, nargs="+", default=[0.5, 0.8],
                    help="offered loads of the serving sample: arrival rate x mean alone service time (recipe: 0.5, 0.8)")
    ap.add_argument("--serving-steps", type=int, default=10, help="steps per serving job (recipe: 20)")
    ap.add_argument("--serving-workers", type=int, nargs="+", default=[1, 2],
                    help="worker-thread counts of the serving loop to measure")
    ap.add_argument("--serving-only", action="store_true",
                    help="run only the serving sample and print it as the JSON line (a separate measurement)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MB",
                    help="also run a plain device copy of this many MiB (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU decomposition is a design, not code)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import hdg_inputs as hi
    from paper_2410_09790_amd import hdg

    torch.cuda.set_device(0)
    if args.serving_only:
        serving = serving_run(hdg, hi, torch, args.serving_jobs, args.serving_nmax, args.serving_steps,
                              tuple(args.serving_rho), tuple(args.serving_workers))
        print(json.dumps({"metric": "serving job latency p50/p99 (s) and throughput", "serving": serving}), flush=True)
        return
    if args.copy_probe:
        # a plain copy kernel of known size: its FETCH_SIZE / WRITE_SIZE counters
        # calibrate the byte counters of the HDG kernels
        src = torch.ones(args.copy_probe * (1 << 20) // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe} MiB read + {args.copy_probe} MiB written per launch, 3 launches")
    if args.tet_only:
        tet = tet_run(hdg, hi, torch, args.tet_n, args.tet_steps, args.warmup, pc_lag=args.tet_pc_lag,
                      mixed=args.tet_mixed)
        print(json.dumps({"metric": "trace DOF-IMEX-stages/sec (FP64), tetrahedra", "tet": tet}), flush=True)
        return
    w = dict(WORKLOAD)
    w["n"], w["k"], w["step1_precond_lag"] = args.n, args.k, args.pc_lag
    if (args.n, args.k) != (WORKLOAD["n"], WORKLOAD["k"]):
        w["workload"] = f"unit_square_{args.n}x{args.n}_k{args.k}_ars222"
    X, C = hi.unit_square_mesh(w["n"])
    t0 = time.perf_counter()
    ctx = hdg.Context(X, C, degree=w["k"], imex=w["scheme"], n_richardson=w["n_richardson"],
                      trace_solver=w["trace_solver"], rtol_trace=w["rtol_trace"],
                      rtol_velocity=w["rtol_velocity"], step1_precond_lag=w["step1_precond_lag"])
    par = hi.stream_function_params(w["seed"])
    xy = ctx.cell_points()
    ctx.set_velocity_from_points(hi.streamfunction_velocity(par, xy[..., 0], xy[..., 1]))
    torch.cuda.synchronize()
    log(f"setup {time.perf_counter() - t0:.2f} s: {ctx.ncells} cells, {ctx.nT} trace DOFs, {ctx.nQ} velocity DOFs")
    t0 = time.perf_counter()
    ctx.advance(w["dt"], args.warmup)
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} step(s) {time.perf_counter() - t0:.2f} s")
    before = ctx.info()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.advance(w["dt"], args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    info = ctx.info()
    ref_state = tuple(t_.clone() for t_ in ctx.get_state())  # the state the mixed leg is compared with
    kinfo, el_prof = {}, el
    if not args.no_profile:
        # per-kernel timing in extra steps after the timed region: HIP events
        # around every PROFILE_EVERY-th launch of each kernel class (event
        # timing runs the Krylov blocks eagerly instead of replaying their
        # graphs, so it stays out of the headline)
        ctx.profile(PROFILE_EVERY)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ctx.advance(w["dt"], args.profile_steps)
        torch.cuda.synchronize()
        el_prof = time.perf_counter() - t1
        kinfo = ctx.info().get("kernels", {})
        ctx.profile(0)
        log(f"profiled {args.profile_steps} more steps: {1e3 * el_prof / args.profile_steps:.1f} ms/step with event timing")
    Q, p, lam = ref_state
    assert bool(torch.isfinite(Q).all()), "non-finite velocity"
    stages = 2
    value = ctx.nT * stages * args.steps / el
    vel_last = info["velocity_iterations_last"]
    pcg = info["pcg_iterations_total"] - before["pcg_iterations_total"]
    bicg = info["velocity_iterations_total"] - before["velocity_iterations_total"]
    nsolves = info["trace_solves"] - before["trace_solves"]
    nvel = info["velocity_solves"] - before["velocity_solves"]
    log(f"Step I iterations per solve (last): {info['velocity_iterations_last']}, restarts {info.get('bicgstab_restarts')}")
    log(f"PCG iterations per solve (last): {info['pcg_iterations_last']}")
    log(f"timed {args.steps} steps: {el:.3f} s, {1e3 * el / args.steps:.1f} ms/step; "
        f"PCG {pcg} its over {nsolves} trace solves, Step I {bicg} its over {nvel} velocity solves")
    kernels = {n_: kv for n_, kv in kinfo.items() if kv.get("timed")}
    for kv in kernels.values():
        kv["avg_us"] = kv["ms"] / kv["timed"] * 1e3
        kv["est_ms"] = kv["avg_us"] * kv["launches"] * 1e-3
    for name, kv in sorted(kernels.items(), key=lambda kv: -kv[1]["est_ms"]):
        log(f"  {name:24s} {kv['launches']:7d} launches ({kv['timed']} timed) {kv['avg_us']:9.1f} us/launch, "
            f"~{kv['est_ms']:9.1f} ms in total")
    roofline = None
    timed = {n_: kv for n_, kv in kernels.items() if algorithmic_cost(n_, 1, 1, 1)[0] is not None}
    nF_int = ctx.nfacets - 4 * w["n"]  # the n x n square has 4 n wall facets
    # every kernel class with a cost model, with its roofline figures
    per_kernel = {}
    for n_, kv in timed.items():
        nb_, fl_ = algorithmic_cost(n_, w["k"], ctx.ncells, ctx.nfacets, nF_int)
        gbs = nb_ / (kv["avg_us"] * 1e-6) / 1e9
        per_kernel[n_] = {"avg_launch_us": round(kv["avg_us"], 2), "launches": kv["launches"],
                          "algorithmic_bytes_per_launch": nb_, "achieved_GBps": round(gbs, 1),
                          "frac": round(gbs / HBM_PEAK_GBS, 4), "share_of_step": round(kv["est_ms"] * 1e-3 / el_prof, 3),
                          "traffic": measured_traffic(n_)}
        mb = method_bytes(n_, w["k"], ctx.ncells)
        if mb is not None:
            per_kernel[n_]["method_bytes_per_launch"] = mb
            per_kernel[n_]["frac_method_bytes"] = round(mb / (kv["avg_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)
    if timed:
        dom = max(timed, key=lambda n_: timed[n_]["est_ms"])
        nbytes, flops = algorithmic_cost(dom, w["k"], ctx.ncells, ctx.nfacets, nF_int)
        avg_s = timed[dom]["avg_us"] * 1e-6
        t_mem, t_alu = nbytes / (HBM_PEAK_GBS * 1e9), flops / (FP64_PEAK_TFLOPS * 1e12)
        if t_mem >= t_alu:
            ach = nbytes / avg_s / 1e9
            roofline = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": measured_traffic(dom), "kernel": dom,
                        "algorithmic_bytes_per_launch": nbytes, "avg_launch_us": round(avg_s * 1e6, 2),
                        "share_of_step": round(timed[dom]["est_ms"] * 1e-3 / el_prof, 3)}
            copy = copy_bandwidth(torch)
            roofline["device_copy_GBps"] = round(copy, 1)
            roofline["frac_of_device_copy"] = round(ach / copy, 4)
            roofline["kernels"] = per_kernel
            log(f"plain device copy (2 GiB): {copy:.0f} GB/s read + written; the dominant kernel reaches "
                f"{ach / copy:.2f} of it")
        else:
            ach = flops / avg_s / 1e12
            roofline = {"bound": "alu", "achieved": round(ach, 2), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(ach / FP64_PEAK_TFLOPS, 4), "traffic": measured_traffic(dom), "kernel": dom,
                        "algorithmic_flops_per_launch": flops, "avg_launch_us": round(avg_s * 1e6, 2),
                        "share_of_step": round(timed[dom]["est_ms"] * 1e-3 / el_prof, 3)}
    mixed = None
    if not args.no_mixed:
        mixed = mixed_run(hdg, hi, torch, w, X, C, args, ref_state)
    latency = None
    if not args.no_latency:
        latency = latency_run(hdg, hi, torch)
    shear = None
    if not args.no_shear:
        shear = shear_layer_run(hdg, hi, torch)
    batched = None
    if not args.no_batched:
        batched = batched_run(hdg, hi, torch, args.batched_instances, args.batched_steps)
    serving = None
    if not args.no_serving:
        serving = serving_run(hdg, hi, torch, args.serving_jobs, args.serving_nmax, args.serving_steps,
                              tuple(args.serving_rho), tuple(args.serving_workers))
    trace_op = None
    if not args.no_trace_op:
        trace_op = trace_operator_run(hdg, hi, torch)
    tet = None
    if not args.no_tet:
        tet = tet_run(hdg, hi, torch, args.tet_n, args.tet_steps, args.warmup, pc_lag=args.tet_pc_lag,
                      mixed=args.tet_mixed)
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline()
        log(f"cpu baseline: {cpu['value']:.1f} {cpu['unit']} ({cpu['sample']})")
    out = {
        "metric": "trace DOF-IMEX-stages/sec (FP64)",
        "value": value,
        "unit": "trace-DOF-stages/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * el / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w["workload"], "cells": ctx.ncells, "trace_dofs": ctx.nT, "degree": w["k"],
                   "imex": w["scheme"], "dt": w["dt"], "n_richardson": w["n_richardson"],
                   "trace_solver": w["trace_solver"], "rtol_trace": w["rtol_trace"],
                   "rtol_velocity": w["rtol_velocity"], "step1_precond": info.get("step1_precond"),
                   "step1_precond_lag": w["step1_precond_lag"],
                   "pcg_iterations": pcg, "trace_solves": nsolves,
                   "pcg_iterations_per_solve": round(pcg / max(nsolves, 1), 1),
                   "velocity_iterations": bicg, "velocity_solves": nvel,
                   "velocity_iterations_per_solve": round(bicg / max(nvel, 1), 1),
                   "velocity_iterations_last": vel_last,
                   "bicgstab_restarts": info["bicgstab_restarts"] - before["bicgstab_restarts"],
                   "velocity_true_residual_max": info["velocity_true_residual_max"],
                   "pcg_floor_stops": info["pcg_floor_stops"] - before["pcg_floor_stops"],
                   "pcg_floor_true_residual_max": info["pcg_floor_true_residual_max"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "mixed": mixed,
        "latency": latency,
        "shear_layer": shear,
        "batched": batched,
        "serving": serving,
        "trace_operator_out_of_cache": trace_op,
        "tetrahedra": tet,
    }
    if mixed is not None:
        mixed["speedup_vs_fp64"] = round(mixed["value"] / value, 3)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
