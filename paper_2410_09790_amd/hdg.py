"""Thin ctypes binding of libhdg.so (see include/hdg.h for the contract).

Argument marshalling only: every numerical step runs in the HIP library.
torch supplies device memory (float64 CUDA tensors) and the HIP stream.
Loading fails loudly when the library has not been built.  Unless the caller
sets it, the launch shape of the Step I operator is taken from the table that
autotune.py measures (launch_table.json beside this file; library default
when it is absent).
"""
from __future__ import annotations

import ctypes
import json
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhdg.so")
# launch shapes of the Step I operator measured by autotune.py
LAUNCH_TABLE = os.path.join(_HERE, "launch_table.json")

IMEX = {"imex_euler": 0, "ars222": 1, "ars233": 2, "ssp2_332": 3, "ssp3_433": 4}
TRACE_SOLVER = {"jacobi_pcg": 0, "mg_pcg": 1}
PRESSURE = {"reconstruct": 0, "first_order": 1}
PRECISION = {"fp64": 0, "mixed": 1}
STEP2 = {"A": 0, "printed": 0, "B": 1, "stage_solve": 1}
STATUS = {0: "OK", 1: "INVALID_ARG", 2: "OUT_OF_MEMORY", 3: "DEVICE", 4: "NOT_CONVERGED", 5: "BAD_STATE",
          6: "UNSUPPORTED"}

EXPORTS = [
    "hdg_default_params", "hdg_create", "hdg_create_periodic", "hdg_destroy", "hdg_footprint_bytes",
    "hdg_batch_create", "hdg_batch_size", "hdg_batch_advance", "hdg_batch_destroy", "hdg_advance_stages",
    "hdg_pending_stage", "hdg_eval_points", "hdg_eval_points_noalloc", "hdg_mesh_square", "hdg_mesh_unit_cube", "hdg_set_tracer", "hdg_get_tracer",
    "hdg_cg_project", "hdg_tracer_rate", "hdg_last_error", "hdg_sizes", "hdg_cell_points",
    "hdg_facet_points", "hdg_set_forcing", "hdg_set_time", "hdg_get_time", "hdg_set_velocity_from_points", "hdg_set_state", "hdg_get_state", "hdg_advance", "hdg_solve_trace",
    "hdg_trace_matvec", "hdg_bdm_project", "hdg_weak_divergence", "hdg_momentum_residual",
    "hdg_tentative_velocity", "hdg_step1_precond", "hdg_constraint_residual", "hdg_reconstruct_pressure", "hdg_profile", "hdg_get_info",
]


class Params(ctypes.Structure):
    _fields_ = [
        ("degree", ctypes.c_int),
        ("tau", ctypes.c_double),
        ("alpha", ctypes.c_double),
        ("delta_up", ctypes.c_double),
        ("imex", ctypes.c_int),
        ("n_richardson", ctypes.c_int),
        ("trace_solver", ctypes.c_int),
        ("rtol_trace", ctypes.c_double),
        ("rtol_velocity", ctypes.c_double),
        ("max_it_trace", ctypes.c_int),
        ("max_it_velocity", ctypes.c_int),
        ("pressure_update", ctypes.c_int),
        ("idr_s", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("use_graphs", ctypes.c_int),
        ("step1_block", ctypes.c_int),
        ("step1_xcd", ctypes.c_int),
        ("step1_precond", ctypes.c_int),
        ("step2_reading", ctypes.c_int),
        ("step1_precond_lag", ctypes.c_int),
        ("dim", ctypes.c_int),
    ]


class HDGError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libhdg.so (raises if it is missing) and declare the signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2410_09790_amd/build.py")
    lib = ctypes.CDLL(path)
    P, D, I64, I = ctypes.c_void_p, ctypes.c_double, ctypes.c_int64, ctypes.c_int
    sig = {
        "hdg_default_params": (None, [ctypes.POINTER(Params)]),
        "hdg_create": (I, [I64, P, I64, P, ctypes.POINTER(Params), P, ctypes.POINTER(P)]),
        "hdg_create_periodic": (I, [I64, P, I64, P, P, ctypes.POINTER(Params), P, ctypes.POINTER(P)]),
        "hdg_footprint_bytes": (I, [I64, P, I64, P, P, ctypes.POINTER(Params), D, ctypes.POINTER(I64)]),
        "hdg_batch_create": (I, [I, P, ctypes.POINTER(P)]),
        "hdg_batch_size": (I, [P]),
        "hdg_batch_advance": (I, [P, P, P, P]),
        "hdg_batch_destroy": (None, [P]),
        "hdg_advance_stages": (I, [P, D, I]),
        "hdg_pending_stage": (I, [P]),
        "hdg_eval_points": (I, [P, P, I, P, P]),
        "hdg_eval_points_noalloc": (I, [P, P, I, P, P]),
        "hdg_mesh_unit_cube": (I, [I, P, P]),
        "hdg_mesh_square": (I, [I, D, I, I, P, P, P]),
        "hdg_set_tracer": (I, [P, P]),
        "hdg_get_tracer": (I, [P, P]),
        "hdg_cg_project": (I, [P, P, P]),
        "hdg_tracer_rate": (I, [P, P, P, P]),
        "hdg_destroy": (None, [P]),
        "hdg_last_error": (ctypes.c_char_p, [P]),
        "hdg_sizes": (I, [P, P, I]),
        "hdg_cell_points": (I, [P, P]),
        "hdg_facet_points": (I, [P, P]),
        "hdg_set_forcing": (I, [P, P, P, D]),
        "hdg_set_time": (I, [P, D]),
        "hdg_get_time": (D, [P]),
        "hdg_set_velocity_from_points": (I, [P, P]),
        "hdg_set_state": (I, [P, P, P, P]),
        "hdg_get_state": (I, [P, P, P, P]),
        "hdg_advance": (I, [P, D, I]),
        "hdg_solve_trace": (I, [P, D, P, P, P, P, P, P]),
        "hdg_trace_matvec": (I, [P, D, P, P]),
        "hdg_bdm_project": (I, [P, P, P]),
        "hdg_weak_divergence": (I, [P, P, P]),
        "hdg_momentum_residual": (I, [P, D, P, P, P, P, P, P]),
        "hdg_tentative_velocity": (I, [P, D, P, P, P]),
        "hdg_step1_precond": (I, [P, D, P, P, P]),
        "hdg_constraint_residual": (I, [P, P, P, P, P, P]),
        "hdg_reconstruct_pressure": (I, [P, P, P, P]),
        "hdg_profile": (I, [P, I]),
        "hdg_get_info": (I, [P, ctypes.c_char_p, ctypes.c_size_t]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def default_params(**kw) -> Params:
    lib = load_library()
    p = Params()
    lib.hdg_default_params(ctypes.byref(p))
    for key, val in kw.items():
        if key == "imex" and isinstance(val, str):
            val = IMEX[val]
        elif key == "trace_solver" and isinstance(val, str):
            val = TRACE_SOLVER[val]
        elif key == "pressure_update" and isinstance(val, str):
            val = PRESSURE[val]
        elif key == "precision" and isinstance(val, str):
            val = PRECISION[val]
        elif key == "step2_reading" and isinstance(val, str):
            val = STEP2[val]
        setattr(p, key, val)
    return p


_launch_cache: dict = {}


def tuned_launch(degree: int, ncells: int, path: str = LAUNCH_TABLE):
    """{"step1_block", "step1_xcd"} that autotune.py measured fastest for this
    degree at the tabulated mesh nearest to ncells (in log scale), or {} when
    the table is missing or holds no entry for the degree."""
    if path not in _launch_cache:
        try:
            with open(path) as f:
                _launch_cache[path] = json.load(f)["entries"]
        except FileNotFoundError:
            _launch_cache[path] = []
    rows = [r for r in _launch_cache[path] if r["degree"] == int(degree)]
    if not rows:
        return {}
    best = min(rows, key=lambda r: abs(np.log(r["ncells"]) - np.log(max(int(ncells), 1))))
    return {"step1_block": int(best["step1_block"]), "step1_xcd": int(best["step1_xcd"])}


def _with_launch(params: dict, ncells: int) -> dict:
    """params with the tuned Step I launch shape filled in unless given."""
    if "step1_block" in params or "step1_xcd" in params:
        return params
    return {**params, **tuned_launch(params.get("degree", 1), ncells)}


def _ptr(t):
    import torch
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("expected a contiguous float64 CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """One HDG-IMEX instance on the current CUDA (HIP) device."""

    def __init__(self, coords, cells, stream=None, vertex_rep=None, **params):
        import torch
        self._lib = load_library()
        coords = np.ascontiguousarray(coords, dtype=np.float64)
        cells = np.ascontiguousarray(cells, dtype=np.int32)
        rep = None if vertex_rep is None else np.ascontiguousarray(vertex_rep, dtype=np.int32)
        if rep is not None and rep.shape != (coords.shape[0],):
            raise ValueError("vertex_rep needs one entry per vertex")
        if coords.ndim != 2 or coords.shape[1] not in (2, 3) or cells.shape[1:] != (coords.shape[1] + 1,):
            raise ValueError("coords [nv][d] and cells [nc][d+1] with d = 2 or 3")
        params = {"dim": coords.shape[1], **params}
        self.dim = params["dim"]
        self.params = default_params(**(_with_launch(params, cells.shape[0]) if self.dim == 2 else params))
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.device = stream.device
        h = ctypes.c_void_p()
        st = self._lib.hdg_create_periodic(
            coords.shape[0], coords.ctypes.data_as(ctypes.c_void_p), cells.shape[0],
            cells.ctypes.data_as(ctypes.c_void_p), None if rep is None else rep.ctypes.data_as(ctypes.c_void_p),
            ctypes.byref(self.params), ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h))
        if st != 0:
            raise HDGError(st, self._lib.hdg_last_error(None).decode())
        self._h = h
        out = (ctypes.c_int64 * 8)()
        self._check(self._lib.hdg_sizes(self._h, out, 8))
        (self.ncells, self.nfacets, self.nQ, self.nP, self.nT, self.nq_cell, self.nverts, self.degree) = list(out)

    def _check(self, st):
        if st != 0:
            raise HDGError(st, self._lib.hdg_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self._lib.hdg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _empty(self, n):
        import torch
        return torch.empty(n, dtype=torch.float64, device=self.device)

    # ------------------------------------------------------------- state
    def cell_points(self) -> np.ndarray:
        xy = np.empty((self.ncells, self.nq_cell, self.dim))
        self._check(self._lib.hdg_cell_points(self._h, xy.ctypes.data_as(ctypes.c_void_p)))
        return xy

    def facet_points(self) -> np.ndarray:
        nqf = (3 * self.degree + 5) // 2
        if self.dim == 3:  # the facet rule on triangles: nqf^2 points
            xy = np.empty((self.ncells, 4, nqf * nqf, 3))
        else:
            xy = np.empty((self.ncells, 3, nqf, 2))
        self._check(self._lib.hdg_facet_points(self._h, xy.ctypes.data_as(ctypes.c_void_p)))
        return xy

    def set_forcing(self, cell_values, facet_values, decay: float):
        """f(x, t) = exp(-decay t) f0(x), f0 given at cell_points() and facet_points();
        None removes the forcing."""
        if cell_values is None:
            self._check(self._lib.hdg_set_forcing(self._h, None, None, float(decay)))
            return
        import torch
        cv = torch.as_tensor(np.ascontiguousarray(cell_values, dtype=np.float64)).to(self.device)
        fv = torch.as_tensor(np.ascontiguousarray(facet_values, dtype=np.float64)).to(self.device)
        self._check(self._lib.hdg_set_forcing(self._h, _ptr(cv), _ptr(fv), float(decay)))

    @property
    def time(self) -> float:
        return float(self._lib.hdg_get_time(self._h))

    @time.setter
    def time(self, t: float):
        self._check(self._lib.hdg_set_time(self._h, float(t)))

    def set_velocity_from_points(self, values):
        import torch
        v = torch.as_tensor(np.ascontiguousarray(values, dtype=np.float64)).to(self.device)
        if v.numel() != self.ncells * self.nq_cell * self.dim:
            raise ValueError(f"expected values at the cell points, shape ({self.ncells}, {self.nq_cell}, {self.dim})")
        self._check(self._lib.hdg_set_velocity_from_points(self._h, _ptr(v)))

    def set_state(self, Q, p, lam):
        self._check(self._lib.hdg_set_state(self._h, _ptr(Q), _ptr(p), _ptr(lam)))

    def get_state(self):
        Q, p, lam = self._empty(self.nQ), self._empty(self.nP), self._empty(self.nT)
        self._check(self._lib.hdg_get_state(self._h, _ptr(Q), _ptr(p), _ptr(lam)))
        return Q, p, lam

    def advance(self, dt: float, nsteps: int):
        self._check(self._lib.hdg_advance(self._h, float(dt), int(nsteps)))

    def advance_stages(self, dt: float, nstages: int):
        self._check(self._lib.hdg_advance_stages(self._h, float(dt), int(nstages)))

    @property
    def pending_stage(self) -> int:
        return int(self._lib.hdg_pending_stage(self._h))

    def set_tracer(self, values):
        """Tracer from its values at cell_points() (ncells, nq_cell); None switches it off."""
        import torch
        if values is None:
            self._check(self._lib.hdg_set_tracer(self._h, None))
            return
        v = torch.as_tensor(np.ascontiguousarray(values, dtype=np.float64)).to(self.device)
        self._check(self._lib.hdg_set_tracer(self._h, _ptr(v)))

    def get_tracer(self):
        q = self._empty(self.nP)
        self._check(self._lib.hdg_get_tracer(self._h, _ptr(q)))
        return q

    def cg_project(self, Q):
        U = self._empty(self.nQ)
        self._check(self._lib.hdg_cg_project(self._h, _ptr(Q), _ptr(U)))
        return U

    def tracer_rate(self, Q, q):
        out = self._empty(self.nP)
        self._check(self._lib.hdg_tracer_rate(self._h, _ptr(Q), _ptr(q), _ptr(out)))
        return out

    def eval_points(self, xy_ref):
        """Velocity (ncells, npts, 2) and pressure (ncells, npts) at reference points."""
        pts = np.ascontiguousarray(xy_ref, dtype=np.float64).reshape(-1, 2)
        Qo = self._empty(self.ncells * pts.shape[0] * 2)
        po = self._empty(self.ncells * pts.shape[0])
        self._check(self._lib.hdg_eval_points(self._h, pts.ctypes.data_as(ctypes.c_void_p), pts.shape[0], _ptr(Qo),
                                              _ptr(po)))
        return Qo.view(self.ncells, pts.shape[0], 2), po.view(self.ncells, pts.shape[0])

    def eval_points_noalloc(self, xy_ref, Qo, po):
        """eval_points into caller buffers (device tensors of ncells * npts * 2 and
        ncells * npts doubles, either may be None), with no device allocation
        inside the library."""
        pts = np.ascontiguousarray(xy_ref, dtype=np.float64).reshape(-1, 2)
        self._check(self._lib.hdg_eval_points_noalloc(self._h, pts.ctypes.data_as(ctypes.c_void_p), pts.shape[0],
                                                      _ptr(Qo), _ptr(po)))

    # ------------------------------------------------------- path pieces
    def solve_trace(self, c, Fw=None, Fpsi=None, Fmu=None):
        U, p, lam = self._empty(self.nQ), self._empty(self.nP), self._empty(self.nT)
        self._check(self._lib.hdg_solve_trace(self._h, float(c), _ptr(Fw), _ptr(Fpsi), _ptr(Fmu), _ptr(U), _ptr(p),
                                              _ptr(lam)))
        return U, p, lam

    def trace_matvec(self, c, x):
        y = self._empty(self.nT)
        self._check(self._lib.hdg_trace_matvec(self._h, float(c), _ptr(x), _ptr(y)))
        return y

    def bdm_project(self, Q):
        out = self._empty(self.nQ)
        self._check(self._lib.hdg_bdm_project(self._h, _ptr(Q), _ptr(out)))
        return out

    def weak_divergence(self, F):
        out = self._empty(self.nP)
        self._check(self._lib.hdg_weak_divergence(self._h, _ptr(F), _ptr(out)))
        return out

    def momentum_residual(self, adt, r, Qstar, Q, p, lam):
        out = self._empty(self.nQ)
        self._check(self._lib.hdg_momentum_residual(self._h, float(adt), _ptr(r), _ptr(Qstar), _ptr(Q), _ptr(p),
                                                    _ptr(lam), _ptr(out)))
        return out

    def tentative_velocity(self, adt, Qstar, rhs):
        out = self._empty(self.nQ)
        self._check(self._lib.hdg_tentative_velocity(self._h, float(adt), _ptr(Qstar), _ptr(rhs), _ptr(out)))
        return out

    def step1_precond(self, adt, Qstar, r):
        """z = B r, the facet-patch preconditioner of the mass-scaled Step I operator."""
        out = self._empty(self.nQ)
        self._check(self._lib.hdg_step1_precond(self._h, float(adt), _ptr(Qstar), _ptr(r), _ptr(out)))
        return out

    def constraint_residual(self, Q, p=None, lam=None):
        """Gamma(psi, mu, Q, p, lam) as dual vectors (Fpsi, Fmu)."""
        Fpsi, Fmu = self._empty(self.nP), self._empty(self.nT)
        self._check(self._lib.hdg_constraint_residual(self._h, _ptr(Q), _ptr(p), _ptr(lam), _ptr(Fpsi), _ptr(Fmu)))
        return Fpsi, Fmu

    def reconstruct_pressure(self, Q):
        p, lam = self._empty(self.nP), self._empty(self.nT)
        self._check(self._lib.hdg_reconstruct_pressure(self._h, _ptr(Q), _ptr(p), _ptr(lam)))
        return p, lam

    def profile(self, every: int):
        """Time every `every`-th launch of each kernel class (0: stop timing)."""
        self._check(self._lib.hdg_profile(self._h, int(every)))

    def info(self) -> dict:
        buf = ctypes.create_string_buffer(1 << 16)
        self._check(self._lib.hdg_get_info(self._h, buf, len(buf)))
        return json.loads(buf.value.decode())


def footprint_bytes(coords, cells, dt: float, vertex_rep=None, **params) -> int:
    """Device bytes a Context with these arguments holds after its first
    advance(dt, .), plus its transient assembly scratch (host-side estimate,
    no device work): the admission figure of the serving loop."""
    lib = load_library()
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    cells = np.ascontiguousarray(cells, dtype=np.int32)
    rep = None if vertex_rep is None else np.ascontiguousarray(vertex_rep, dtype=np.int32)
    p = default_params(**_with_launch(params, cells.shape[0]))
    out = ctypes.c_int64()
    st = lib.hdg_footprint_bytes(coords.shape[0], coords.ctypes.data_as(ctypes.c_void_p), cells.shape[0],
                                 cells.ctypes.data_as(ctypes.c_void_p),
                                 None if rep is None else rep.ctypes.data_as(ctypes.c_void_p), ctypes.byref(p),
                                 float(dt), ctypes.byref(out))
    if st != 0:
        raise HDGError(st, lib.hdg_last_error(None).decode())
    return int(out.value)


class Batch:
    """Non-owning group of distinct Contexts advanced together: hdg_batch_advance
    runs the members on host threads, so members on distinct streams overlap
    on the device."""

    def __init__(self, contexts):
        self._lib = load_library()
        self.contexts = list(contexts)
        arr = (ctypes.c_void_p * len(self.contexts))(*[c._h.value for c in self.contexts])
        h = ctypes.c_void_p()
        st = self._lib.hdg_batch_create(len(self.contexts), arr, ctypes.byref(h))
        if st != 0:
            raise HDGError(st, self._lib.hdg_last_error(None).decode())
        self._h = h

    def advance(self, dt, nsteps):
        """dt, nsteps: one value per member (or scalars).  Raises on the first
        failed member; returns the per-member statuses."""
        n = len(self.contexts)
        dts = np.ascontiguousarray(np.broadcast_to(np.asarray(dt, dtype=np.float64), (n,)))
        nst = np.ascontiguousarray(np.broadcast_to(np.asarray(nsteps, dtype=np.int32), (n,)))
        status = np.zeros(n, dtype=np.int32)
        st = self._lib.hdg_batch_advance(self._h, dts.ctypes.data_as(ctypes.c_void_p),
                                         nst.ctypes.data_as(ctypes.c_void_p), status.ctypes.data_as(ctypes.c_void_p))
        if st != 0:
            bad = int(np.nonzero(status)[0][0])
            raise HDGError(st, f"member {bad}: " + self._lib.hdg_last_error(self.contexts[bad]._h).decode())
        return status

    def close(self):
        if getattr(self, "_h", None):
            self._lib.hdg_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mesh_unit_cube(n: int):
    """The library's Kuhn mesh of the unit cube (6 n^3 tetrahedra): (coords, cells)."""
    lib = load_library()
    coords = np.empty(((n + 1) ** 3, 3), dtype=np.float64)
    cells = np.empty((6 * n ** 3, 4), dtype=np.int32)
    st = lib.hdg_mesh_unit_cube(int(n), coords.ctypes.data_as(ctypes.c_void_p), cells.ctypes.data_as(ctypes.c_void_p))
    if st != 0:
        raise HDGError(st, "invalid mesh size")
    return coords, cells


def mesh_square(n: int, length: float = 1.0, periodic: bool = False, diagonal: int = 0):
    """The library's split-square mesh of [0, length]^2 (diagonal 0: "/", 1: "\\"):
    (coords, cells, vertex_rep)."""
    lib = load_library()
    coords = np.empty(((n + 1) ** 2, 2), dtype=np.float64)
    cells = np.empty((2 * n * n, 3), dtype=np.int32)
    rep = np.empty((n + 1) ** 2, dtype=np.int32)
    st = lib.hdg_mesh_square(int(n), float(length), int(diagonal), int(bool(periodic)),
                             coords.ctypes.data_as(ctypes.c_void_p), cells.ctypes.data_as(ctypes.c_void_p),
                             rep.ctypes.data_as(ctypes.c_void_p))
    if st != 0:
        raise HDGError(st, "invalid mesh size")
    return coords, cells, rep
