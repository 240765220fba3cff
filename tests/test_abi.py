"""The C-ABI library loads and exports every entry point declared in
include/hdg.h (CPU only: no compute call is made)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hdg.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hdg_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib_path():
    from paper_2410_09790_amd import build, hdg
    if not os.path.exists(hdg.LIB_PATH):
        build.build()
    return hdg.LIB_PATH


def test_header_declares_the_path_entry_points():
    names = _declared()
    for required in ("hdg_create", "hdg_advance", "hdg_solve_trace", "hdg_destroy"):
        assert required in names


def test_every_declared_symbol_is_exported(lib_path):
    lib = ctypes.CDLL(lib_path)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header(lib_path):
    from paper_2410_09790_amd import hdg
    assert sorted(hdg.EXPORTS) == _declared()


def test_default_params_and_create_errors(lib_path):
    from paper_2410_09790_amd import hdg
    lib = hdg.load_library()
    p = hdg.default_params()
    assert p.degree == 1 and p.tau == 1.0 and p.n_richardson == 3 and p.rtol_trace == 1e-12
    # invalid arguments are rejected on the host before any device work
    h = ctypes.c_void_p()
    p.degree = 9
    st = lib.hdg_create(3, None, 1, None, ctypes.byref(p), None, ctypes.byref(h))
    assert st == 6 and not h.value
    assert b"degree" in lib.hdg_last_error(None)


def test_precision_parameter_is_checked_on_the_host(lib_path):
    from paper_2410_09790_amd import hdg
    lib = hdg.load_library()
    assert hdg.default_params(precision="mixed").precision == 1
    p = hdg.default_params()
    assert p.precision == 0
    p.precision = 2
    h = ctypes.c_void_p()
    st = lib.hdg_create(3, None, 1, None, ctypes.byref(p), None, ctypes.byref(h))
    assert st == 1 and not h.value
    assert b"invalid parameter" in lib.hdg_last_error(None)


def test_clockwise_mesh_is_rejected_on_the_host(lib_path):
    import numpy as np
    from paper_2410_09790_amd import hdg
    lib = hdg.load_library()
    p = hdg.default_params()
    X = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    C = np.array([[0, 2, 1]], dtype=np.int32)  # clockwise
    h = ctypes.c_void_p()
    st = lib.hdg_create(3, X.ctypes.data_as(ctypes.c_void_p), 1, C.ctypes.data_as(ctypes.c_void_p),
                        ctypes.byref(p), None, ctypes.byref(h))
    assert st == 1 and not h.value
    assert b"counter-clockwise" in lib.hdg_last_error(None)


def test_graph_parameter_is_checked_on_the_host(lib_path):
    from paper_2410_09790_amd import hdg
    lib = hdg.load_library()
    assert hdg.default_params().use_graphs == 1
    assert hdg.default_params(use_graphs=0).use_graphs == 0
    p = hdg.default_params()
    p.use_graphs = 2
    h = ctypes.c_void_p()
    st = lib.hdg_create(3, None, 1, None, ctypes.byref(p), None, ctypes.byref(h))
    assert st == 1 and not h.value
    assert b"invalid parameter" in lib.hdg_last_error(None)


def test_step1_launch_shape_is_checked_on_the_host(lib_path):
    from paper_2410_09790_amd import hdg
    lib = hdg.load_library()
    p = hdg.default_params()
    assert (p.step1_block, p.step1_xcd) == (256, 1)
    h = ctypes.c_void_p()
    for block, xcd in ((96, 1), (512, 1), (0, 1), (64, 2), (128, -1)):
        p = hdg.default_params(step1_block=block, step1_xcd=xcd)
        st = lib.hdg_create(3, None, 1, None, ctypes.byref(p), None, ctypes.byref(h))
        assert st == 1 and not h.value
        assert b"invalid parameter" in lib.hdg_last_error(None)


def test_tuned_launch_table_lookup(tmp_path):
    """The binding takes the tabulated shape of the nearest mesh size (log
    scale) for the degree; an explicit shape or a missing table leaves the
    library default."""
    import json
    from paper_2410_09790_amd import hdg
    path = str(tmp_path / "t.json")
    rows = [{"degree": 2, "ncells": 512, "step1_block": 64, "step1_xcd": 0},
            {"degree": 2, "ncells": 131072, "step1_block": 256, "step1_xcd": 1},
            {"degree": 3, "ncells": 512, "step1_block": 128, "step1_xcd": 1}]
    with open(path, "w") as f:
        json.dump({"entries": rows}, f)
    assert hdg.tuned_launch(2, 600, path) == {"step1_block": 64, "step1_xcd": 0}
    assert hdg.tuned_launch(2, 8000, path) == {"step1_block": 64, "step1_xcd": 0}  # log midpoint 8192
    assert hdg.tuned_launch(2, 8400, path) == {"step1_block": 256, "step1_xcd": 1}
    assert hdg.tuned_launch(3, 10 ** 6, path) == {"step1_block": 128, "step1_xcd": 1}
    assert hdg.tuned_launch(4, 512, path) == {}
    assert hdg.tuned_launch(1, 512, str(tmp_path / "none.json")) == {}
    # the committed table covers every degree with valid shapes
    if os.path.exists(hdg.LAUNCH_TABLE):
        with open(hdg.LAUNCH_TABLE) as f:
            tab = json.load(f)["entries"]
        assert sorted({r["degree"] for r in tab}) == [1, 2, 3, 4]
        assert all(r["step1_block"] in (64, 128, 256) and r["step1_xcd"] in (0, 1) for r in tab)


def test_params_struct_layout_matches_the_header(tmp_path):
    """The ctypes mirror of hdg_params has the C compiler's size and offsets."""
    import shutil
    import subprocess
    from paper_2410_09790_amd import hdg
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    names = [f[0] for f in hdg.Params._fields_]
    src = tmp_path / "layout.c"
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"hdg.h\"\nint main(void) {\n"
                   "  printf(\"%zu\\n\", sizeof(hdg_params));\n"
                   + "".join(f"  printf(\"%zu\\n\", offsetof(hdg_params, {n}));\n" for n in names)
                   + "  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert out[0] == ctypes.sizeof(hdg.Params)
    assert out[1:] == [getattr(hdg.Params, n).offset for n in names]


def _create_periodic(lib, X, C, rep):
    from paper_2410_09790_amd import hdg
    import numpy as np
    p = hdg.default_params()
    X = np.ascontiguousarray(X, dtype=np.float64)
    C = np.ascontiguousarray(C, dtype=np.int32)
    rep = np.ascontiguousarray(rep, dtype=np.int32)
    h = ctypes.c_void_p()
    st = lib.hdg_create_periodic(X.shape[0], X.ctypes.data_as(ctypes.c_void_p), C.shape[0],
                                 C.ctypes.data_as(ctypes.c_void_p), rep.ctypes.data_as(ctypes.c_void_p),
                                 ctypes.byref(p), None, ctypes.byref(h))
    return st, h


def test_bad_periodic_meshes_are_rejected_on_the_host(lib_path):
    """Mesh errors are found before any device work (no GPU needed)."""
    import hdg_inputs as hi
    from paper_2410_09790_amd import hdg
    lib = hdg.load_library()
    X, C, rep = hi.periodic_square_mesh(3)
    bad = rep.copy()
    bad[5] = X.shape[0]  # out of range
    st, h = _create_periodic(lib, X, C, bad)
    assert st == 1 and not h.value and b"vertex_rep" in lib.hdg_last_error(None)
    # 2 x 2 squares: two edges of a row become one facet of four cells
    X2, C2 = hi.unit_square_mesh(2)
    i, j = np.meshgrid(np.arange(3), np.arange(3), indexing="xy")
    rep2 = ((j.ravel() % 2) * 3 + (i.ravel() % 2)).astype(np.int32)
    st, h = _create_periodic(lib, X2, C2, rep2)
    assert st == 1 and not h.value and b"non-manifold" in lib.hdg_last_error(None)
    # a right-edge vertex moved without its left copy: identified facets differ in length
    X3 = X.copy()
    X3[2 * 4 - 1, 0] += 0.1  # vertex (3, 1)
    st, h = _create_periodic(lib, X3, C, rep)
    assert st == 1 and not h.value and b"differ in length" in lib.hdg_last_error(None)


def test_footprint_estimate_runs_on_the_host(lib_path):
    """hdg_footprint_bytes needs no device: it grows with the mesh and the
    degree, FP32 cell-matrix storage lowers it, and bad meshes are refused."""
    import hdg_inputs as hi
    from paper_2410_09790_amd import hdg
    X, C = hi.unit_square_mesh(16)
    X2, C2 = hi.unit_square_mesh(32)
    f1 = hdg.footprint_bytes(X, C, 1e-3, degree=1)
    f2 = hdg.footprint_bytes(X2, C2, 1e-3, degree=1)
    f3 = hdg.footprint_bytes(X2, C2, 1e-3, degree=3)
    f3m = hdg.footprint_bytes(X2, C2, 1e-3, degree=3, precision="mixed")
    assert 0 < f1 < f2 < f3 and f3m < f3
    Xp, Cp, rep = hi.periodic_square_mesh(8)
    assert hdg.footprint_bytes(Xp, Cp, 0.04, vertex_rep=rep, degree=2, imex="ssp3_433") > 0
    with pytest.raises(hdg.HDGError):
        hdg.footprint_bytes(X, C[:, ::-1], 1e-3)  # clockwise cells


@pytest.mark.parametrize("n,periodic", [(1, False), (5, False), (4, True)])
def test_library_mesh_follows_the_documented_recipe(lib_path, n, periodic):
    """hdg_mesh_square (host only) gives the documented split-square mesh,
    the same arrays as the seeded input module."""
    import hdg_inputs as hi
    from paper_2410_09790_amd import hdg
    X, C, rep = hdg.mesh_square(n, 2.0 * np.pi if periodic else 1.0, periodic)
    if periodic:
        Xr, Cr, repr_ = hi.periodic_square_mesh(n)
        assert np.array_equal(rep, repr_)
    else:
        Xr, Cr = hi.unit_square_mesh(n)
        assert np.array_equal(rep, np.arange((n + 1) ** 2))
    assert np.allclose(X, Xr, rtol=0, atol=1e-14) and np.array_equal(C, Cr)
    with pytest.raises(hdg.HDGError):
        hdg.mesh_square(2, 1.0, True)


def test_library_mesh_other_diagonal(lib_path):
    """The "\\" split: same vertices, counter-clockwise cells, the same facet
    count; the host mesh check (via hdg_footprint_bytes) accepts it."""
    from paper_2410_09790_amd import hdg
    X, C, _ = hdg.mesh_square(5, 1.0, diagonal=1)
    X0, C0, _ = hdg.mesh_square(5, 1.0)
    assert np.array_equal(X, X0) and not np.array_equal(C, C0)
    v = X[C]
    det = (v[:, 1, 0] - v[:, 0, 0]) * (v[:, 2, 1] - v[:, 0, 1]) - (v[:, 2, 0] - v[:, 0, 0]) * (v[:, 1, 1] - v[:, 0, 1])
    assert (det > 0).all() and np.allclose(det, (1 / 5) ** 2)
    assert hdg.footprint_bytes(X, C, 1e-3, degree=2) > 0
    Xp, Cp, rep = hdg.mesh_square(4, 2.0, periodic=True, diagonal=1)
    assert hdg.footprint_bytes(Xp, Cp, 1e-3, vertex_rep=rep, degree=1) > 0


def test_library_cube_mesh_follows_the_documented_recipe(lib_path):
    """hdg_mesh_unit_cube (host only) gives the Kuhn mesh of the input recipe."""
    import hdg_inputs as hi
    from paper_2410_09790_amd import hdg
    for n in (1, 2, 3):
        X, C = hdg.mesh_unit_cube(n)
        X0, C0 = hi.unit_cube_mesh(n)
        assert np.array_equal(X, X0) and np.array_equal(C, C0)
    with pytest.raises(hdg.HDGError):
        hdg.mesh_unit_cube(0)


def test_tetrahedra_parameters_are_checked_on_the_host(lib_path):
    """dim, degree, precision and mesh orientation on tetrahedra are checked
    before any device work (no GPU needed)."""
    import hdg_inputs as hi
    from paper_2410_09790_amd import hdg
    lib = hdg.load_library()
    assert hdg.default_params().dim == 2
    X, C = hi.unit_cube_mesh(1)
    h = ctypes.c_void_p()

    def create(p, X=X, C=C):
        X = np.ascontiguousarray(X, dtype=np.float64)
        C = np.ascontiguousarray(C, dtype=np.int32)
        return lib.hdg_create(X.shape[0], X.ctypes.data_as(ctypes.c_void_p), C.shape[0],
                              C.ctypes.data_as(ctypes.c_void_p), ctypes.byref(p), None, ctypes.byref(h))

    assert create(hdg.default_params(dim=4)) == 1 and b"dim" in lib.hdg_last_error(None)
    assert create(hdg.default_params(dim=3, degree=3)) == 6 and b"tetrahedra" in lib.hdg_last_error(None)
    bad = C.copy()
    bad[:, [2, 3]] = bad[:, [3, 2]]  # negatively oriented
    assert create(hdg.default_params(dim=3, degree=2), C=bad) == 1
    assert b"positively oriented" in lib.hdg_last_error(None)
    assert not h.value
