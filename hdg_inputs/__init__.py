"""Seeded synthetic inputs shared by the CPU oracle tests and the GPU path.

This module holds none of the method's arithmetic: it only produces meshes
(vertex coordinates and cell->vertex connectivity) and evaluates analytic
velocity fields at points that the caller supplies.  Both the oracle and the
GPU library project those point values themselves.

Workload recipe (the paper's test setup, Section "Setup": the unit square cut
into n x n squares, each split into two right-angled triangles):

* mesh: vertex (i, j) has id j*(n+1)+i and coordinates (i/n, j/n); square
  (i, j) is cut along its "/" diagonal into the cells (v00, v10, v11) and
  (v00, v11, v01), both counter-clockwise, cell ids 2*(j*n+i) and 2*(j*n+i)+1.
* initial velocity: the curl Q = (d_y psi, -d_x psi) of the stream function
  psi = sum_m A_m sin(k_m pi x) sin(l_m pi y), m = 1..4, drawn from
  numpy.random.default_rng(seed) in the order A_m = standard_normal(),
  k_m = integers(1, 4), l_m = integers(1, 4) per term.  psi vanishes on the
  boundary, so n.Q = 0 on the walls.
* Taylor-Green vortex (Section "Taylor Green vortex"): velocity and forcing
  as printed; the pressure is the mean-zero field that satisfies the momentum
  equation (the printed pressure does not).
* batched and serving workloads (independent instances on one GPU): the
  draws of batched_instance / serving_job / serving_arrivals below.
* double-layer shear flow (Section "Double-layer shear flow"): the periodic
  square [0, 2 pi]^2 on the same n x n split-square mesh with the right/top
  vertices identified with the left/bottom ones, and the printed initial
  velocity with rho = pi/15, delta = 0.05.
* three dimensions (the method is stated for d = 2 and 3; the paper computes
  in 2D only): the unit cube cut into n^3 cubes of six tetrahedra each (the
  Kuhn split: every tetrahedron of a cube contains its main diagonal from
  the corner nearest the origin), and the initial velocity Q = curl A of the
  vector potential A_c = sum_m a_cm sin(k1 pi x) sin(k2 pi y) sin(k3 pi z),
  m = 1..4, drawn from default_rng(seed) per component c, per term, in the
  order a_cm = standard_normal(), then k1, k2, k3 = integers(1, 3).  A
  vanishes on the walls, so n.Q = 0 there.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "unit_square_mesh",
    "stream_function_params",
    "streamfunction_velocity",
    "taylor_green_velocity",
    "taylor_green_forcing",
    "taylor_green_pressure",
    "random_mesh_perturbation",
    "periodic_square_mesh",
    "shear_layer_velocity",
    "steady_vortex_velocity",
    "steady_vortex_pressure",
    "stream_function_params_from",
    "batched_instance",
    "serving_job",
    "serving_arrivals",
    "unit_cube_mesh",
    "random_cube_perturbation",
    "vector_potential_params",
    "curl_potential_velocity",
]


def unit_square_mesh(n: int):
    """Return (coords float64[(n+1)^2, 2], cells int32[2 n^2, 3])."""
    if n < 1:
        raise ValueError("n must be >= 1")
    i, j = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="xy")
    coords = np.stack([i.ravel() / n, j.ravel() / n], axis=1).astype(np.float64)
    si, sj = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    si = si.ravel()
    sj = sj.ravel()
    v00 = sj * (n + 1) + si
    v10 = v00 + 1
    v01 = v00 + (n + 1)
    v11 = v01 + 1
    cells = np.empty((2 * n * n, 3), dtype=np.int32)
    cells[0::2] = np.stack([v00, v10, v11], axis=1)
    cells[1::2] = np.stack([v00, v11, v01], axis=1)
    return coords, cells


def random_mesh_perturbation(coords: np.ndarray, n: int, amplitude: float, seed: int):
    """Move interior vertices of a unit-square mesh by a seeded random offset.

    Boundary vertices stay put, so the domain is unchanged.  amplitude is a
    fraction of the grid spacing 1/n (keep it below ~0.3 to keep cells valid).
    """
    rng = np.random.default_rng(seed)
    out = coords.copy()
    interior = (
        (coords[:, 0] > 1e-12) & (coords[:, 0] < 1 - 1e-12)
        & (coords[:, 1] > 1e-12) & (coords[:, 1] < 1 - 1e-12)
    )
    out[interior] += amplitude / n * rng.uniform(-1.0, 1.0, size=(int(interior.sum()), 2))
    return out


def periodic_square_mesh(n: int, length: float = 2.0 * np.pi, amplitude: float = 0.0, seed: int = 0):
    """Doubly periodic mesh of [0, length]^2.

    Returns (coords, cells, vertex_rep): the unit_square_mesh connectivity
    scaled by length, and for every vertex the vertex it is identified with
    (vertices on the right and top edges map to their copies on the left and
    bottom edges, the other vertices to themselves).  With amplitude > 0 each
    class of identified vertices moves by one seeded offset (a fraction of the
    spacing length/n), applied to all its copies, so the mesh stays periodic.
    n >= 3 keeps the facets of the periodic mesh distinct.
    """
    if n < 3:
        raise ValueError("periodic meshes need n >= 3")
    coords, cells = unit_square_mesh(n)
    coords = coords * length
    i, j = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="xy")
    i, j = i.ravel(), j.ravel()
    rep = ((j % n) * (n + 1) + (i % n)).astype(np.int32)
    if amplitude:
        rng = np.random.default_rng(seed)
        off = amplitude * length / n * rng.uniform(-1.0, 1.0, size=(n * n, 2))
        coords = coords + off[(j % n) * n + (i % n)]
    return coords, cells, rep


def shear_layer_velocity(x, y, rho: float = np.pi / 15.0, delta: float = 0.05):
    """Initial velocity of the double-layer shear flow on [0, 2 pi]^2 (Section
    "Double-layer shear flow"): tanh profiles of width rho about y = pi/2 and
    y = 3 pi/2, plus a transverse perturbation delta sin(x); y is taken
    modulo 2 pi."""
    y = np.mod(y, 2.0 * np.pi)
    qx = np.where(y <= np.pi, np.tanh((y - 0.5 * np.pi) / rho), np.tanh((1.5 * np.pi - y) / rho))
    return np.stack([qx, delta * np.sin(x)], axis=-1)


def steady_vortex_velocity(x, y):
    """A steady Euler solution on the 2 pi-periodic square (the Taylor-Green
    cell pattern without decay): u = (sin x cos y, -cos x sin y)."""
    return np.stack([np.sin(x) * np.cos(y), -np.cos(x) * np.sin(y)], axis=-1)


def steady_vortex_pressure(x, y):
    """Pressure of steady_vortex_velocity, (cos 2x + cos 2y)/4 (mean zero)."""
    return 0.25 * (np.cos(2.0 * x) + np.cos(2.0 * y))


def stream_function_params(seed: int, nterms: int = 4):
    """Amplitudes and wavenumbers of the seeded stream function."""
    return stream_function_params_from(np.random.default_rng(seed), nterms)


def stream_function_params_from(rng, nterms: int = 4):
    """The stream-function terms drawn from an existing generator (in the
    order amplitude, x wavenumber, y wavenumber per term)."""
    amp = np.empty(nterms)
    kx = np.empty(nterms, dtype=np.int64)
    ky = np.empty(nterms, dtype=np.int64)
    for m in range(nterms):
        amp[m] = rng.standard_normal()
        kx[m] = rng.integers(1, 4)
        ky[m] = rng.integers(1, 4)
    return amp, kx, ky


def batched_instance(j: int):
    """Instance j of the batched workload: default_rng(j) draws, in this
    order, n = integers(32, 257), k = integers(1, 5), then the 4 terms of
    the stream-function initial data.  Returns (n, k, params)."""
    rng = np.random.default_rng(j)
    n = int(rng.integers(32, 257))
    k = int(rng.integers(1, 5))
    return n, k, stream_function_params_from(rng)


def serving_job(j: int):
    """Job j of the serving workload: default_rng(10000 + j) draws
    n = round(exp(U(ln 16, ln 512))), k = integers(1, 5), then the 4
    stream-function terms.  Returns (n, k, params)."""
    rng = np.random.default_rng(10000 + j)
    n = int(round(np.exp(rng.uniform(np.log(16), np.log(512)))))
    k = int(rng.integers(1, 5))
    return n, k, stream_function_params_from(rng)


def serving_arrivals(mean_gap: float, njobs: int):
    """Arrival times of the serving workload: 0, then exponential gaps of the
    given mean from default_rng(999)."""
    gaps = np.random.default_rng(999).exponential(mean_gap, size=njobs)
    return np.concatenate([[0.0], np.cumsum(gaps[1:])])


def streamfunction_velocity(params, x: np.ndarray, y: np.ndarray):
    """Q = (d psi/dy, -d psi/dx) at the points (x, y); returns shape x.shape + (2,)."""
    amp, kx, ky = params
    qx = np.zeros(np.broadcast(x, y).shape)
    qy = np.zeros_like(qx)
    for a, k, l in zip(amp, kx, ky):
        qx += a * l * np.pi * np.sin(k * np.pi * x) * np.cos(l * np.pi * y)
        qy -= a * k * np.pi * np.cos(k * np.pi * x) * np.sin(l * np.pi * y)
    return np.stack([qx, qy], axis=-1)


def _tg_angles(x, y):
    return (2.0 * x - 1.0) * np.pi / 2.0, (2.0 * y - 1.0) * np.pi / 2.0


def taylor_green_velocity(x, y, t: float = 0.0, kappa: float = 0.5):
    a, b = _tg_angles(np.asarray(x, float), np.asarray(y, float))
    e = np.exp(-kappa * t)
    return np.stack([-e * np.cos(a) * np.sin(b), e * np.sin(a) * np.cos(b)], axis=-1)


def taylor_green_forcing(x, y, t: float, kappa: float = 0.5):
    return -kappa * taylor_green_velocity(x, y, t, kappa)


def taylor_green_pressure(x, y, t: float = 0.0, kappa: float = 0.5):
    """Mean-zero pressure that balances (Q.grad)Q for the Taylor-Green velocity."""
    a, b = _tg_angles(np.asarray(x, float), np.asarray(y, float))
    return -0.25 * np.exp(-2.0 * kappa * t) * (np.cos(2.0 * a) + np.cos(2.0 * b))


def unit_cube_mesh(n: int):
    """Kuhn split of [0, 1]^3: returns (coords float64[(n+1)^3, 3], cells
    int32[6 n^3, 4]).

    Vertex (i, j, l) has id (l*(n+1) + j)*(n+1) + i and coordinates
    (i, j, l)/n.  Cube (i, j, l) gives the cells 6*((l*n + j)*n + i) + r,
    r = 0..5, one per permutation (a, b, c) of the axes in lexicographic
    order: the path corner, corner + e_a, corner + e_a + e_b, corner + 1 along
    the cube's edges.  Each cell's last two vertices are swapped where needed
    so that every cell is positively oriented.
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    m = n + 1
    g = np.arange(n)
    I, J, L = np.meshgrid(g, g, g, indexing="ij")
    I, J, L = (a.transpose(2, 1, 0).ravel() for a in (I, J, L))  # i fastest
    corner = np.stack([I, J, L], axis=1)
    vid = lambda p: (p[:, 2] * m + p[:, 1]) * m + p[:, 0]
    perms = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
    cells = np.empty((n ** 3, 6, 4), dtype=np.int64)
    for r, perm in enumerate(perms):
        p = corner.copy()
        cells[:, r, 0] = vid(p)
        for s, ax in enumerate(perm):
            p = p.copy()
            p[:, ax] += 1
            cells[:, r, s + 1] = vid(p)
        # the orientation of a path simplex is the sign of its permutation
        odd = sum(1 for a in range(3) for b in range(a + 1, 3) if perm[a] > perm[b]) % 2
        if odd:
            cells[:, r, [2, 3]] = cells[:, r, [3, 2]]
    gi, gj, gl = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    coords = np.stack([gi.transpose(2, 1, 0).ravel(), gj.transpose(2, 1, 0).ravel(),
                       gl.transpose(2, 1, 0).ravel()], axis=1) / n
    return coords.astype(np.float64), cells.reshape(-1, 4).astype(np.int32)


def random_cube_perturbation(coords: np.ndarray, n: int, amplitude: float, seed: int):
    """Move interior vertices of a unit-cube mesh by a seeded random offset of
    at most amplitude/n per coordinate (keep amplitude below ~0.15 so that
    every tetrahedron stays positively oriented); boundary vertices stay put."""
    rng = np.random.default_rng(seed)
    out = coords.copy()
    interior = np.all((coords > 1e-12) & (coords < 1 - 1e-12), axis=1)
    out[interior] += amplitude / n * rng.uniform(-1.0, 1.0, size=(int(interior.sum()), 3))
    return out


def vector_potential_params(seed: int, nterms: int = 4):
    """Amplitudes (3, nterms) and wavenumbers (3, nterms, 3) of the seeded
    vector potential (draw order in the module header)."""
    rng = np.random.default_rng(seed)
    amp = np.empty((3, nterms))
    wav = np.empty((3, nterms, 3), dtype=np.int64)
    for c in range(3):
        for t in range(nterms):
            amp[c, t] = rng.standard_normal()
            for a in range(3):
                wav[c, t, a] = rng.integers(1, 3)
    return amp, wav


def curl_potential_velocity(params, x, y, z):
    """Q = curl A at the points (x, y, z); returns shape x.shape + (3,)."""
    amp, wav = params
    X = np.broadcast_arrays(np.asarray(x, float), np.asarray(y, float), np.asarray(z, float))
    grad = np.zeros(X[0].shape + (3, 3))  # grad[..., c, a] = d A_c / d x_a
    for c in range(3):
        for t in range(amp.shape[1]):
            k = wav[c, t] * np.pi
            s = [np.sin(k[a] * X[a]) for a in range(3)]
            co = [np.cos(k[a] * X[a]) for a in range(3)]
            grad[..., c, 0] += amp[c, t] * k[0] * co[0] * s[1] * s[2]
            grad[..., c, 1] += amp[c, t] * k[1] * s[0] * co[1] * s[2]
            grad[..., c, 2] += amp[c, t] * k[2] * s[0] * s[1] * co[2]
    return np.stack([grad[..., 2, 1] - grad[..., 1, 2],
                     grad[..., 0, 2] - grad[..., 2, 0],
                     grad[..., 1, 0] - grad[..., 0, 1]], axis=-1)
