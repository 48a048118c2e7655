"""Seeded synthetic workloads: array layouts, incidences and per-type operator data.

The paper's own geometries (helix, Jerusalem-cross and meander reflectarrays,
section VI) and its feeds are not reproducible here, so five synthetic arrays of
the same shape stand in for them: a square lattice of elements at 0.6 wavelength
pitch, each enclosed by an identical cubic equivalent surface, a few distinct
element types, and plane-wave excitations.

What this module draws, all from numpy's PCG64 with one integer seed per
workload and one independent stream per kind of draw:
  * the element type at every lattice site (stream 0);
  * incidence angles and polarisations (stream 1);
  * the PEC scatterer of every element kind (geometry only): square plates and the
    Jerusalem cross, from which the physical per-kind blocks M_t = T_t A_t^-1 B_t and
    D_t (section II, section IV) are computed by the library (and by the oracle in
    tests);
  * seeded stand-ins for M_t and D_t, kept for kernel tests whose results do not
    depend on the operator's physics: dense complex Gaussian blocks with a fixed
    spectral scale (stream 2) and a sparse D with the pattern of the RWG / dual-RWG
    overlap and diagonally dominant seeded values (stream 3);
  * test vectors for matrix-vector products (stream 4).
Nothing here evaluates an integral, a basis function or an operator product.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .mesh import SurfaceMesh, cube_surface, jerusalem_cross, square_plate

ETA0 = 376.730313668
K0 = 2.0 * math.pi

STREAM_TYPES, STREAM_INC, STREAM_MACRO, STREAM_D, STREAM_VEC = range(5)


def rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([int(seed), int(stream)]))


@dataclass
class Workload:
    """One array problem: geometry, AIM parameters, excitation and operator data."""
    name: str
    px: int
    py: int
    box_side: float
    box_n: int
    n_types: int
    elem_type: np.ndarray            # (py*px,) int32, site m = iy*px + ix
    theta: np.ndarray                # (nrhs,) radians
    phi: np.ndarray                  # (nrhs,) radians
    pol: np.ndarray                  # (nrhs,) int32, 0 = TM (theta-hat), 1 = TE (phi-hat)
    restart: int = 50
    tol: float = 1e-6
    k: float = K0
    eta: float = ETA0
    h: float = 0.1
    order: int = 2
    r_near: float = 0.3
    pitch_cells: int = 6
    seed: int = 0
    macro_scale: float = 1.0e-3
    element_specs: tuple = ()
    _mesh: SurfaceMesh | None = field(default=None, repr=False)

    @property
    def n_elem(self) -> int:
        return self.px * self.py

    @property
    def nrhs(self) -> int:
        return int(self.theta.shape[0])

    @property
    def surface(self) -> SurfaceMesh:
        if self._mesh is None:
            self._mesh = cube_surface(self.box_side, self.box_n)
        return self._mesh

    @property
    def n_rwg(self) -> int:
        return self.surface.n_rwg

    @property
    def n_unknowns(self) -> int:
        return self.n_elem * self.n_rwg

    def elem_offset_cells(self) -> np.ndarray:
        """Integer lattice offset of every element in grid cells, (n_elem, 3)."""
        m = np.arange(self.n_elem)
        ix, iy = m % self.px, m // self.px
        return np.stack([ix * self.pitch_cells, iy * self.pitch_cells, 0 * m], axis=1).astype(np.int64)

    def elem_center(self) -> np.ndarray:
        """Element centres in wavelengths, (n_elem, 3)."""
        return self.elem_offset_cells().astype(np.float64) * self.h

    def macromodels(self) -> np.ndarray:
        return synthetic_macromodels(self.n_types, self.n_rwg, self.seed, self.macro_scale)

    def element_meshes(self) -> list[SurfaceMesh]:
        """The PEC scatterer surface of every element kind, in the element's local frame
        (geometry only): the plates and Jerusalem crosses that the equivalent boxes enclose."""
        return [element_mesh(spec) for spec in self.element_specs]

    def d_matrix(self):
        return synthetic_d_matrix(self.surface, self.seed)

    def test_vectors(self, nrhs: int | None = None, dtype=np.complex128) -> np.ndarray:
        """Complex N(0,1) + jN(0,1) vectors, (nrhs, n_unknowns)."""
        r = rng(self.seed, STREAM_VEC)
        n = self.nrhs if nrhs is None else nrhs
        z = r.standard_normal((n, self.n_unknowns)) + 1j * r.standard_normal((n, self.n_unknowns))
        return z.astype(dtype)


def element_mesh(spec: tuple) -> SurfaceMesh:
    """("plate", side, n): square plate of that side on n x n squares;
    ("jc", cell): the Jerusalem cross (arms 0.4, width 0.04, caps 0.2 x 0.02) on cell-sized squares."""
    if spec[0] == "plate":
        return square_plate(float(spec[1]), int(spec[2]))
    if spec[0] == "jc":
        return jerusalem_cross(cell=float(spec[1]))
    raise ValueError(f"unknown element {spec!r}")


def synthetic_macromodels(n_types: int, n: int, seed: int, scale: float) -> np.ndarray:
    """(n_types, n, n) complex128 dense blocks with entries of variance scale^2 / n."""
    r = rng(seed, STREAM_MACRO)
    out = np.empty((n_types, n, n), dtype=np.complex128)
    for t in range(n_types):
        out[t] = (r.standard_normal((n, n)) + 1j * r.standard_normal((n, n))) * (scale / math.sqrt(2.0 * n))
    return out


def d_pattern(mesh: SurfaceMesh) -> tuple[np.ndarray, np.ndarray]:
    """(rows, cols) of D_t: RWG n couples to n' when a triangle of n touches a vertex of edge n'."""
    vt: list[set[int]] = [set() for _ in range(mesh.n_vert)]
    for t, row in enumerate(mesh.tri):
        for v in row:
            vt[int(v)].add(t)
    tri_rwg: list[list[int]] = [[] for _ in range(mesh.n_tri)]
    for n, (_, _, tp, tm) in enumerate(mesh.rwg):
        tri_rwg[int(tp)].append(n)
        tri_rwg[int(tm)].append(n)
    rows, cols = [], []
    for npr, (va, vb, _, _) in enumerate(mesh.rwg):
        touching = vt[int(va)] | vt[int(vb)]
        nb = sorted({n for t in touching for n in tri_rwg[t]})
        rows.extend(nb)
        cols.extend([npr] * len(nb))
    rows = np.asarray(rows, dtype=np.int32)
    cols = np.asarray(cols, dtype=np.int32)
    order = np.lexsort((cols, rows))
    return rows[order], cols[order]


def synthetic_d_matrix(mesh: SurfaceMesh, seed: int):
    """Sparse D_t as (rows, cols, complex values), diagonally dominant by rows."""
    rows, cols = d_pattern(mesh)
    r = rng(seed, STREAM_D)
    edge = mesh.vert[mesh.rwg[:, 1]] - mesh.vert[mesh.rwg[:, 0]]
    length = np.sqrt((edge * edge).sum(axis=1))
    vals = 0.05 * length[rows] * length[cols] * r.uniform(-1.0, 1.0, rows.shape[0])
    diag = rows == cols
    vals[diag] = 0.5 * length[rows[diag]] ** 2 * (1.0 + 0.1 * r.uniform(-1.0, 1.0, int(diag.sum())))
    return rows, cols, vals.astype(np.complex128)


def _angles_uniform(r: np.random.Generator, nrhs: int, theta_max_deg: float = 60.0):
    th = np.empty(nrhs)
    ph = np.empty(nrhs)
    for i in range(nrhs):
        th[i] = math.radians(r.uniform(0.0, theta_max_deg))
        ph[i] = math.radians(r.uniform(0.0, 360.0))
    return th, ph


def make_workload(index: int, seed: int = 0, px: int | None = None, py: int | None = None,
                  nrhs: int | None = None) -> Workload:
    """The synthetic workloads 0..4; px/py/nrhs override the lattice and RHS count (slices)."""
    if index == 0:
        P = 2 if px is None else px
        Q = P if py is None else py
        types = np.zeros(P * Q, dtype=np.int32)
        return Workload("plates-2x2-fp64", P, Q, 0.5, 4, 1, types,
                        np.array([0.0]), np.array([0.0]), np.array([0], dtype=np.int32), seed=seed,
                        element_specs=(("plate", 0.4, 8),))
    if index == 1:
        P = 32 if px is None else px
        Q = P if py is None else py
        types = np.zeros(P * Q, dtype=np.int32)
        n = 1 if nrhs is None else nrhs
        return Workload("jc-32x32-mixed", P, Q, 0.55, 6, 1, types,
                        np.full(n, math.radians(30.0)), np.full(n, math.radians(45.0)),
                        np.zeros(n, dtype=np.int32), seed=seed, element_specs=(("jc", 0.01),))
    if index == 2:
        P = 16 if px is None else px
        Q = P if py is None else py
        types = rng(seed, STREAM_TYPES).integers(0, 3, P * Q).astype(np.int32)
        n = 64 if nrhs is None else nrhs
        th, ph = _angles_uniform(rng(seed, STREAM_INC), n)
        pol = np.array([0 if i % 2 == 1 else 1 for i in range(n)], dtype=np.int32)
        return Workload("plates-16x16-64rhs", P, Q, 0.5, 4, 3, types, th, ph, pol, seed=seed,
                        element_specs=(("plate", 0.30, 8), ("plate", 0.35, 8), ("plate", 0.40, 8)))
    if index == 4:
        P = 64 if px is None else px
        Q = P if py is None else py
        r = rng(seed, STREAM_TYPES)
        types = (r.uniform(0.0, 1.0, P * Q) < 0.10).astype(np.int32)
        n = 8 if nrhs is None else nrhs
        th = np.array([math.radians((0.0, 20.0, 40.0, 60.0)[(i // 2) % 4]) for i in range(n)])
        pol = np.array([i % 2 for i in range(n)], dtype=np.int32)
        return Workload("jc-64x64-8rhs", P, Q, 0.55, 6, 2, types, th, np.zeros(n), pol,
                        restart=80, seed=seed, element_specs=(("jc", 0.01), ("plate", 0.3, 8)))
    raise ValueError(f"no workload {index} (workload 3 is the request trace, see serving_trace)")


def standard_mom_workload(px: int = 32, py: int | None = None, cell: float = 0.01, seed: int = 0) -> Workload:
    """The 32 x 32 Jerusalem-cross array of workload 1 with each element's own PEC
    surface meshed (arms 0.4, width 0.04, caps 0.2 x 0.02 wavelength on `cell`-sized
    squares: 1,196 RWG at 0.01) instead of its equivalent box: the system a standard
    AIM-MoM solves, G J = V, for the unknown-count and iteration comparison with the
    macromodel system.  Same lattice, AIM grid, near radius and incidence as workload 1."""
    P = px
    Q = P if py is None else py
    return Workload("jc-32x32-standard-mom", P, Q, 0.0, 0, 1, np.zeros(P * Q, dtype=np.int32),
                    np.full(1, math.radians(30.0)), np.full(1, math.radians(45.0)), np.zeros(1, dtype=np.int32),
                    seed=seed, _mesh=jerusalem_cross(cell=cell))


@dataclass
class Request:
    arrival_s: float
    side: int
    elem_type: np.ndarray
    theta: np.ndarray
    phi: np.ndarray
    pol: np.ndarray


def serving_trace(seed: int = 0, n_requests: int = 2000, rate_hz: float = 20.0,
                  side_range=(4, 24), rhs_range=(1, 16)) -> list[Request]:
    """Poisson arrivals of square-array solves built from the three plate types."""
    r = rng(seed, STREAM_TYPES)
    t = 0.0
    out = []
    for _ in range(n_requests):
        t += r.exponential(1.0 / rate_hz)
        side = int(r.integers(side_range[0], side_range[1] + 1))
        nr = int(r.integers(rhs_range[0], rhs_range[1] + 1))
        types = r.integers(0, 3, side * side).astype(np.int32)
        th, ph = _angles_uniform(r, nr)
        pol = np.array([i % 2 for i in range(nr)], dtype=np.int32)
        out.append(Request(t, side, types, th, ph, pol))
    return out
