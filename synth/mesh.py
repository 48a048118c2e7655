"""Structured triangle meshes and RWG edge tables (geometry and topology only).

This module builds the discretisation that the method starts from (section II-A:
RWG functions on the equivalent box surface), but it evaluates no basis function,
integral or operator: it only produces vertex coordinates, triangle vertex lists
and, for every interior edge, the pair of triangles that share it.

Conventions shared by every consumer of these tables:
  * lengths are in wavelengths, each element is centred at its own origin;
  * triangles are listed counter-clockwise seen from outside the closed surface
    (their right-hand normal points outwards);
  * a unit square of a face, with corners P(i,j) in the face's (u, v) frame, is
    split along the diagonal P(i,j)-P(i+1,j+1) into (P00, P10, P11) and
    (P00, P11, P01);
  * an RWG row is (v_a, v_b, T+, T-): the edge's end vertices with v_a < v_b, and
    the two triangles sharing that edge with T+ < T-.  Rows are sorted by
    (v_a, v_b).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class SurfaceMesh:
    vert: np.ndarray  # (n_vert, 3) float64
    tri: np.ndarray   # (n_tri, 3) int32
    rwg: np.ndarray   # (n_rwg, 4) int32: v_a, v_b, T+, T-

    @property
    def n_vert(self) -> int:
        return int(self.vert.shape[0])

    @property
    def n_tri(self) -> int:
        return int(self.tri.shape[0])

    @property
    def n_rwg(self) -> int:
        return int(self.rwg.shape[0])


def rwg_table(tri: np.ndarray) -> np.ndarray:
    """Interior edges of a triangle list as (v_a, v_b, T+, T-) rows.

    Edges with a single adjacent triangle (open boundary) carry no RWG function.
    An edge shared by more than two triangles is rejected (non-manifold).
    """
    owners: dict[tuple[int, int], list[int]] = {}
    for t, (a, b, c) in enumerate(np.asarray(tri, dtype=np.int64)):
        for u, v in ((a, b), (b, c), (c, a)):
            key = (int(min(u, v)), int(max(u, v)))
            owners.setdefault(key, []).append(t)
    rows = []
    for key in sorted(owners):
        ts = owners[key]
        if len(ts) == 1:
            continue
        if len(ts) != 2:
            raise ValueError(f"non-manifold edge {key} shared by {len(ts)} triangles")
        rows.append((key[0], key[1], min(ts), max(ts)))
    return np.asarray(rows, dtype=np.int32).reshape(-1, 4)


def cube_surface(side: float, n: int) -> SurfaceMesh:
    """Closed surface of an axis-aligned cube of the given side, n x n squares per face.

    Vertices are shared between faces, so the surface is closed and every edge is
    interior: 6 n^2 + 2 vertices, 12 n^2 triangles, 18 n^2 RWG functions.
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    index: dict[tuple[int, int, int], int] = {}
    verts: list[tuple[float, float, float]] = []

    def vid(i: int, j: int, k: int) -> int:
        key = (i, j, k)
        if key not in index:
            index[key] = len(verts)
            verts.append(tuple(-0.5 * side + side * q / n for q in key))
        return index[key]

    # (fixed axis, fixed value, u axis, v axis) with u x v along the outward normal.
    faces = (
        (0, n, 1, 2), (0, 0, 2, 1),
        (1, n, 2, 0), (1, 0, 0, 2),
        (2, n, 0, 1), (2, 0, 1, 0),
    )
    tris: list[tuple[int, int, int]] = []
    for fixed, val, ua, va in faces:
        def P(i: int, j: int) -> int:
            c = [0, 0, 0]
            c[fixed] = val
            c[ua] = i
            c[va] = j
            return vid(*c)
        for j in range(n):
            for i in range(n):
                p00, p10, p11, p01 = P(i, j), P(i + 1, j), P(i + 1, j + 1), P(i, j + 1)
                tris.append((p00, p10, p11))
                tris.append((p00, p11, p01))
    tri = np.asarray(tris, dtype=np.int32)
    return SurfaceMesh(np.asarray(verts, dtype=np.float64), tri, rwg_table(tri))


def square_plate(side: float, n: int, z: float = 0.0) -> SurfaceMesh:
    """Zero-thickness square plate in the plane z, n x n squares, normal +z."""
    if n < 1:
        raise ValueError("n must be >= 1")
    g = -0.5 * side + side * np.arange(n + 1) / n
    vert = np.array([(g[i], g[j], z) for j in range(n + 1) for i in range(n + 1)], dtype=np.float64)

    def P(i: int, j: int) -> int:
        return j * (n + 1) + i

    tris = []
    for j in range(n):
        for i in range(n):
            tris.append((P(i, j), P(i + 1, j), P(i + 1, j + 1)))
            tris.append((P(i, j), P(i + 1, j + 1), P(i, j + 1)))
    tri = np.asarray(tris, dtype=np.int32)
    return SurfaceMesh(vert, tri, rwg_table(tri))


def vertex_triangles(mesh: SurfaceMesh) -> list[list[int]]:
    """For every vertex, the triangles that contain it (topology only)."""
    out: list[list[int]] = [[] for _ in range(mesh.n_vert)]
    for t, row in enumerate(mesh.tri):
        for v in row:
            out[int(v)].append(t)
    return out


def icosphere(radius: float, level: int) -> SurfaceMesh:
    """Closed triangulated sphere: an icosahedron whose faces are split in four `level`
    times, vertices pushed onto the sphere (20 * 4**level triangles)."""
    t = (1.0 + 5.0 ** 0.5) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    verts = [np.asarray(p, dtype=np.float64) / np.linalg.norm(p) for p in v]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
             (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5),
             (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(level):
        mid: dict[tuple[int, int], int] = {}

        def midpoint(a: int, b: int) -> int:
            key = (min(a, b), max(a, b))
            if key not in mid:
                p = verts[a] + verts[b]
                verts.append(p / np.linalg.norm(p))
                mid[key] = len(verts) - 1
            return mid[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    vert = radius * np.asarray(verts)
    tri = np.asarray(faces, dtype=np.int32)
    # counter-clockwise seen from outside: the right-hand normal points away from the centre
    p = vert[tri]
    nrm = np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0])
    flip = np.einsum("ij,ij->i", nrm, p.mean(1)) < 0
    tri[flip] = tri[flip][:, [0, 2, 1]]
    return SurfaceMesh(vert, tri, rwg_table(tri))


def jerusalem_cross(arm: float = 0.4, width: float = 0.04, cap_len: float = 0.2, cap_w: float = 0.02,
                    cell: float = 0.01) -> SurfaceMesh:
    """Zero-thickness Jerusalem-cross plate in the plane z = 0, normal +z: two crossed
    arms (arm x width) with an end cap (cap_w along the arm, cap_len across it) centred
    on each arm end.  The shape is rasterised on square cells of side `cell` centred on
    the origin (a cell is kept when its centre lies in the shape) and every kept cell
    is split in two triangles as in square_plate."""
    half = int(round(0.5 * (arm + cap_w) / cell)) + 1
    centres = (np.arange(-half, half) + 0.5) * cell

    def inside(x: float, y: float) -> bool:
        eps = 1e-9
        if abs(y) <= 0.5 * width + eps and abs(x) <= 0.5 * arm + eps:
            return True
        if abs(x) <= 0.5 * width + eps and abs(y) <= 0.5 * arm + eps:
            return True
        for s in (-1.0, 1.0):
            if abs(x - s * 0.5 * arm) <= 0.5 * cap_w + eps and abs(y) <= 0.5 * cap_len + eps:
                return True
            if abs(y - s * 0.5 * arm) <= 0.5 * cap_w + eps and abs(x) <= 0.5 * cap_len + eps:
                return True
        return False

    n = 2 * half
    keep = [(i, j) for j in range(n) for i in range(n) if inside(centres[i], centres[j])]
    ids: dict[tuple[int, int], int] = {}
    verts = []

    def P(i: int, j: int) -> int:
        if (i, j) not in ids:
            ids[(i, j)] = len(verts)
            verts.append(((i - half) * cell, (j - half) * cell, 0.0))
        return ids[(i, j)]

    tris = []
    for i, j in keep:
        p00, p10, p11, p01 = P(i, j), P(i + 1, j), P(i + 1, j + 1), P(i, j + 1)
        tris.append((p00, p10, p11))
        tris.append((p00, p11, p01))
    tri = np.asarray(tris, dtype=np.int32)
    return SurfaceMesh(np.asarray(verts, dtype=np.float64), tri, rwg_table(tri))
