"""Triangle quadrature and RWG function geometry (section II-A, eq. J_expand / Hhat_expand).

RWG function of interior edge n with length l, shared by triangles T+ and T-
with free (opposite) vertices p+ and p-:
    Lambda_n(r) = +l / (2 A+) (r - p+)  on T+,
    Lambda_n(r) = -l / (2 A-) (r - p-)  on T-,
    div Lambda_n = +l / A+ on T+,  -l / A- on T-.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def seven_point_rule():
    """Symmetric 7-point rule of polynomial degree 5 on a triangle (Radon's rule).

    Returns barycentric points (7, 3) and weights (7,) that sum to 1, so that
    integral_T f dS ~= A * sum_q w_q f(r_q).
    """
    s15 = np.sqrt(15.0)
    a1, b1 = (9.0 - 2.0 * s15) / 21.0, (6.0 + s15) / 21.0
    a2, b2 = (9.0 + 2.0 * s15) / 21.0, (6.0 - s15) / 21.0
    w0, w1, w2 = 9.0 / 40.0, (155.0 + s15) / 1200.0, (155.0 - s15) / 1200.0
    bary = np.array([
        [1 / 3, 1 / 3, 1 / 3],
        [a1, b1, b1], [b1, a1, b1], [b1, b1, a1],
        [a2, b2, b2], [b2, a2, b2], [b2, b2, a2],
    ])
    w = np.array([w0, w1, w1, w1, w2, w2, w2])
    return bary, w


def gauss_triangle_rule(n: int):
    """Collapsed (Duffy) Gauss-Legendre product rule, exact to degree 2n-1; for pins only."""
    x, wx = np.polynomial.legendre.leggauss(n)
    u = 0.5 * (x + 1.0)
    wu = 0.5 * wx
    pts, ws = [], []
    for i in range(n):
        for j in range(n):
            s, t = u[i], u[j]
            l1 = s
            l2 = (1.0 - s) * t
            pts.append([1.0 - l1 - l2, l1, l2])
            ws.append(wu[i] * wu[j] * (1.0 - s) * 2.0)
    return np.array(pts), np.array(ws)


def tri_area_normal(tv: np.ndarray):
    """Areas and unit normals of triangles given as (..., 3, 3) vertex arrays."""
    c = np.cross(tv[..., 1, :] - tv[..., 0, :], tv[..., 2, :] - tv[..., 0, :])
    two_a = np.linalg.norm(c, axis=-1)
    return 0.5 * two_a, c / two_a[..., None]


@dataclass(frozen=True)
class RwgGeom:
    """Per-RWG geometry of one element-local surface mesh."""
    tri_vert: np.ndarray   # (n_tri, 3, 3)
    tri_area: np.ndarray   # (n_tri,)
    tp: np.ndarray         # (n_rwg,) triangle T+
    tm: np.ndarray         # (n_rwg,) triangle T-
    pp: np.ndarray         # (n_rwg, 3) free vertex of T+
    pm: np.ndarray         # (n_rwg, 3) free vertex of T-
    length: np.ndarray     # (n_rwg,)
    center: np.ndarray     # (n_rwg, 3) edge midpoint

    @property
    def n_rwg(self) -> int:
        return int(self.tp.shape[0])


def rwg_geometry(vert: np.ndarray, tri: np.ndarray, rwg: np.ndarray) -> RwgGeom:
    tv = vert[tri]
    area, _ = tri_area_normal(tv)
    va, vb, tp, tm = (rwg[:, i].astype(np.int64) for i in range(4))

    def free_vertex(t, a, b):
        rows = tri[t]
        mask = (rows != a[:, None]) & (rows != b[:, None])
        if not np.all(mask.sum(axis=1) == 1):
            raise ValueError("RWG triangle does not contain its edge")
        return vert[rows[mask]]

    pp = free_vertex(tp, va, vb)
    pm = free_vertex(tm, va, vb)
    e = vert[vb] - vert[va]
    return RwgGeom(tv, area, tp, tm, pp, pm, np.linalg.norm(e, axis=1), 0.5 * (vert[va] + vert[vb]))


def rwg_at_points(g: RwgGeom, n: np.ndarray, tri_sel: str, pts: np.ndarray):
    """Lambda_n at points on T+ (tri_sel='+') or T- ('-'); n (P,), pts (P, Q, 3)."""
    if tri_sel == "+":
        a = g.tri_area[g.tp[n]]
        return (g.length[n] / (2.0 * a))[:, None, None] * (pts - g.pp[n][:, None, :])
    a = g.tri_area[g.tm[n]]
    return -(g.length[n] / (2.0 * a))[:, None, None] * (pts - g.pm[n][:, None, :])
