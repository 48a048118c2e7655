"""Macromodel of one element (section II) and its product M_t = T A^-1 B (section III).

TEST INFRASTRUCTURE ONLY (see the package docstring): plain numpy, FP64.

For one element: PEC scatterer surface S (RWG functions Lambda_n, current J), closed
equivalent surface S^ around it (RWG functions Lambda^_n for n x H^, Buffa-Christiansen
dual functions Lambda^'_n for n x E^), n the normal pointing into S^ (section II-A).

Matrices (section II-C, eq. Gm_EJ_1 - Gm_EJ_3 on S, eq. G1 - G3 on S^):
    L-type  G^(X,Y)_ab = j omega mu0 < f_a, n x n x L g_b > = -j k eta0 int int
            [f_a . g_b - k^-2 div f_a div' g_b] G dS' dS          (f, g RWG functions)
    K-type  G^(X,E^)_ab = < f_a, -n x n x K Lambda^'_b > = < f_a, (K Lambda^'_b)_tan >
            (K X)(r) = curl int G X dS' = int grad G(r, r') x X(r') dS'
    D_ab = < Lambda^_a, n x Lambda^'_b >                               (section IV)
Then (eq. Hdiscretized1, eq. JM, eq. JABE, eq. Tm1)
    A = G^(E,J) - G^(E,H^) [G^(E^,H^)]^-1 G^(E^,J)
    B = G^(E,E^) - G^(E,H^) [G^(E^,H^)]^-1 G^(E^,E^)
    T = [G^(E^,H^)]^-1 G^(E^,J),   R = A^-1 B,   M = T R,
so that J = -R E^ and the equivalent current is J^ = T J = -M E^ (eq. Toperator), and
the final system (eq. finalsystem) of an array is (D - G M) E^ = V^.

Readings of points the paper leaves open (each checked by a pin in the tests):
  * "n pointing into S^" is the inward normal of the closed surface; it is the n of
    the dual expansion n x E^ = sum E^_n Lambda^'_n and of D.
  * The Stratton-Chu equations evaluated on S^ (eq. EFIE1, eq. EFIE3) hold in the
    exterior limit (the extinction theorem: the fields of the surface and interior
    sources vanish outside).  The K operator on its own surface then splits into its
    principal value and a jump: (K M)_tan -> PV + (1/2) n x M with n the inward
    normal, so G^(E^,E^) = PV + D / 2.  On a flat face the principal value vanishes
    (grad G and the dual function lie in the face plane, their cross product is
    normal to it), so only pairs on different faces contribute.
  * Dual functions: Buffa-Christiansen functions on the barycentric refinement of
    S^ (the paper cites three dual constructions without choosing).  The function of
    coarse edge e = (v1, v2) carries a total flux l_e from the dual cell of v1 (the
    refined triangles around v1) to that of v2, half through each of the two refined
    edges that join the edge midpoint to the adjacent barycentres, with the charge
    spread equally over the 2 N_v refined triangles of each cell; its direction is
    chosen so that n x Lambda^'_e points along Lambda^_e (positive diagonal of D).
  * Quadrature: the 7-point degree-5 rule on test and source triangles.  The static
    parts 1/(4 pi R) (L-type) and grad 1/(4 pi R) (K-type) are subtracted and
    integrated in closed form over the source triangle for every pair; test
    triangles near their source triangle are split into 4^level parts.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

from .galerkin import tri_pair_moments
from .geometry import RwgGeom, rwg_geometry, seven_point_rule, tri_area_normal

_BARY, _W = seven_point_rule()


# ---- barycentric refinement and Buffa-Christiansen dual functions -------------------

@dataclass(frozen=True)
class DualBasis:
    """Dual functions as linear pieces f(r) = (s r - q) / (2 A_t) on refined triangles t."""
    rvert: np.ndarray      # (n_rv, 3) refined vertices
    rtri: np.ndarray       # (n_rt, 3) refined triangles (counter-clockwise seen from outside)
    parent: np.ndarray     # (n_rt,) coarse triangle of each refined triangle
    fn: np.ndarray         # (P,) dual function (coarse edge index) of each piece
    tr: np.ndarray         # (P,) refined triangle of each piece
    s: np.ndarray          # (P,) net outflow of the piece (its divergence times A_t)
    q: np.ndarray          # (P, 3)

    @property
    def n_fn(self) -> int:
        return int(self.fn.max()) + 1 if self.fn.size else 0


def barycentric_refinement(vert: np.ndarray, tri: np.ndarray):
    """Split each triangle (v0, v1, v2) into six through its barycentre b and edge
    midpoints: (v0, m01, b), (m01, v1, b), (v1, m12, b), (m12, v2, b), (v2, m20, b),
    (m20, v0, b).  Returns refined vertices, triangles, parent index and the maps
    edge (sorted vertex pair) -> midpoint index, triangle -> barycentre index."""
    mids: dict[tuple[int, int], int] = {}
    pts = [v for v in vert]
    for a, b, c in tri:
        for u, w in ((a, b), (b, c), (c, a)):
            key = (int(min(u, w)), int(max(u, w)))
            if key not in mids:
                mids[key] = len(pts)
                pts.append(0.5 * (vert[u] + vert[w]))
    bary = {}
    for t, (a, b, c) in enumerate(tri):
        bary[t] = len(pts)
        pts.append((vert[a] + vert[b] + vert[c]) / 3.0)
    rtri, parent = [], []
    for t, (a, b, c) in enumerate(tri):
        m = lambda u, w: mids[(int(min(u, w)), int(max(u, w)))]  # noqa: E731
        bc = bary[t]
        for p0, p1 in ((a, m(a, b)), (m(a, b), b), (b, m(b, c)), (m(b, c), c), (c, m(c, a)), (m(c, a), a)):
            rtri.append((p0, p1, bc))
            parent.append(t)
    return np.asarray(pts), np.asarray(rtri, dtype=np.int64), np.asarray(parent, dtype=np.int64), mids, bary


def bc_dual_basis(vert: np.ndarray, tri: np.ndarray, rwg: np.ndarray) -> DualBasis:
    """Buffa-Christiansen function of every RWG edge of a closed triangulated surface."""
    rvert, rtri, parent, mids, bary = barycentric_refinement(vert, tri)
    # refined triangle by (vertex, midpoint, barycentre)
    rt_of = {}
    for i, (p0, p1, bc) in enumerate(rtri):
        v, m = (p0, p1) if p0 < vert.shape[0] else (p1, p0)
        rt_of[(int(v), int(m), int(bc))] = i
    edge_tris: dict[tuple[int, int], list[int]] = {}
    for t, (a, b, c) in enumerate(tri):
        for u, w in ((a, b), (b, c), (c, a)):
            edge_tris.setdefault((int(min(u, w)), int(max(u, w))), []).append(t)
    _, tnorm = tri_area_normal(vert[tri])
    cent = vert[tri].mean(axis=1)

    def other_edge(t: int, v: int, e: tuple[int, int]) -> tuple[int, int]:
        for u in tri[t]:
            u = int(u)
            if u != v and u not in e:
                return (min(u, v), max(u, v))
        raise ValueError("degenerate triangle")

    def cell_outflows(v: int, e: tuple[int, int], tp: int, tm: int, F0: float):
        """Outflows of the source cell of vertex v for the dual function of edge e,
        whose two triangles are tp and tm: {refined triangle: {edge (i, j): flux}}."""
        # walk around v from (v, m_e, b_tp), away from e, to (v, m_e, b_tm): two refined
        # triangles per coarse triangle, (v, m_in, b_t) then (v, m_out, b_t)
        chain = [(e, tp)]
        t, ed = tp, e
        while True:
            ed2 = other_edge(t, v, ed)
            chain.append((ed2, t))
            if t == tm:
                if ed2 != e:
                    raise ValueError("walk around a vertex did not close on its edge")
                break
            ts = edge_tris[ed2]
            t = ts[0] if ts[1] == t else ts[1]
            ed = ed2
            chain.append((ed, t))
            if len(chain) > 4 * len(tri):
                raise ValueError("open fan around a vertex (surface not closed)")
        n2 = len(chain)
        if n2 % 2:
            raise ValueError("odd number of refined triangles around a vertex")
        N = n2 // 2
        out = {}
        me = mids[e]
        for k, (ed_k, t_k) in enumerate(chain, start=1):
            m_k, b_k = mids[ed_k], bary[t_k]
            rti = rt_of[(v, m_k, b_k)]
            fl = out.setdefault(rti, {})
            # spokes: odd k crosses (v, b) to k+1 and came over (v, m); even k the reverse
            to_next = (v, b_k) if k % 2 == 1 else (v, m_k)
            to_prev = (v, m_k) if k % 2 == 1 else (v, b_k)
            if k < n2:
                fl[to_next] = fl.get(to_next, 0.0) - F0 * (N - k) / (2.0 * N)
            if k > 1:
                fl[to_prev] = fl.get(to_prev, 0.0) + F0 * (N - (k - 1)) / (2.0 * N)
            if k == 1 or k == n2:
                if m_k != me:
                    raise ValueError("chain does not end on the edge's refined triangles")
                fl[(m_k, b_k)] = fl.get((m_k, b_k), 0.0) + 0.5 * F0
        return out

    fns, trs, ss, qs = [], [], [], []
    for n, (va, vb, tp, tm) in enumerate(rwg):
        va, vb, tp, tm = int(va), int(vb), int(tp), int(tm)
        e = (min(va, vb), max(va, vb))
        le = float(np.linalg.norm(vert[vb] - vert[va]))
        ehat = (vert[vb] - vert[va]) / le
        mid = 0.5 * (vert[va] + vert[vb])
        # source cell so that n_in x Lambda' points from T+ across the edge (like Lambda^)
        n_in = -tnorm[tp]
        along = float(np.dot(np.cross(n_in, ehat), mid - cent[tp]))
        src, snk = (va, vb) if along > 0 else (vb, va)
        pieces: dict[int, dict] = {}
        for v, sign in ((src, 1.0), (snk, -1.0)):
            flows = cell_outflows(v, e, tp, tm, le)
            for rti, fl in flows.items():
                d = pieces.setdefault(rti, {})
                for key, val in fl.items():
                    d[key] = d.get(key, 0.0) + sign * val
        for rti, fl in pieces.items():
            p0, p1, p2 = (int(x) for x in rtri[rti])
            s = 0.0
            q = np.zeros(3)
            for (i, j), flux in fl.items():
                opp = ({p0, p1, p2} - {i, j}).pop()
                s += flux
                q += flux * rvert[opp]
            fns.append(n)
            trs.append(rti)
            ss.append(s)
            qs.append(q)
    return DualBasis(rvert, rtri, parent, np.asarray(fns), np.asarray(trs), np.asarray(ss), np.asarray(qs))


def dual_at_points(db: DualBasis, pts_t: np.ndarray, fn: int) -> np.ndarray:
    """Values of dual function fn at points (n_rt, Q, 3) given per refined triangle."""
    tv = db.rvert[db.rtri]
    area, _ = tri_area_normal(tv)
    out = np.zeros(pts_t.shape)
    sel = db.fn == fn
    for t, s, q in zip(db.tr[sel], db.s[sel], db.q[sel]):
        out[t] += (s * pts_t[t] - q) / (2.0 * area[t])
    return out


def dual_gram(geo: RwgGeom, db: DualBasis, n_out: np.ndarray) -> np.ndarray:
    """D_ab = < Lambda^_a, n x Lambda^'_b > with n = -n_out the inward normal (section IV).

    The integrand is quadratic on each refined triangle t, so its centroid c_t gives it
    exactly:  int_t (r - p) . (n x (s r - q)) dS / (2 A_t)
            = [ -s p . (n x c_t) + (p - c_t) . (n x q) ] / 2.
    """
    nb = geo.n_rwg
    tv = db.rvert[db.rtri]
    ct = tv.mean(axis=1)
    D = np.zeros((nb, db.n_fn))
    # RWG incidences by coarse triangle
    inc: dict[int, list[tuple[int, float, np.ndarray]]] = {}
    for a in range(nb):
        inc.setdefault(int(geo.tp[a]), []).append((a, 1.0, geo.pp[a]))
        inc.setdefault(int(geo.tm[a]), []).append((a, -1.0, geo.pm[a]))
    for b, t, s, q in zip(db.fn, db.tr, db.s, db.q):
        T = int(db.parent[t])
        n_in = -n_out[T]
        for a, sg, p in inc.get(T, ()):
            val = -s * np.dot(p, np.cross(n_in, ct[t])) + np.dot(p - ct[t], np.cross(n_in, q))
            D[a, b] += sg * geo.length[a] / (2.0 * geo.tri_area[T]) * 0.5 * val
    return D


# ---- K-type Galerkin entries --------------------------------------------------------

def static_gradient(r: np.ndarray, tv: np.ndarray) -> np.ndarray:
    """grad_r int_t 1 / |r - r'| dS' in closed form, r (P, Q, 3), tv (P, 3, 3).

    Normal part: the signed solid angle Omega of t seen from r (van Oosterom and
    Strackee), times the unit normal; in-plane part: -sum_i u_i int_{edge i} dl / R,
    with u_i the outward in-plane normal of edge i (divergence theorem on t)."""
    _, nrm = tri_area_normal(tv)
    a = tv[:, None, 0, :] - r
    b = tv[:, None, 1, :] - r
    c = tv[:, None, 2, :] - r
    la, lb, lc = (np.linalg.norm(x, axis=-1) for x in (a, b, c))
    num = np.einsum("pqk,pqk->pq", a, np.cross(b, c))
    den = (la * lb * lc + np.einsum("pqk,pqk->pq", a, b) * lc + np.einsum("pqk,pqk->pq", a, c) * lb
           + np.einsum("pqk,pqk->pq", b, c) * la)
    omega = 2.0 * np.arctan2(num, den)
    g = omega[..., None] * nrm[:, None, :]
    for i in range(3):
        va, vb = tv[:, i, :], tv[:, (i + 1) % 3, :]
        e = vb - va
        le = np.linalg.norm(e, axis=1)
        lhat = e / le[:, None]
        uhat = np.cross(lhat, nrm)
        sm = np.einsum("pqk,pk->pq", va[:, None, :] - r, lhat)
        sp = np.einsum("pqk,pk->pq", vb[:, None, :] - r, lhat)
        rr = va[:, None, :] - r
        r0 = np.sqrt(np.maximum(np.einsum("pqk,pqk->pq", rr, rr) - sm * sm, 0.0))
        f = np.arcsinh(sp / r0) - np.arcsinh(sm / r0)
        g -= f[..., None] * uhat[:, None, :]
    return g


def _smooth_grad_factor(R: np.ndarray, k: float) -> np.ndarray:
    """h(R) = d/dR [(exp(-j k R) - 1) / (4 pi R)] = [1 - (1 + j k R) exp(-j k R)] / (4 pi R^2),
    with its series -k^2/(8 pi) + j k^3 R / (12 pi) for small k R."""
    x = k * R
    small = x < 1e-3
    Rs = np.where(small, 1.0, R)
    val = (1.0 - (1.0 + 1j * k * Rs) * np.exp(-1j * k * Rs)) / (4.0 * np.pi * Rs * Rs)
    ser = -k * k / (8.0 * np.pi) + 1j * k ** 3 * R / (12.0 * np.pi)
    return np.where(small, ser, val)


def grad_green_integral(r: np.ndarray, tv: np.ndarray, k: float, level: int = 0) -> np.ndarray:
    """W(r) = int_t grad_r G(r, r') dS' for points r (P, Q, 3) and triangles tv (P, 3, 3):
    closed-form static part plus the 7-point rule on the bounded remainder, over the
    triangle split into 4^level parts (the remainder turns with the direction of r - r',
    so points close to t need the finer rule)."""
    area, _ = tri_area_normal(tv)
    bary, w = (_BARY, _W) if level == 0 else _subdivided_rule(level)
    rs = np.einsum("si,pik->psk", bary, tv)                       # (P, S, 3)
    diff = r[:, :, None, :] - rs[:, None, :, :]                    # (P, Q, S, 3)
    R = np.sqrt((diff * diff).sum(-1))
    h = _smooth_grad_factor(R, k) / np.where(R > 0, R, 1.0)
    Ws = np.einsum("s,pqs,pqsk->pqk", w, h, diff) * area[:, None, None]
    return Ws + static_gradient(r, tv) / (4.0 * np.pi)


def _subdivided_rule(level: int):
    """Barycentric points and weights (sum 1) of the 7-point rule on 4^level sub-triangles."""
    tris = [np.eye(3)]
    for _ in range(level):
        nt = []
        for T in tris:
            a, b, c = T
            ab, bc, ca = 0.5 * (a + b), 0.5 * (b + c), 0.5 * (c + a)
            nt += [np.array([a, ab, ca]), np.array([ab, b, bc]), np.array([ca, bc, c]), np.array([ab, bc, ca])]
        tris = nt
    pts = np.concatenate([_BARY @ T for T in tris])
    w = np.tile(_W, len(tris)) / len(tris)
    return pts, w


def _pair_UV(ta: np.ndarray, tb: np.ndarray, k: float, level: int = 0):
    """U = int_Ta W(r) dS, V = int_Ta W(r) x r dS for test triangles ta (P,3,3) and
    source triangles tb (P,3,3), both rules on 4^level parts."""
    bary, w = (_BARY, _W) if level == 0 else _subdivided_rule(level)
    area, _ = tri_area_normal(ta)
    rq = np.einsum("qi,pik->pqk", bary, ta)
    Wq = grad_green_integral(rq, tb, k, level)
    wa = w[None, :] * area[:, None]
    U = np.einsum("pq,pqk->pk", wa, Wq)
    V = np.einsum("pq,pqk->pk", wa, np.cross(Wq, rq))
    return U, V


def _test_features(geo: RwgGeom):
    """Sparse map (RWG a) x (test triangle T, feature alpha in {1, p_x, p_y, p_z}) with the
    RWG prefactor sigma l / (2 A_T); Lambda_a = sigma l / (2 A_T) (r - p) on T."""
    rows, cols, vals = [], [], []
    for a in range(geo.n_rwg):
        for T, sg, p in ((geo.tp[a], 1.0, geo.pp[a]), (geo.tm[a], -1.0, geo.pm[a])):
            c = sg * geo.length[a] / (2.0 * geo.tri_area[T])
            rows += [a] * 4
            cols += [4 * T + i for i in range(4)]
            vals += [c, c * p[0], c * p[1], c * p[2]]
    return np.asarray(rows), np.asarray(cols), np.asarray(vals)


def k_fill(geo_t: RwgGeom, shift_t: np.ndarray, db: DualBasis, k: float, skip_coplanar: bool,
           near_level: int = 1, chunk: int = 8) -> np.ndarray:
    """K-type entries < Lambda_a, int grad G x Lambda^'_b dS' > for every test RWG a of geo_t
    (translated by shift_t) and every dual function b (principal value: pairs of test and
    source triangles in one plane are skipped when skip_coplanar).

    Since grad_r G(r, r') is parallel to r - r', grad G x (s r' - q) = grad G x (s r - q),
    and the entry between a test feature (1 or p) and a source piece (s, q) needs only
        U = int_T W dS, V = int_T W x r dS  (W = int_t grad G dS'):
        int_T (r - p) . (W x (s r - q)) dS = -s p . V + q . V + q . (p x U).
    """
    tvt = geo_t.tri_vert + shift_t
    tvs = db.rvert[db.rtri]
    nT, nt = tvt.shape[0], tvs.shape[0]
    At, nrm_s = tri_area_normal(tvs)
    _, nrm_t = tri_area_normal(tvt)
    ct_t = tvt.mean(1)
    ct_s = tvs.mean(1)
    size_t = np.sqrt(np.max(((tvt - ct_t[:, None, :]) ** 2).sum(-1), axis=1))
    size_s = np.sqrt(np.max(((tvs - ct_s[:, None, :]) ** 2).sum(-1), axis=1))
    # source features (s, q_x, q_y, q_z) / (2 A_t) of every piece, as a dense (4 nt, n_fn) map
    nf = db.n_fn
    S = np.zeros((4 * nt, nf))
    for b, t, s, q in zip(db.fn, db.tr, db.s, db.q):
        S[4 * t, b] += s / (2.0 * At[t])
        S[4 * t + 1:4 * t + 4, b] += q / (2.0 * At[t])
    # test features
    rr, cc, vv = _test_features(geo_t)
    F = np.zeros((geo_t.n_rwg, 4 * nT))
    np.add.at(F, (rr, cc), vv)
    eps = np.zeros((3, 3, 3))
    eps[0, 1, 2] = eps[1, 2, 0] = eps[2, 0, 1] = 1.0
    eps[0, 2, 1] = eps[2, 1, 0] = eps[1, 0, 2] = -1.0
    out = np.zeros((geo_t.n_rwg, nf), dtype=np.complex128)
    for T0 in range(0, nT, chunk):
        Ts = np.arange(T0, min(T0 + chunk, nT))
        TA = np.repeat(Ts, nt)
        TB = np.tile(np.arange(nt), Ts.size)
        U = np.zeros((TA.size, 3), dtype=np.complex128)
        V = np.zeros((TA.size, 3), dtype=np.complex128)
        live = np.ones(TA.size, dtype=bool)
        if skip_coplanar:
            # principal value: a test triangle in the plane of its source triangle gives 0
            dplane = np.abs(np.einsum("pik,pk->pi", tvt[TA] - tvs[TB][:, None, 0, :], nrm_s[TB]))
            live = ~((np.max(dplane, axis=1) < 1e-12) &
                     (np.abs(np.einsum("pk,pk->p", nrm_t[TA], nrm_s[TB])) > 1 - 1e-12))
        dist = np.linalg.norm(ct_t[TA] - ct_s[TB], axis=1)
        near = live & (dist < 1.5 * (size_t[TA] + size_s[TB])) & (near_level > 0)
        far = live & ~near
        if np.any(far):
            U[far], V[far] = _pair_UV(tvt[TA[far]], tvs[TB[far]], k)
        if np.any(near):
            U[near], V[near] = _pair_UV(tvt[TA[near]], tvs[TB[near]], k, near_level)
        # pair matrix over (test feature alpha, source feature beta)
        Mp = np.zeros((TA.size, 4, 4), dtype=np.complex128)
        Mp[:, 1:, 0] = -V                                  # -s p . V
        Mp[:, 0, 1:] = V                                   # q . V
        Mp[:, 1:, 1:] = np.einsum("kij,pj->pik", eps, U)   # q . (p x U): eps_kij p_i U_j q_k
        Mp = Mp.reshape(Ts.size, nt, 4, 4).transpose(0, 2, 1, 3).reshape(4 * Ts.size, 4 * nt)
        out += F[:, 4 * T0:4 * (T0 + Ts.size)] @ (Mp @ S)
    return out


# ---- L-type Galerkin entries between two meshes -------------------------------------

def l_fill(ga: RwgGeom, shift_a: np.ndarray, gb: RwgGeom, shift_b: np.ndarray, k: float, eta: float,
           chunk: int = 8192) -> np.ndarray:
    """Dense G_ab = -j k eta int int [Lambda_a . Lambda_b - k^-2 div div'] G for every test RWG
    a of ga and source RWG b of gb (eq. Gouter1's integrand between two surfaces)."""
    ta_v = ga.tri_vert + shift_a
    tb_v = gb.tri_vert + shift_b
    na, nbt = ta_v.shape[0], tb_v.shape[0]
    TA, TB = np.meshgrid(np.arange(na), np.arange(nbt), indexing="ij")
    TA, TB = TA.ravel(), TB.ravel()
    m0 = np.empty(TA.size, dtype=np.complex128)
    m1 = np.empty((TA.size, 3), dtype=np.complex128)
    m2 = np.empty((TA.size, 3), dtype=np.complex128)
    m3 = np.empty(TA.size, dtype=np.complex128)
    for s in range(0, TA.size, chunk):
        sl = slice(s, min(s + chunk, TA.size))
        m0[sl], m1[sl], m2[sl], m3[sl] = tri_pair_moments(ta_v[TA[sl]], tb_v[TB[sl]], k)
    m0 = m0.reshape(na, nbt)
    m1 = m1.reshape(na, nbt, 3)
    m2 = m2.reshape(na, nbt, 3)
    m3 = m3.reshape(na, nbt)
    out = np.zeros((ga.n_rwg, gb.n_rwg), dtype=np.complex128)
    for sga, tai, pai in ((1.0, ga.tp, ga.pp), (-1.0, ga.tm, ga.pm)):
        pa = pai + shift_a
        for sgb, tbi, pbi in ((1.0, gb.tp, gb.pp), (-1.0, gb.tm, gb.pm)):
            pb = pbi + shift_b
            Ab = gb.tri_area[tbi]
            i0, i1 = tai[:, None], tbi[None, :]
            dot = (m3[i0, i1] - np.einsum("bk,abk->ab", pb, m2[i0, i1]) - np.einsum("ak,abk->ab", pa, m1[i0, i1])
                   + (pa @ pb.T) * m0[i0, i1])
            la = ga.length[:, None]
            lb = gb.length[None, :]
            out += sga * sgb * (la * lb / (4.0 * Ab[None, :]) * dot - la * lb / Ab[None, :] * m0[i0, i1] / (k * k))
    return -1j * k * eta * out


# ---- the macromodel ------------------------------------------------------------------

@dataclass
class Macromodel:
    GEJ: np.ndarray     # G^(E,J)    N x N     (eq. Gm_EJ_1)
    GEH: np.ndarray     # G^(E,H^)   N x N^    (eq. Gm_EJ_2)
    GEE: np.ndarray     # G^(E,E^)   N x N^    (eq. Gm_EJ_3)
    GHJ: np.ndarray     # G^(E^,J)   N^ x N    (eq. G1)
    GHH: np.ndarray     # G^(E^,H^)  N^ x N^   (eq. G2)
    GHE: np.ndarray     # G^(E^,E^)  N^ x N^   (eq. G3)
    D: np.ndarray       # N^ x N^              (section IV)
    A: np.ndarray
    B: np.ndarray
    T: np.ndarray
    R: np.ndarray       # A^-1 B (current recovery J = -R E^)
    M: np.ndarray       # T A^-1 B


def element_macromodel(scat: RwgGeom, box: RwgGeom, box_mesh, k: float, eta: float,
                       near_level: int = 1) -> Macromodel:
    """All matrices of section II for one element, in its local frame."""
    db = bc_dual_basis(box_mesh.vert, box_mesh.tri, box_mesh.rwg)
    _, n_out = tri_area_normal(box.tri_vert)
    z = np.zeros(3)
    GEJ = l_fill(scat, z, scat, z, k, eta)
    GEH = l_fill(scat, z, box, z, k, eta)
    GHJ = l_fill(box, z, scat, z, k, eta)
    GHH = l_fill(box, z, box, z, k, eta)
    GEE = k_fill(scat, z, db, k, skip_coplanar=False, near_level=near_level)
    D = dual_gram(box, db, n_out)
    GHE = k_fill(box, z, db, k, skip_coplanar=True, near_level=near_level) + 0.5 * D
    lu = sla.lu_factor(GHH)
    T = sla.lu_solve(lu, GHJ)
    A = GEJ - GEH @ T
    B = GEE - GEH @ sla.lu_solve(lu, GHE)
    R = np.linalg.solve(A, B)
    M = T @ R
    return Macromodel(GEJ, GEH, GEE, GHJ, GHH, GHE, D, A, B, T, R, M)


def mesh_geometry(mesh) -> RwgGeom:
    return rwg_geometry(mesh.vert, mesh.tri, mesh.rwg)
