"""Galerkin EFIE entries between RWG functions (section IV eq. Gouter1, section II-C operator L).

Entry between test RWG a and source RWG b:
    G_ab = j omega mu0 < Lambda_a, n x n x [L Lambda_b] >
         = -j k eta0  int int [Lambda_a . Lambda_b - k^-2 div Lambda_a div' Lambda_b] G(R) dS' dS
with G(R) = exp(-j k R) / (4 pi R).  The n x n x acting on a tangential testing
function flips the sign; the k^-2 grad div part is moved onto the testing function
by integration by parts (RWG functions have no normal flux at their boundary).

Quadrature (the paper does not state one): the 7-point degree-5 rule on the test
triangle and on the source triangle, with the static part 1/(4 pi R) of the kernel
subtracted and integrated in closed form over the source triangle for every pair.
The closed forms for int 1/R dS' and int (r' - rho)/R dS' over a flat triangle are
the standard potential integrals of Wilton et al. (1984) and Graglia (1993).
"""
from __future__ import annotations

import numpy as np

from .geometry import RwgGeom, seven_point_rule, tri_area_normal

_BARY, _W = seven_point_rule()


def static_potentials(r: np.ndarray, tv: np.ndarray):
    """Closed-form I1 = int_T 1/|r-r'| dS' and Iv = int_T (r' - rho)/|r-r'| dS'.

    r: (P, Q, 3) observation points, tv: (P, 3, 3) source triangles.  rho is the
    projection of r onto the triangle's plane.  Returns I1 (P, Q), Iv (P, Q, 3).
    """
    _, nrm = tri_area_normal(tv)                          # (P, 3)
    v0 = tv[:, 0, :]
    d = np.einsum("pqk,pk->pq", r - v0[:, None, :], nrm)  # signed height
    rho = r - d[..., None] * nrm[:, None, :]
    ad = np.abs(d)
    I1 = np.zeros(d.shape)
    Iv = np.zeros(r.shape)
    for i in range(3):
        va = tv[:, i, :]
        vb = tv[:, (i + 1) % 3, :]
        e = vb - va
        le = np.linalg.norm(e, axis=1)
        lhat = e / le[:, None]
        uhat = np.cross(lhat, nrm)                        # in-plane, points out of the triangle
        sm = np.einsum("pqk,pk->pq", va[:, None, :] - rho, lhat)
        sp = np.einsum("pqk,pk->pq", vb[:, None, :] - rho, lhat)
        t0 = np.einsum("pqk,pk->pq", va[:, None, :] - rho, uhat)
        r0sq = t0 * t0 + d * d
        rp = np.sqrt(r0sq + sp * sp)
        rm = np.sqrt(r0sq + sm * sm)
        r0 = np.sqrt(r0sq)
        tiny = r0 <= 1e-14 * le[:, None]
        r0s = np.where(tiny, 1.0, r0)
        f = np.where(tiny, 0.0, np.arcsinh(sp / r0s) - np.arcsinh(sm / r0s))
        beta = (np.arctan2(t0 * sp, r0sq + ad * rp) - np.arctan2(t0 * sm, r0sq + ad * rm))
        I1 += t0 * f - ad * beta
        Iv += 0.5 * (r0sq * f + sp * rp - sm * rm)[..., None] * uhat[:, None, :]
    return I1, Iv


def smooth_kernel(R: np.ndarray, k: float) -> np.ndarray:
    """(exp(-j k R) - 1) / (4 pi R), with its limit -j k / (4 pi) at R = 0."""
    Rs = np.where(R > 0.0, R, 1.0)
    half = np.sin(0.5 * k * Rs)
    val = (-2.0 * half * half - 1j * np.sin(k * Rs)) / (4.0 * np.pi * Rs)
    return np.where(R > 0.0, val, -1j * k / (4.0 * np.pi))


def tri_pair_moments(ta: np.ndarray, tb: np.ndarray, k: float):
    """Moments of the source potential over test-triangle quadrature points.

    With K0(r) = int_Tb G dS' and K1(r) = int_Tb G r' dS', and r_q the test points:
        m0 = sum_q w_q K0(r_q),  m1 = sum_q w_q K1(r_q),
        m2 = sum_q w_q r_q K0(r_q),  m3 = sum_q w_q r_q . K1(r_q).
    ta, tb: (P, 3, 3).  Returns m0 (P,), m1 (P,3), m2 (P,3), m3 (P,).
    """
    rq = np.einsum("qi,pik->pqk", _BARY, ta)                  # (P, 7, 3) test points
    rs = np.einsum("qi,pik->pqk", _BARY, tb)                  # (P, 7, 3) source points
    ab, _ = tri_area_normal(tb)
    diff = rq[:, :, None, :] - rs[:, None, :, :]              # (P, 7, 7, 3)
    R = np.sqrt((diff * diff).sum(axis=-1))
    gs = smooth_kernel(R, k) * (_W[None, None, :] * ab[:, None, None])
    K0 = gs.sum(axis=2)
    K1 = np.einsum("pqs,psk->pqk", gs, rs)
    I1, Iv = static_potentials(rq, tb)
    _, nrm = tri_area_normal(tb)
    d = np.einsum("pqk,pk->pq", rq - tb[:, None, 0, :], nrm)
    rho = rq - d[..., None] * nrm[:, None, :]
    K0 = K0 + I1 / (4.0 * np.pi)
    K1 = K1 + (Iv + rho * I1[..., None]) / (4.0 * np.pi)
    m0 = np.einsum("q,pq->p", _W, K0)
    m1 = np.einsum("q,pqk->pk", _W, K1)
    m2 = np.einsum("q,pqk,pq->pk", _W, rq, K0)
    m3 = np.einsum("q,pqk,pqk->p", _W, rq, K1)
    return m0, m1, m2, m3


def efie_pairs(ga: RwgGeom, shift_a: np.ndarray, a: np.ndarray,
               gb: RwgGeom, shift_b: np.ndarray, b: np.ndarray,
               k: float, eta: float, chunk: int = 4096) -> np.ndarray:
    """G_ab for the listed pairs: test RWG a[i] of mesh ga translated by shift_a[i],
    source RWG b[i] of mesh gb translated by shift_b[i].  Returns (P,) complex."""
    a = np.asarray(a, dtype=np.int64)
    b = np.asarray(b, dtype=np.int64)
    shift_a = np.broadcast_to(np.asarray(shift_a, dtype=np.float64), (a.shape[0], 3))
    shift_b = np.broadcast_to(np.asarray(shift_b, dtype=np.float64), (b.shape[0], 3))
    out = np.zeros(a.shape[0], dtype=np.complex128)
    for s in range(0, a.shape[0], chunk):
        sl = slice(s, min(s + chunk, a.shape[0]))
        aa, bb, sa, sb = a[sl], b[sl], shift_a[sl], shift_b[sl]
        acc = np.zeros(aa.shape[0], dtype=np.complex128)
        for sga, ta_idx, pa_all in ((+1.0, ga.tp, ga.pp), (-1.0, ga.tm, ga.pm)):
            ta = ga.tri_vert[ta_idx[aa]] + sa[:, None, :]
            Aa = ga.tri_area[ta_idx[aa]]
            pa = pa_all[aa] + sa
            for sgb, tb_idx, pb_all in ((+1.0, gb.tp, gb.pp), (-1.0, gb.tm, gb.pm)):
                tb = gb.tri_vert[tb_idx[bb]] + sb[:, None, :]
                Ab = gb.tri_area[tb_idx[bb]]
                pb = pb_all[bb] + sb
                m0, m1, m2, m3 = tri_pair_moments(ta, tb, k)
                # sum_q A_a w_q Lambda_a(r_q) . int Lambda_b G  with both RWG prefactors
                dot = (m3 - np.einsum("pk,pk->p", pb, m2) - np.einsum("pk,pk->p", pa, m1)
                       + np.einsum("pk,pk->p", pa, pb) * m0)
                vec = Aa * (ga.length[aa] / (2.0 * Aa)) * (gb.length[bb] / (2.0 * Ab)) * dot
                sca = Aa * (ga.length[aa] / Aa) * (gb.length[bb] / Ab) * m0
                acc += sga * sgb * (vec - sca / (k * k))
        out[sl] = -1j * k * eta * acc
    return out


def efie_dense(geo: RwgGeom, shifts: np.ndarray, k: float, eta: float, rows=None) -> np.ndarray:
    """Dense G over every (element, RWG) pair of an array; brute force for small arrays.

    Moments are computed once per (test triangle, source triangle) pair and then
    combined into RWG entries; `rows` restricts the test functions (global indices).
    """
    ne, nb, nt = shifts.shape[0], geo.n_rwg, geo.tri_vert.shape[0]
    tv = (geo.tri_vert[None, :, :, :] + shifts[:, None, None, :]).reshape(ne * nt, 3, 3)
    area = np.tile(geo.tri_area, ne)
    idx = np.arange(ne * nb)
    rows = idx if rows is None else np.asarray(rows, dtype=np.int64)
    ea, ra = np.divmod(rows, nb)
    eb, rb = np.divmod(idx, nb)
    # triangles needed on the test side
    tri_a = np.unique(np.concatenate([ea * nt + geo.tp[ra], ea * nt + geo.tm[ra]]))
    pos = -np.ones(ne * nt, dtype=np.int64)
    pos[tri_a] = np.arange(tri_a.size)
    TA, TB = np.meshgrid(tri_a, np.arange(ne * nt), indexing="ij")
    TA, TB = TA.ravel(), TB.ravel()
    m0 = np.empty(TA.size, dtype=np.complex128)
    m1 = np.empty((TA.size, 3), dtype=np.complex128)
    m2 = np.empty((TA.size, 3), dtype=np.complex128)
    m3 = np.empty(TA.size, dtype=np.complex128)
    for s in range(0, TA.size, 8192):
        sl = slice(s, min(s + 8192, TA.size))
        m0[sl], m1[sl], m2[sl], m3[sl] = tri_pair_moments(tv[TA[sl]], tv[TB[sl]], k)
    out = np.zeros((rows.size, idx.size), dtype=np.complex128)
    ntot = ne * nt
    for sga, tai, pai in ((1.0, geo.tp, geo.pp), (-1.0, geo.tm, geo.pm)):
        ta = ea * nt + tai[ra]
        pa = pai[ra] + shifts[ea]
        for sgb, tbi, pbi in ((1.0, geo.tp, geo.pp), (-1.0, geo.tm, geo.pm)):
            tb = eb * nt + tbi[rb]
            pb = pbi[rb] + shifts[eb]
            Ab = area[tb]
            p = pos[ta][:, None] * ntot + tb[None, :]
            dot = (m3[p] - np.einsum("bk,abk->ab", pb, m2[p]) - np.einsum("ak,abk->ab", pa, m1[p])
                   + (pa @ pb.T) * m0[p])
            la = geo.length[ra][:, None]
            lb = geo.length[rb][None, :]
            out += sga * sgb * (la * lb / (4.0 * Ab[None, :]) * dot - la * lb / Ab[None, :] * m0[p] / (k * k))
    return -1j * k * eta * out
