"""Independent references for Galerkin EFIE entries between RWG functions (eq. Gouter1's
integrand), shared by the oracle's pins and the library's host checks: a high-order
product rule of the full kernel for separated pairs, and the oracle's pair rule applied
on 4^levels sub-triangles of both triangles for touching pairs."""
import math

import numpy as np

from oracle.geometry import gauss_triangle_rule


def plain_entry(geo, a, sa, b, sb, k, eta, n=20):
    """G_ab by a high-order product rule of the full kernel (well separated pairs only)."""
    bary, w = gauss_triangle_rule(n)
    tot = 0.0
    for sga, ta, pa in ((1, geo.tp, geo.pp), (-1, geo.tm, geo.pm)):
        tva = geo.tri_vert[ta[a]] + sa
        Aa = geo.tri_area[ta[a]]
        ra = bary @ tva
        la = sga * geo.length[a] / (2 * Aa) * (ra - (pa[a] + sa))
        da = sga * geo.length[a] / Aa
        for sgb, tb, pb in ((1, geo.tp, geo.pp), (-1, geo.tm, geo.pm)):
            tvb = geo.tri_vert[tb[b]] + sb
            Ab = geo.tri_area[tb[b]]
            rb = bary @ tvb
            lb = sgb * geo.length[b] / (2 * Ab) * (rb - (pb[b] + sb))
            db = sgb * geo.length[b] / Ab
            R = np.linalg.norm(ra[:, None, :] - rb[None, :, :], axis=-1)
            G = np.exp(-1j * k * R) / (4 * math.pi * R)
            integrand = (la @ lb.T - da * db / (k * k)) * G
            tot += Aa * Ab * np.einsum("i,j,ij->", w, w, integrand)
    return -1j * k * eta * tot


def refined_entry(geo, a, b, k, eta, levels=2):
    """G_ab with the test and source triangles split into 4^levels pieces (same rule per piece)."""
    from oracle.galerkin import tri_pair_moments

    def split(t):
        out = [t]
        for _ in range(levels):
            nxt = []
            for v in out:
                m01, m12, m20 = 0.5 * (v[0] + v[1]), 0.5 * (v[1] + v[2]), 0.5 * (v[2] + v[0])
                nxt += [np.array([v[0], m01, m20]), np.array([m01, v[1], m12]),
                        np.array([m20, m12, v[2]]), np.array([m01, m12, m20])]
            out = nxt
        return np.array(out)

    tot = 0.0
    for sga, ta, pa in ((1, geo.tp, geo.pp), (-1, geo.tm, geo.pm)):
        Aa = geo.tri_area[ta[a]]
        for sgb, tb, pb in ((1, geo.tp, geo.pp), (-1, geo.tm, geo.pm)):
            Ab = geo.tri_area[tb[b]]
            A_sub = split(geo.tri_vert[ta[a]])
            B_sub = split(geo.tri_vert[tb[b]])
            I, J = np.meshgrid(np.arange(len(A_sub)), np.arange(len(B_sub)), indexing="ij")
            ta_s, tb_s = A_sub[I.ravel()], B_sub[J.ravel()]
            m0, m1, m2, m3 = tri_pair_moments(ta_s, tb_s, k)
            aa = 0.5 * np.linalg.norm(np.cross(ta_s[:, 1] - ta_s[:, 0], ta_s[:, 2] - ta_s[:, 0]), axis=1)
            P, Pb = pa[a], pb[b]
            dot = m3 - m2 @ Pb - m1 @ P + np.dot(P, Pb) * m0
            # the sub-triangle's own area weights its quadrature points
            tot += sga * sgb * np.sum(aa * (geo.length[a] / (2 * Aa)) * (geo.length[b] / (2 * Ab)) * dot
                                      - aa * (geo.length[a] / Aa) * (geo.length[b] / Ab) * m0 / (k * k))
    return -1j * k * eta * tot
