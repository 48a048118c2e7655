"""Pins of the oracle's macromodel half (section II, section III, section IV) to things
other than itself: the definition of the Buffa-Christiansen functions, closed forms and
finite differences, brute-force quadrature, the reciprocity of the L-type blocks, the
factor identity M = T A^-1 B, the single-element (M = 1) reduction to the direct EFIE
of the scatterer, the equivalence theorem (section II-B), and the RCS of a 2 x 2 array
against the dense method of moments on the original plates (the paper's own validation,
section VI).  CPU only."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle.excitation import plane_wave_rhs, radiated_field, radiated_near_field, rcs_db
from oracle.galerkin import efie_dense, static_potentials
from oracle.geometry import gauss_triangle_rule, seven_point_rule, tri_area_normal
from oracle.macromodel import (bc_dual_basis, dual_at_points, dual_gram, element_macromodel, grad_green_integral,
                               k_fill, mesh_geometry, static_gradient)
from synth import make_workload
from synth.mesh import cube_surface, square_plate

K0 = 2.0 * np.pi
ETA = 376.730313668


@pytest.fixture(scope="module")
def elem4():
    """The 0.4-wavelength plate (8 x 8) in the 0.5-wavelength cube (4 x 4 per face)."""
    plate, box = square_plate(0.4, 8), cube_surface(0.5, 4)
    gs, gb = mesh_geometry(plate), mesh_geometry(box)
    return plate, box, gs, gb, element_macromodel(gs, gb, box, K0, ETA)


def _m1_errors(gs, gb, mm, incidences):
    """Single-element macromodel solve (D - G_self M) E = V, J = -R E, against the direct
    EFIE of the plate G^(E,J) J = V_plate; and the far field of T J against that of J."""
    c = np.zeros((1, 3))
    rh = np.array([[np.sin(a) * np.cos(b), np.sin(a) * np.sin(b), np.cos(a)]
                   for a in np.linspace(0, np.pi, 13) for b in (0.0, 0.7, 1.9)])
    errs, eqs = [], []
    for th, ph, pol in incidences:
        Jd = np.linalg.solve(mm.GEJ, plane_wave_rhs(gs, c, th, ph, pol, K0))
        E = np.linalg.solve(mm.D - mm.GHH @ mm.M, plane_wave_rhs(gb, c, th, ph, pol, K0))
        errs.append(np.linalg.norm(-mm.R @ E - Jd) / np.linalg.norm(Jd))
        Fj = radiated_field(gs, c, Jd, rh, K0, ETA)
        Fh = radiated_field(gb, c, mm.T @ Jd, rh, K0, ETA)
        eqs.append(np.linalg.norm(Fh - Fj) / np.linalg.norm(Fj))
    return max(errs), max(eqs)


# ---- dual functions ------------------------------------------------------------------

def test_bc_functions_follow_their_definition():
    """Each dual function: zero net charge; charge +l_e / (2 N_v) on every refined triangle of
    one vertex cell and -l_e / (2 N_v) on the other; normal flux continuous across every
    refined edge (a linear combination of refined RWG functions is divergence-conforming);
    no flux through the boundary of its support."""
    mesh = cube_surface(0.5, 3)
    db = bc_dual_basis(mesh.vert, mesh.tri, mesh.rwg)
    nv = mesh.n_vert
    valence = np.zeros(nv, dtype=int)
    for t in mesh.tri:
        valence[t] += 1
    tv = db.rvert[db.rtri]
    area, _ = tri_area_normal(tv)
    for b in range(mesh.n_rwg):
        sel = np.flatnonzero(db.fn == b)
        le = np.linalg.norm(mesh.vert[mesh.rwg[b, 1]] - mesh.vert[mesh.rwg[b, 0]])
        assert abs(db.s[sel].sum()) < 1e-14
        # the coarse vertex of each refined triangle decides its cell
        for i in sel:
            v = int(db.rtri[db.tr[i]][db.rtri[db.tr[i]] < nv][0])
            assert v in mesh.rwg[b, :2]
            assert abs(abs(db.s[i]) - le / (2 * valence[v])) < 1e-14
        # normal flux across refined edges, from the pieces' values at edge midpoints
        flux = {}
        for i in sel:
            t = db.tr[i]
            p = tv[t]
            for j in range(3):
                a, c = p[j], p[(j + 1) % 3]
                key = tuple(sorted((int(db.rtri[t][j]), int(db.rtri[t][(j + 1) % 3]))))
                mid = 0.5 * (a + c)
                e = c - a
                nrm = np.cross(e, np.cross(p[1] - p[0], p[2] - p[0]))
                nrm /= np.linalg.norm(nrm)
                f = (db.s[i] * mid - db.q[i]) / (2 * area[t])
                flux[key] = flux.get(key, 0.0) + float(np.dot(f, nrm)) * np.linalg.norm(e)
        assert max(abs(v) for v in flux.values()) < 1e-13


def test_dual_gram_matches_pointwise_quadrature():
    """D from the closed centroid formula equals the 7-point rule applied to the functions'
    pointwise values (both integrands are quadratic, so both are exact); D is well
    conditioned, and each dual function is nearly orthogonal to its own RWG function."""
    mesh = cube_surface(0.5, 3)
    geo = mesh_geometry(mesh)
    db = bc_dual_basis(mesh.vert, mesh.tri, mesh.rwg)
    _, n_out = tri_area_normal(geo.tri_vert)
    D = dual_gram(geo, db, n_out)
    bary, w = seven_point_rule()
    tv = db.rvert[db.rtri]
    area, _ = tri_area_normal(tv)
    pts = np.einsum("qi,tik->tqk", bary, tv)
    for b in (0, 17, 55, 100):
        f = dual_at_points(db, pts, b)                      # (n_rt, 7, 3)
        for a in range(geo.n_rwg):
            val = 0.0
            for T, sg, p in ((geo.tp[a], 1.0, geo.pp[a]), (geo.tm[a], -1.0, geo.pm[a])):
                for t in np.flatnonzero(db.parent == T):
                    lam = sg * geo.length[a] / (2 * geo.tri_area[T]) * (pts[t] - p)
                    n_in = -n_out[T]
                    val += area[t] * np.sum(w[:, None] * lam * np.cross(n_in, f[t]))
            assert abs(val - D[a, b]) < 1e-15
    assert np.all(np.diag(D) > 0)
    assert np.linalg.cond(D) < 10.0


# ---- K-type kernel integrals ----------------------------------------------------------

def test_static_gradient_is_the_gradient_of_the_pinned_potential():
    """grad int 1/R: closed form against central differences of the closed-form potential
    (itself pinned against Duffy quadrature in test_oracle_pins), off and near the plane."""
    rng = np.random.default_rng(1)
    tv = rng.standard_normal((3, 3, 3)) * 0.1
    r = rng.standard_normal((3, 5, 3)) * 0.1
    g = static_gradient(r, tv)
    h = 1e-6
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        fd = (static_potentials(r + e, tv)[0] - static_potentials(r - e, tv)[0]) / (2 * h)
        assert np.max(np.abs(g[..., k] - fd)) < 1e-8 * np.max(np.abs(g))


def test_grad_green_integral_against_gauss_quadrature():
    """int_t grad G dS' against a 60 x 60 collapsed Gauss rule at points 0.05-0.2 away from
    a triangle about 0.15 across: the closed-form static part is exact; the bounded
    remainder needs the subdivided rule (level 2) near the triangle."""
    rng = np.random.default_rng(4)
    tv = rng.standard_normal((1, 3, 3)) * 0.1
    _, nrm = tri_area_normal(tv)
    c = tv[0].mean(0)
    r = (c + np.outer([0.05, 0.1, 0.2], nrm[0]) + rng.standard_normal((3, 3)) * 0.02)[None]
    W0 = grad_green_integral(r, tv, K0)
    W2 = grad_green_integral(r, tv, K0, level=2)
    pts, w = gauss_triangle_rule(60)
    A, _ = tri_area_normal(tv[0])
    rs = pts @ tv[0]
    for q in range(3):
        d = r[0, q] - rs
        R = np.linalg.norm(d, axis=1)
        gp = -(1 + 1j * K0 * R) * np.exp(-1j * K0 * R) / (4 * np.pi * R ** 2)
        ref = A * np.sum(w[:, None] * d / R[:, None] * gp[:, None], axis=0)
        assert np.max(np.abs(W2[0, q] - ref)) < 1e-4 * np.max(np.abs(ref))
        assert np.max(np.abs(W0[0, q] - ref)) < 1e-2 * np.max(np.abs(ref))


def test_k_fill_against_brute_force():
    """Entries <Lambda_a, int grad G x Lambda'_b dS'> between a plate's RWG functions and a
    box's dual functions against plain 12 x 12 Gauss rules on both triangles, the cross
    product formed at every point pair (no closed forms, no identities)."""
    plate, box = square_plate(0.4, 4), cube_surface(0.5, 2)
    gs, gb = mesh_geometry(plate), mesh_geometry(box)
    db = bc_dual_basis(box.vert, box.tri, box.rwg)
    K = k_fill(gs, np.zeros(3), db, K0, skip_coplanar=False)
    pts, w = gauss_triangle_rule(12)
    tv_r = db.rvert[db.rtri]
    area_r, _ = tri_area_normal(tv_r)
    rng = np.random.default_rng(2)
    for a, b in zip(rng.integers(0, gs.n_rwg, 6), rng.integers(0, gb.n_rwg, 6)):
        ref = 0.0
        for T, sg, p in ((gs.tp[a], 1.0, gs.pp[a]), (gs.tm[a], -1.0, gs.pm[a])):
            rt = pts @ gs.tri_vert[T]
            lam = sg * gs.length[a] / (2 * gs.tri_area[T]) * (rt - p)
            wt = w * gs.tri_area[T]
            for i in np.flatnonzero(db.fn == b):
                t = db.tr[i]
                rsrc = pts @ tv_r[t]
                f = (db.s[i] * rsrc - db.q[i]) / (2 * area_r[t])
                d = rt[:, None, :] - rsrc[None, :, :]
                R = np.linalg.norm(d, axis=-1)
                gp = -(1 + 1j * K0 * R) * np.exp(-1j * K0 * R) / (4 * np.pi * R ** 2)
                grad = d / R[..., None] * gp[..., None]
                cr = np.cross(grad, f[None, :, :])
                ref += np.einsum("q,s,qk,qsk->", wt, w * area_r[t], lam, cr)
        assert abs(K[a, b] - ref) < 1e-5 * np.abs(K).max()


# ---- the macromodel -------------------------------------------------------------------

def test_l_type_blocks_are_reciprocal(elem4):
    """G^(E^,J) = (G^(E,H^))^T (the Galerkin form of L is symmetric), from two independent
    fills with test and source roles exchanged; they differ by quadrature only."""
    _, _, _, _, mm = elem4
    err = np.abs(mm.GHJ - mm.GEH.T).max() / np.abs(mm.GHJ).max()
    assert err < 1.5e-2


def test_macromodel_factor_identity(elem4):
    """M x = T (A^-1 (B x)) with the factors applied one after the other (section III)."""
    _, _, _, _, mm = elem4
    rng = np.random.default_rng(0)
    x = rng.standard_normal((mm.M.shape[1], 3)) + 1j * rng.standard_normal((mm.M.shape[1], 3))
    ref = mm.T @ np.linalg.solve(mm.A, mm.B @ x)
    assert np.abs(mm.M @ x - ref).max() < 1e-12 * np.abs(ref).max()
    # and the elimination of H^ (eq. Hdiscretized1) inside A and B
    H = -np.linalg.solve(mm.GHH, mm.GHE @ x[:, :1] + mm.GHJ @ (-mm.R @ x[:, :1]))
    resid = mm.GEJ @ (-mm.R @ x[:, :1]) + mm.GEH @ H + mm.GEE @ x[:, :1]
    assert np.abs(resid).max() < 1e-10 * np.abs(mm.GEE @ x[:, :1]).max()


def test_single_element_reduces_to_direct_efie(elem4):
    """M = 1: the macromodel solve's J = -R E^ against the scatterer's own EFIE solution, and
    the far field of J^ = T J against that of J (equivalence theorem), a few 0.1% at 4 x 4
    per face.  Sign errors in the jump term, D or the normal give O(1)."""
    _, _, gs, gb, mm = elem4
    err, eq = _m1_errors(gs, gb, mm, ((0.0, 0.0, 0), (0.6, 0.3, 1), (1.1, 2.0, 0)))
    assert err < 1e-2
    assert eq < 1.5e-2
    # the same system with the jump term of the other sign is far off
    lu = sla.lu_factor(mm.GHH)
    B = mm.GEE - mm.GEH @ sla.lu_solve(lu, mm.GHE - mm.D)
    Mw = mm.T @ np.linalg.solve(mm.A, B)
    c = np.zeros((1, 3))
    Jd = np.linalg.solve(mm.GEJ, plane_wave_rhs(gs, c, 0.0, 0.0, 0, K0))
    E = np.linalg.solve(mm.D - mm.GHH @ Mw, plane_wave_rhs(gb, c, 0.0, 0.0, 0, K0))
    Jw = -np.linalg.solve(mm.A, B) @ E
    assert np.linalg.norm(Jw - Jd) / np.linalg.norm(Jd) > 0.5


def test_single_element_error_shrinks_under_refinement(elem4):
    """The M = 1 and equivalence-theorem errors fall when the box mesh goes from 4 x 4 to
    6 x 6 squares per face (measured about 5e-3 -> 1.4e-3 and 9e-3 -> 2.8e-3)."""
    _, _, gs, gb, mm = elem4
    inc = ((0.0, 0.0, 0), (0.6, 0.3, 1))
    e4, q4 = _m1_errors(gs, gb, mm, inc)
    box6 = cube_surface(0.5, 6)
    gb6 = mesh_geometry(box6)
    mm6 = element_macromodel(gs, gb6, box6, K0, ETA)
    e6, q6 = _m1_errors(gs, gb6, mm6, inc)
    assert e6 < 0.5 * e4
    assert q6 < 0.5 * q4


def test_equivalence_theorem_near_field(elem4):
    """E radiated by J^ = T J equals E radiated by J at points 0.5 wavelength outside the
    box (section II-B), within the box discretisation error."""
    _, _, gs, gb, mm = elem4
    c = np.zeros((1, 3))
    Jd = np.linalg.solve(mm.GEJ, plane_wave_rhs(gs, c, 0.3, 0.2, 0, K0))
    rng = np.random.default_rng(5)
    v = rng.standard_normal((40, 3))
    pts = v / np.linalg.norm(v, axis=1, keepdims=True) * (0.25 * np.sqrt(3) + 0.5)
    Ej = radiated_near_field(gs, c, Jd, pts, K0, ETA)
    Eh = radiated_near_field(gb, c, mm.T @ Jd, pts, K0, ETA)
    assert np.linalg.norm(Eh - Ej) / np.linalg.norm(Ej) < 2e-2


def test_near_field_evaluation_matches_far_field():
    """radiated_near_field times r exp(j k r) at 400 wavelengths tends to radiated_field."""
    plate = square_plate(0.4, 4)
    g = mesh_geometry(plate)
    rng = np.random.default_rng(7)
    J = rng.standard_normal(g.n_rwg) + 1j * rng.standard_normal(g.n_rwg)
    rh = np.array([[0.3, 0.4, np.sqrt(1 - 0.25)], [0.0, 0.0, 1.0], [1.0, 0.0, 0.0]])
    r = 400.0
    En = radiated_near_field(g, np.zeros((1, 3)), J, rh * r, K0, ETA) * r * np.exp(1j * K0 * r)
    Ef = radiated_field(g, np.zeros((1, 3)), J, rh, K0, ETA)
    assert np.abs(En - Ef).max() < 2e-3 * np.abs(Ef).max()


def test_array_rcs_matches_dense_mom_on_the_plates(elem4):
    """The 2 x 2 plate array (pitch 0.6): the final system (D - G M) E^ = V^ with the dense
    exact G between boxes, far field of J^ = -M E^, against the dense EFIE of the four
    plates themselves; bistatic RCS within 0.3 dB wherever it is within 20 dB of its peak
    (the paper compares its macromodel patterns with full-wave references the same way)."""
    plate, box, gs, gb, mm = elem4
    wl = make_workload(0)
    centers = wl.elem_center()
    ne, nb = centers.shape[0], gb.n_rwg
    G = efie_dense(gb, centers, K0, ETA)
    Gp = efie_dense(gs, centers, K0, ETA)
    rh = np.array([[np.sin(a) * np.cos(b), np.sin(a) * np.sin(b), np.cos(a)]
                   for a in np.radians(np.arange(0, 91, 3)) for b in np.radians([0.0, 45.0, 90.0])])
    for th, ph, pol in ((0.0, 0.0, 0), (0.5, 0.8, 1)):
        Vh = plane_wave_rhs(gb, centers, th, ph, pol, K0)
        Mb = np.kron(np.eye(ne), mm.M)
        Db = np.kron(np.eye(ne), mm.D)
        E = np.linalg.solve(Db - G @ Mb, Vh)
        db_m = rcs_db(radiated_field(gb, centers, -(Mb @ E), rh, K0, ETA))
        Jp = np.linalg.solve(Gp, plane_wave_rhs(gs, centers, th, ph, pol, K0))
        db_p = rcs_db(radiated_field(gs, centers, Jp, rh, K0, ETA))
        keep = db_p >= db_p.max() - 20.0
        assert np.max(np.abs(db_m[keep] - db_p[keep])) < 0.3
