"""Pins of the CPU oracle against closed forms, library routines, brute force and invariants.

Each test ties one oracle function to something other than itself, so that a
dropped term, a wrong sign, a wrong index or a transposed operand in the oracle
fails at least one of them.
"""
import math

import numpy as np
import pytest
import scipy.special

from galerkin_refs import plain_entry, refined_entry
from oracle import aim
from oracle.excitation import plane_wave_rhs
from oracle.galerkin import efie_pairs, smooth_kernel, static_potentials
from oracle.geometry import gauss_triangle_rule, rwg_geometry, seven_point_rule
from oracle.gmres import gmres
from oracle.system import OracleOperator
from synth import make_workload

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(np.asarray(b))))


# ---- quadrature -----------------------------------------------------------------
def test_seven_point_rule_degree_five():
    """Radon's rule integrates every monomial of degree <= 5 on a triangle exactly."""
    bary, w = seven_point_rule()
    ref_b, ref_w = gauss_triangle_rule(12)
    tv = np.array([[0.1, -0.2, 0.0], [0.9, 0.1, 0.0], [0.3, 0.8, 0.0]])
    p7 = bary @ tv
    pr = ref_b @ tv
    for a in range(6):
        for b in range(6 - a):
            f7 = np.sum(w * p7[:, 0] ** a * p7[:, 1] ** b)
            fr = np.sum(ref_w * pr[:, 0] ** a * pr[:, 1] ** b)
            assert abs(f7 - fr) <= 1e-14 * max(1.0, abs(fr))
    # and not degree 6
    assert abs(np.sum(w * p7[:, 0] ** 6) - np.sum(ref_w * pr[:, 0] ** 6)) > 1e-8


def test_duffy_rule_exact_area_moments():
    """The pin rule itself: int_T x dS over the unit right triangle is 1/6, int x^2 y^2 is 1/180."""
    b, w = gauss_triangle_rule(8)
    tv = np.array([[0.0, 0, 0], [1.0, 0, 0], [0.0, 1, 0]])
    p = b @ tv
    A = 0.5
    assert abs(A * np.sum(w * p[:, 0]) - 1 / 6) < 1e-15
    assert abs(A * np.sum(w * p[:, 0] ** 2 * p[:, 1] ** 2) - 1 / 180) < 1e-15


# ---- closed-form potentials and kernel ---------------------------------------------
@pytest.mark.parametrize("r", [(0.05, 0.03, 0.04), (0.3, -0.1, 0.02), (-0.02, 0.05, -0.001),
                               (0.2, 0.2, 0.3)])
def test_static_potentials_match_fine_quadrature(r):
    """Closed-form int 1/R and int (r'-rho)/R against a 60 x 60 Duffy rule, points off the plane."""
    tv = np.array([[[0.0, 0.0, 0.0], [0.13, 0.01, 0.0], [0.02, 0.11, 0.0]]])
    r = np.array(r)
    I1, Iv = static_potentials(r[None, None, :], tv)
    b, w = gauss_triangle_rule(60)
    pts = b @ tv[0]
    A = 0.5 * np.linalg.norm(np.cross(tv[0, 1] - tv[0, 0], tv[0, 2] - tv[0, 0]))
    R = np.linalg.norm(pts - r, axis=1)
    rho = np.array([r[0], r[1], 0.0])
    assert abs(I1[0, 0] - A * np.sum(w / R)) < 1e-9 * abs(I1[0, 0])
    assert np.max(np.abs(Iv[0, 0] - A * np.sum(w[:, None] * (pts - rho) / R[:, None], axis=0))) < 1e-9


def test_static_potential_rotated_triangle():
    """Same closed forms for a triangle that is not in a coordinate plane."""
    rng = np.random.default_rng(3)
    tv = rng.uniform(-0.1, 0.1, (1, 3, 3))
    r = np.array([0.05, -0.07, 0.12])
    I1, Iv = static_potentials(r[None, None, :], tv)
    b, w = gauss_triangle_rule(80)
    pts = b @ tv[0]
    nrm = np.cross(tv[0, 1] - tv[0, 0], tv[0, 2] - tv[0, 0])
    A = 0.5 * np.linalg.norm(nrm)
    nrm /= np.linalg.norm(nrm)
    rho = r - nrm * np.dot(r - tv[0, 0], nrm)
    R = np.linalg.norm(pts - r, axis=1)
    assert abs(I1[0, 0] - A * np.sum(w / R)) < 1e-9 * abs(I1[0, 0])
    assert np.max(np.abs(Iv[0, 0] - A * np.sum(w[:, None] * (pts - rho) / R[:, None], axis=0))) < 1e-9


def test_green_function_is_spherical_hankel():
    """G(R) = exp(-jkR)/(4 pi R) = -j k/(4 pi) h0^(2)(kR), via scipy's spherical Bessel functions."""
    k, h = 2 * math.pi, 0.1
    Gs = aim.green_samples((4, 4, 3), h, k)
    for d in [(1, 0, 0), (2, 3, 1), (3, 3, 2), (-2, 1, -1)]:
        R = h * math.sqrt(sum(x * x for x in d))
        kr = k * R
        h02 = scipy.special.spherical_jn(0, kr) - 1j * scipy.special.spherical_yn(0, kr)
        val = -1j * k / (4 * math.pi) * h02
        assert abs(Gs[d[0] + 3, d[1] + 3, d[2] + 2] - val) < 1e-14 * abs(val)
    assert Gs[3, 3, 2] == 0.0


def test_smooth_kernel_limit_and_identity():
    k = 2 * math.pi
    R = np.array([1e-9, 1e-4, 0.05, 0.3])
    val = smooth_kernel(R, k)
    direct = (np.exp(-1j * k * R) - 1.0) / (4 * math.pi * R)
    assert _rel(val[1:], direct[1:]) < 1e-12
    assert abs(val[0] - (-1j * k / (4 * math.pi))) < 1e-8
    assert smooth_kernel(np.array([0.0]), k)[0] == -1j * k / (4 * math.pi)


# ---- Galerkin entries ------------------------------------------------------------
def test_galerkin_far_pair_matches_high_order_rule(op0):
    geo, wl = op0.geo, op0.wl
    sa, sb = np.zeros(3), np.array([1.2, 0.6, 0.0])
    for a, b in [(0, 5), (17, 200), (140, 33)]:
        ours = efie_pairs(geo, sa, [a], geo, sb, [b], wl.k, wl.eta)[0]
        ref = plain_entry(geo, a, sa, b, sb, wl.k, wl.eta)
        assert abs(ours - ref) < 2e-5 * abs(ref)


@pytest.mark.parametrize("pair", [(0, 0), (0, 1), (5, 9), (100, 101)])
def test_galerkin_singular_pairs_converge_under_refinement(op0, pair):
    """Touching and coincident pairs: refining both triangles converges (16 vs 64 pieces agree
    to 2e-3) and the single-rule entry lies within the 7-point outer rule's few-percent error of
    the converged value; a dropped term or a sign error would be off by O(1)."""
    geo, wl = op0.geo, op0.wl
    a, b = pair
    ours = efie_pairs(geo, np.zeros(3), [a], geo, np.zeros(3), [b], wl.k, wl.eta)[0]
    ref2 = refined_entry(geo, a, b, wl.k, wl.eta, levels=2)
    ref3 = refined_entry(geo, a, b, wl.k, wl.eta, levels=3)
    assert abs(ref2 - ref3) < 2e-3 * abs(ref3)
    assert abs(ours - ref3) < 3e-2 * abs(ref3)


def test_galerkin_near_symmetry(op0):
    """G_ab and G_ba are computed by different quadrature paths yet must agree (reciprocity)."""
    geo, wl = op0.geo, op0.wl
    rng = np.random.default_rng(1)
    a = rng.integers(0, geo.n_rwg, 200)
    b = rng.integers(0, geo.n_rwg, 200)
    ab = efie_pairs(geo, np.zeros(3), a, geo, np.zeros(3), b, wl.k, wl.eta)
    ba = efie_pairs(geo, np.zeros(3), b, geo, np.zeros(3), a, wl.k, wl.eta)
    assert _rel(ab, ba) < 2e-3
    sh = np.array([0.6, 0.0, 0.0])
    ab = efie_pairs(geo, np.zeros(3), a, geo, sh, b, wl.k, wl.eta)
    ba = efie_pairs(geo, sh, b, geo, np.zeros(3), a, wl.k, wl.eta)
    assert _rel(ab, ba) < 1e-3


# ---- AIM pieces ------------------------------------------------------------------
def test_projection_weights_moment_identity(op0):
    """sum_g W_psi[a,g] p(r_g) = int f_psi p dS for tensor monomials of degree <= N_O per axis,
    with the right side from an independent 10 x 10 Duffy rule."""
    geo, wl = op0.geo, op0.wl
    s, W = op0.s_local, op0.W
    q = wl.order + 1
    b10, w10 = gauss_triangle_rule(10)
    rng = np.random.default_rng(0)
    for a in rng.choice(geo.n_rwg, 12, replace=False):
        nodes = (s[a][None, :] + np.stack(np.meshgrid(*[np.arange(q)] * 3, indexing="ij"), -1).reshape(-1, 3)) * wl.h
        for al in [(0, 0, 0), (1, 0, 0), (0, 2, 1), (2, 2, 2), (1, 2, 0)]:
            pg = np.prod((nodes - geo.center[a]) ** np.array(al), axis=1)
            for psi in range(4):
                lhs = np.sum(W[psi, a].reshape(-1) * pg)
                rhs = 0.0
                for sg, ti, pv in ((1, geo.tp, geo.pp), (-1, geo.tm, geo.pm)):
                    tv = geo.tri_vert[ti[a]]
                    A = geo.tri_area[ti[a]]
                    r = b10 @ tv
                    f = (sg * geo.length[a] / (2 * A) * (r - pv[a]))[:, psi] if psi < 3 else \
                        np.full(r.shape[0], sg * geo.length[a] / A)
                    rhs += A * np.sum(w10 * f * np.prod((r - geo.center[a]) ** np.array(al), axis=1))
                assert abs(lhs - rhs) < 1e-12 * max(1e-3, abs(rhs)), (a, al, psi)


def test_stencil_origin_centres_the_anchor():
    """The stencil is centred on the node nearest the anchor (N_O even) and ties go upward."""
    c = np.array([[0.25, -0.25, 0.0], [0.04, 0.06, -0.151], [0.249999999, 0.15, 0.35]])
    s = aim.stencil_origin(c, 0.1, 2)
    assert np.array_equal(s[0], [2, -3, -1])
    assert np.array_equal(s[1], [-1, 0, -3])
    assert np.array_equal(s[2], [1, 1, 3])
    s3 = aim.stencil_origin(c, 0.1, 3)
    assert np.array_equal(s3[1], [-1, -1, -3])  # anchor in [s+1, s+2) for N_O = 3


def test_fft_convolution_equals_direct_sum(op0):
    rng = np.random.default_rng(0)
    Q = rng.standard_normal((4,) + op0.grid.shape) + 1j * rng.standard_normal((4,) + op0.grid.shape)
    d = aim.convolve_direct(Q, op0.Gs)
    f = aim.convolve_fft(Q, op0.Gs)
    assert _rel(f, d) < 1e-13


def test_padded_size_invariance(op0):
    rng = np.random.default_rng(1)
    shp = op0.grid.shape
    Q = rng.standard_normal((1,) + shp) + 1j * rng.standard_normal((1,) + shp)
    base = aim.convolve_fft(Q, op0.Gs)
    for pad in [tuple(2 * n - 2 for n in shp), (27, 27, 15), (32, 30, 16), (36, 40, 20)]:
        assert _rel(aim.convolve_fft(Q, op0.Gs, pad), base) < 1e-13


def test_grid_self_term_cancels():
    """G(0) never reaches a far pair, so the operator is the same for any value of it."""
    wl = make_workload(0)
    x = wl.test_vectors(1)[0]
    a = OracleOperator(wl, g0=0.0).matvec(x)
    b = OracleOperator(wl, g0=1.0 + 2.0j).matvec(x)
    assert _rel(a, b) < 1e-13


def test_translation_invariance_of_near_blocks():
    """Per-offset blocks computed in the element frame equal the element-pair construction."""
    wl = make_workload(2, px=3, py=2, nrhs=1)
    a = OracleOperator(wl, near_mode="global")
    b = OracleOperator(wl, near_mode="offset")
    assert abs(a.C - b.C).max() < 1e-13 * abs(a.C).max()


def test_near_blocks_applied_by_offset_equal_global_matrix():
    """The per-offset application used for large arrays equals the global sparse matrix."""
    wl = make_workload(2, px=6, py=5, nrhs=1)
    op = OracleOperator(wl)
    u = op.macro_apply(wl.test_vectors(1)[0])
    assert _rel(op.near_apply(u, by_blocks=True), op.C @ u) < 1e-14


def test_near_pairs_are_exact_galerkin(op0, dense0):
    """On near pairs the AIM operator reproduces the Galerkin entry (pre-correction)."""
    nb = op0.nb
    e = np.zeros(op0.wl.n_unknowns, dtype=np.complex128)
    C = op0.C.tocsr()
    cols = np.unique(C[:nb].indices)[::7]
    for j in cols:
        e[:] = 0
        e[j] = 1
        col = op0.g_apply(e)[:nb]
        near = np.asarray(C[:nb, j].todense()).ravel() != 0
        assert np.max(np.abs(col[near] - dense0[near, j])) < 1e-12 * np.abs(dense0).max()


def test_far_pairs_within_aim_error(op0, dense0):
    """Far pairs: AIM approximates the Galerkin entries (order 2, h = lambda/10)."""
    nb = op0.nb
    n = op0.wl.n_unknowns
    GA = np.empty((nb, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for j in range(n):
        e[:] = 0
        e[j] = 1
        GA[:, j] = op0.g_apply(e)[:nb]
    far = np.asarray(op0.C[:nb].todense()) == 0
    err = np.linalg.norm((GA - dense0)[far]) / np.linalg.norm(dense0[far])
    assert err < 0.06


def test_far_error_shrinks_with_order_three():
    """Raising the interpolation order reduces the far-field AIM error."""
    from oracle.galerkin import efie_dense
    errs = []
    for order in (2, 3):
        wl = make_workload(0, px=2, py=1)
        wl.order = order
        op = OracleOperator(wl)
        nb, n = op.nb, wl.n_unknowns
        dense = efie_dense(op.geo, wl.elem_center(), wl.k, wl.eta, rows=range(nb))
        rows = np.arange(nb)
        GA = np.empty((nb, n), dtype=np.complex128)
        e = np.zeros(n, dtype=np.complex128)
        for j in range(n):
            e[:] = 0
            e[j] = 1
            GA[:, j] = op.g_apply(e)[rows]
        far = np.asarray(op.C[:nb].todense()) == 0
        errs.append(np.linalg.norm((GA - dense)[far]) / np.linalg.norm(dense[far]))
    assert errs[1] < 0.7 * errs[0]


def test_far_operator_complex_symmetric(op0):
    """I_psi = P_psi^T and an even kernel make the grid part exactly complex symmetric."""
    rng = np.random.default_rng(2)
    n = op0.wl.n_unknowns
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    y = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    assert abs(x @ op0.far_field(y) - y @ op0.far_field(x)) < 1e-13 * abs(x @ op0.far_field(y))


def test_projection_interpolation_adjoint(op0):
    """<P u, Phi> = <u, P^T Phi> per potential, checking project and interpolate index the same."""
    rng = np.random.default_rng(3)
    n = op0.wl.n_unknowns
    u = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    Q = aim.project(op0.grid, op0.W, u)
    k, eta = op0.wl.k, op0.wl.eta
    for psi in range(4):
        Phi = np.zeros((4,) + op0.grid.shape, dtype=np.complex128)
        Phi[psi] = rng.standard_normal(op0.grid.shape)
        v = aim.interpolate(op0.grid, op0.W, Phi, k, eta)
        sig = 1.0 if psi < 3 else -1.0 / (k * k)
        lhs = np.sum(Q[psi] * Phi[psi])
        rhs = np.sum(u * v) / (-1j * k * eta * sig)
        assert abs(lhs - rhs) < 1e-12 * abs(lhs)


# ---- excitation, operator, solver ---------------------------------------------------
def test_plane_wave_rhs_closed_form_normal_incidence():
    """Normal incidence, x polarisation: on a horizontal face the phase is constant and
    int_T Lambda dS = (l/2)(centroid - free vertex), so V_n = -exp(jkz) x . (l/2)[(c+ - p+) + (p- - c-)]."""
    wl = make_workload(0, px=1, py=1)
    mesh = wl.surface
    geo = rwg_geometry(mesh.vert, mesh.tri, mesh.rwg)
    V = plane_wave_rhs(geo, np.zeros((1, 3)), 0.0, 0.0, 0, wl.k)
    cp = geo.tri_vert[geo.tp].mean(axis=1)
    cm = geo.tri_vert[geo.tm].mean(axis=1)
    z = cp[:, 2]
    flat = (np.abs(np.abs(z) - 0.25) < 1e-12) & (np.abs(cm[:, 2] - z) < 1e-12)
    assert flat.sum() > 50
    ref = -np.exp(1j * wl.k * z) * 0.5 * geo.length * ((cp - geo.pp)[:, 0] + (geo.pm - cm)[:, 0])
    assert np.max(np.abs(V[flat] - ref[flat])) < 1e-15


def test_macro_apply_is_block_diagonal(op0):
    import scipy.linalg
    wl = op0.wl
    x = wl.test_vectors(1)[0]
    big = scipy.linalg.block_diag(*[op0.M[t] for t in wl.elem_type])
    assert _rel(op0.macro_apply(x), big @ x) < 1e-14


def test_matvec_linear_and_direct_consistent(op0):
    rng = np.random.default_rng(5)
    n = op0.wl.n_unknowns
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    y = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    a = 0.3 - 1.1j
    lhs = op0.matvec(a * x + y)
    rhs = a * op0.matvec(x) + op0.matvec(y)
    assert _rel(lhs, rhs) < 1e-13
    assert _rel(op0.matvec(x, direct=True), op0.matvec(x)) < 1e-13


def test_gmres_matches_dense_solve(op0):
    wl = op0.wl
    A = op0.dense()
    b = plane_wave_rhs(op0.geo, wl.elem_center(), 0.0, 0.0, 0, wl.k)
    xs = np.linalg.solve(A, b)
    x, info = gmres(op0.matvec, b, restart=30, tol=1e-12, max_iters=2000)
    assert info["converged"]
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-9
    assert info["restarts"] >= 2


def test_radiated_field_reciprocity_with_plane_wave_rhs(op0):
    """Reciprocity: the far field of currents J along rhat, polarisation e (e . rhat = 0),
    equals (j k eta / 4 pi) sum_a J_a V_a for the plane wave arriving from rhat with
    polarisation e (V of eq. V1), for two independently written integrals."""
    from oracle.excitation import incidence, radiated_field
    wl = op0.wl
    rng = np.random.default_rng(5)
    J = rng.standard_normal(wl.n_unknowns) + 1j * rng.standard_normal(wl.n_unknowns)
    centers = wl.elem_center()
    for th, ph in ((0.3, 1.1), (1.2, -2.0), (0.0, 0.0), (2.5, 0.4)):
        rhat = np.array([[np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)]])
        E = radiated_field(op0.geo, centers, J, rhat, wl.k, wl.eta)[0]
        for pol in (0, 1):
            _, e = incidence(th, ph, pol)
            V = plane_wave_rhs(op0.geo, centers, th, ph, pol, wl.k)
            ref = 1j * wl.k * wl.eta / (4 * np.pi) * np.sum(J * V)
            assert abs(np.dot(e, E) - ref) <= 1e-12 * abs(ref)
        assert abs(np.dot(rhat[0], E)) <= 1e-12 * np.linalg.norm(E)


# ---- Mie series for a PEC sphere -------------------------------------------------------
def test_mie_rayleigh_limit():
    """Small spheres: backscatter sigma / (pi a^2) -> 9 (k a)^4 (perfect conductor)."""
    from oracle import mie
    for x in (0.01, 0.02):
        sig = mie.bistatic_rcs(1.0, x, np.array([np.pi]), np.array([0.0]))[0]
        assert abs(sig / (np.pi * x ** 2) / (9 * x ** 4) - 1) < 1e-3


@pytest.mark.parametrize("x", [0.5, 1.26, 3.0, 8.0])
def test_mie_optical_theorem_and_truncation(x):
    """A perfect conductor absorbs nothing: the optical-theorem extinction equals the
    scattering sum; ten more terms change neither."""
    from oracle import mie
    ext, sca = mie.extinction_and_scattering(1.0, x)
    assert abs(ext - sca) <= 1e-10 * sca
    n0 = int(np.ceil(x + 4.0 * x ** (1.0 / 3.0) + 2.0))
    ext2, _ = mie.extinction_and_scattering(1.0, x, n_max=n0 + 10)
    assert abs(ext2 - ext) <= 1e-9 * ext
    # the two principal planes agree at forward and back scattering (S1 = S2 there)
    s_e = mie.bistatic_rcs(1.0, x, np.array([0.0, np.pi]), np.zeros(2))
    s_h = mie.bistatic_rcs(1.0, x, np.array([0.0, np.pi]), np.full(2, np.pi / 2))
    assert np.allclose(s_e, s_h, rtol=1e-12)


@pytest.fixture(scope="module")
def sphere_solutions():
    """Dense EFIE solves of a PEC sphere of radius 0.2 wavelength (k a = 1.26) meshed at
    two refinements (480 and 1920 RWG), x-polarised plane wave arriving from +z."""
    from oracle.excitation import radiated_field, rcs_db
    from oracle.galerkin import efie_dense
    from synth.mesh import icosphere
    k, eta, a = 2 * np.pi, 376.730313668, 0.2
    th = np.linspace(0, np.pi, 37)
    out = []
    for level in (2, 3):
        m = icosphere(a, level)
        geo = rwg_geometry(m.vert, m.tri, m.rwg)
        c = np.zeros((1, 3))
        J = np.linalg.solve(efie_dense(geo, c, k, eta), plane_wave_rhs(geo, c, 0.0, 0.0, 0, k))
        cuts = []
        for phi in (0.0, np.pi / 2):
            rh = np.stack([np.sin(th) * np.cos(phi), np.sin(th) * np.sin(phi), np.cos(th)], 1)
            cuts.append(rcs_db(radiated_field(geo, c, J, rh, k, eta)))
        out.append(np.stack(cuts))
    return k, a, th, out


def test_efie_sphere_matches_mie_and_converges(sphere_solutions):
    """EFIE entries, excitation and far field together against the analytic Mie series:
    within 0.5 dB at 480 RWG, and the error shrinks by more than half at 1920 RWG."""
    from oracle import mie
    k, a, th, sols = sphere_solutions
    ref = np.stack([10 * np.log10(mie.bistatic_rcs(k, a, np.pi - th, np.full_like(th, p)))
                    for p in (0.0, np.pi / 2)])
    err = [np.abs(s - ref).max() for s in sols]
    assert err[0] < 0.5
    assert err[1] < 0.5 * err[0]


def test_oracle_without_near_field_keeps_the_grid_part():
    """near=False only skips the near-field build: the grid part is bitwise the same,
    and every use of the near field raises."""
    wl = make_workload(0)
    full = OracleOperator(wl)
    far = OracleOperator(wl, near=False)
    x = wl.test_vectors(1)[0]
    assert np.array_equal(full.far_field(x), far.far_field(x))
    with pytest.raises(RuntimeError):
        far.near_apply(x)
    with pytest.raises(RuntimeError):
        far.matvec(x)


def test_row_products_equal_full_products():
    """OracleOperator.matvec_rows and far_field_rows (the row-sampled products used for
    arrays too large for a global near matrix) against the full matvec and far field, on a
    three-kind 5 x 4 array, rows at both ends and in between."""
    wl = make_workload(2, px=5, py=4, nrhs=1)
    o = OracleOperator(wl)
    x = wl.test_vectors(1)[0]
    rows = np.concatenate([[0, 1, wl.n_unknowns - 1], np.random.default_rng(3).choice(wl.n_unknowns, 40,
                                                                                       replace=False)])
    full = o.matvec(x)
    assert _rel(o.matvec_rows(x, rows), full[rows]) < 1e-13
    u = o.macro_apply(x)
    assert _rel(o.far_field_rows(u, rows), o.far_field(u)[rows]) < 1e-13


def test_d_application_is_test_by_source():
    """The operator applies D as (D x)_a = sum_b D_ab x_b with a the testing RWG function
    and b the dual function (section IV): with the physical D of the box, d_apply of a unit
    vector e_b is column b of <Lambda^_a, n x Lambda^'_b>, element by element."""
    from oracle.macromodel import bc_dual_basis, dual_gram
    from oracle.geometry import tri_area_normal
    wl = make_workload(0)
    mesh = wl.surface
    geo = rwg_geometry(mesh.vert, mesh.tri, mesh.rwg)
    _, n_out = tri_area_normal(geo.tri_vert)
    D = dual_gram(geo, bc_dual_basis(mesh.vert, mesh.tri, mesh.rwg), n_out)
    assert np.abs(D - D.T).max() > 1e-3 * np.abs(D).max()  # not symmetric: orientation matters
    r, c = np.nonzero(D)
    o = OracleOperator(wl, D=(r, c, D[r, c].astype(np.complex128)), near=False)
    nb = geo.n_rwg
    for b in (0, 7, nb - 1):
        e = np.zeros(wl.n_unknowns, np.complex128)
        e[nb + b] = 1.0  # element 1
        y = o.d_apply(e)
        assert np.abs(y[nb:2 * nb] - D[:, b]).max() == 0.0
        assert np.abs(y[:nb]).max() == 0.0 and np.abs(y[2 * nb:]).max() == 0.0
