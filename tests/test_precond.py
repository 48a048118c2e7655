"""Block-Jacobi preconditioner: oracle pins and host-side library parity (no GPU).

The oracle's diagonal block D - G_self M_t is pinned against the full final-system
operator it is cut from (a one-element array's dense matrix, and the diagonal
blocks of a 2 x 2 array's operator), and its preconditioned GMRES against the
unpreconditioned solve and an independent residual.  The library computes the same
blocks on the host in its own code (direct stencil sums, its own LU); they must
agree with the oracle's to FP64 rounding.
"""
import ctypes

import numpy as np
import pytest

from oracle import precond as opre
from oracle.excitation import plane_wave_rhs
from oracle.gmres import gmres
from oracle.system import OracleOperator
from synth import make_workload

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(np.asarray(b))))


@pytest.fixture(scope="module")
def wl2():
    # three kinds of element on a 2 x 2 lattice
    return make_workload(2, px=2, py=2, nrhs=1)


@pytest.fixture(scope="module")
def gself2(wl2):
    return opre.self_block(wl2)


def test_one_element_block_is_the_whole_operator(wl2, gself2):
    """For a 1 x 1 array the diagonal block is the final-system matrix itself, so P inverts it."""
    wl1 = opre.one_element(wl2)
    A1 = OracleOperator(wl1).dense()
    blocks = opre.diagonal_blocks(wl2, gself2)
    assert _rel(blocks[0], A1) < 1e-13
    P = opre.block_jacobi(wl2, gself2)
    assert np.abs(A1 @ P[0] - np.eye(A1.shape[0])).max() < 1e-12


def test_diagonal_blocks_of_an_array_are_translation_invariant(wl2, gself2):
    """Rows and columns of one element cut from the 2 x 2 array's operator equal D - G_self M_t(m)."""
    op = OracleOperator(wl2)
    n = op.nb
    blocks = opre.diagonal_blocks(wl2, gself2)
    e = np.zeros(wl2.n_unknowns, dtype=np.complex128)
    for m in (0, 3):
        A_mm = np.empty((n, n), dtype=np.complex128)
        for j in range(n):
            e[:] = 0
            e[m * n + j] = 1
            A_mm[:, j] = op.matvec(e)[m * n:(m + 1) * n]
        assert _rel(A_mm, blocks[wl2.elem_type[m]]) < 1e-12, m


def test_kinds_give_distinct_blocks(wl2, gself2):
    P = opre.block_jacobi(wl2, gself2)
    assert P.shape == (3, 288, 288)
    assert _rel(P[0], P[1]) > 1e-3 and _rel(P[1], P[2]) > 1e-3


def test_preconditioned_gmres_matches_plain_solve():
    wl = make_workload(0, px=3, py=3)
    op = OracleOperator(wl)
    P = opre.block_jacobi(wl)
    b = plane_wave_rhs(op.geo, wl.elem_center(), 0.3, 0.2, 1, wl.k)
    x0, i0 = gmres(op.matvec, b, restart=30, tol=1e-11, max_iters=2000)
    x1, i1 = gmres(op.matvec, b, restart=30, tol=1e-11, max_iters=2000,
                   precond=lambda v: opre.apply(P, wl.elem_type, v))
    assert i0["converged"] and i1["converged"]
    assert i1["iters"] < i0["iters"]
    # an independent residual of the preconditioned solution
    assert np.linalg.norm(b - op.matvec(x1)) / np.linalg.norm(b) <= 1e-11
    assert np.linalg.norm(x1 - x0) / np.linalg.norm(x0) < 1e-9


def test_preconditioned_gmres_on_one_element_takes_one_step(wl2, gself2):
    wl1 = opre.one_element(wl2)
    op = OracleOperator(wl1)
    P = opre.block_jacobi(wl2, gself2)
    b = plane_wave_rhs(op.geo, wl1.elem_center(), 0.0, 0.0, 0, wl1.k)
    x, info = gmres(op.matvec, b, restart=10, tol=1e-10, precond=lambda v: opre.apply(P, wl1.elem_type, v))
    assert info["converged"] and info["iters"] == 1


# ---- library (host part) ------------------------------------------------------------
@pytest.fixture(scope="module")
def lib():
    import os
    from paper_1712_02443_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1712_02443_amd.build import build
        build()
    return _lib.load()


def _host_op_with_data(wl):
    from paper_1712_02443_amd import AimOperator
    op = AimOperator.from_workload(wl, host_only=True)
    op.set_macromodels(wl.macromodels())
    r, c, v = wl.d_matrix()
    op.set_dmatrix(r, c, v)
    return op


@pytest.mark.parametrize("lattice", [(2, 2), (3, 1)])
def test_library_blocks_match_oracle(lib, wl2, gself2, lattice):
    """The library's FP64 blocks equal the oracle's for every kind, on any lattice."""
    wl = make_workload(2, px=lattice[0], py=lattice[1], nrhs=1)
    op = _host_op_with_data(wl)
    op.build_preconditioner()
    P = op.preconditioner()
    Po = opre.block_jacobi(wl2, gself2)
    for t in range(3):
        assert _rel(P[t], Po[t]) < 1e-12, t
    op.close()


def test_library_blocks_648_rwg_surface(lib):
    wl = make_workload(1, px=2, py=1, nrhs=1)
    op = _host_op_with_data(wl)
    op.build_preconditioner()
    P = op.preconditioner()[0]
    A = opre.diagonal_blocks(wl)[0]
    assert np.abs(A @ P - np.eye(A.shape[0])).max() < 1e-12
    op.close()


def test_preconditioner_state_errors(lib):
    from paper_1712_02443_amd import AimOperator, _lib
    wl = make_workload(0)
    op = AimOperator.from_workload(wl, host_only=True)
    assert lib.aim_build_preconditioner(op._op) == _lib.AIM_ESTATE
    assert b"must be set" in lib.aim_last_error()
    assert lib.aim_build_preconditioner(None) == _lib.AIM_EINVAL
    op.set_macromodels(wl.macromodels())
    r, c, v = wl.d_matrix()
    op.set_dmatrix(r, c, v)
    buf = np.zeros(2 * 288 * 288)
    assert lib.aim_get_preconditioner(op._op, buf.ctypes.data_as(_lib._f64p)) == _lib.AIM_ESTATE
    op.build_preconditioner()
    assert lib.aim_get_preconditioner(op._op, buf.ctypes.data_as(_lib._f64p)) == _lib.AIM_OK
    # new macromodels make the blocks stale
    op.set_macromodels(wl.macromodels())
    assert lib.aim_get_preconditioner(op._op, buf.ctypes.data_as(_lib._f64p)) == _lib.AIM_ESTATE
    # device entry points still refuse a host-only op
    assert lib.precond_apply(op._op, ctypes.c_void_p(1), ctypes.c_void_p(2), 1, 0, None) == _lib.AIM_ESTATE
    # unknown preconditioner codes are rejected before any device work
    opts = _lib.GmresOpts(10, 10, 0, 0, 1, 7, 0, 0, 1e-6)
    stats = (_lib.GmresStat * 1)()
    assert lib.gmres_solve(op._op, ctypes.c_void_p(1), ctypes.c_void_p(2), 1, ctypes.byref(opts), stats,
                           None) == _lib.AIM_EINVAL
    assert b"preconditioner" in lib.aim_last_error()
    op.close()
