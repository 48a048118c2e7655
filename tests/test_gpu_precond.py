"""Block-Jacobi preconditioner on the device, through the C ABI, against the oracle.

The device blocks are the library's own host FP64 inverses (pinned against the
oracle's on the CPU); here the grouped product that applies them and the right-
preconditioned GMRES are compared with the oracle's apply and preconditioned GMRES.
Tolerances as for the product: FP64 <= 1e-12, mixed <= 1e-5 relative.
"""
import sys

import numpy as np
import pytest

from oracle import precond as opre
from oracle.gmres import gmres as oracle_gmres
from oracle.system import OracleOperator
from synth import make_workload

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-5}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


_OPS = {}


def make(torch, idx, **kw):
    """Device op with its preconditioner, oracle op and oracle blocks (cached)."""
    key = (idx, tuple(sorted(kw.items())))
    if key not in _OPS:
        from paper_1712_02443_amd import AimOperator
        wl = make_workload(idx, **kw)
        say(f"build {wl.name} px={wl.px} py={wl.py} types={wl.n_types} rhs={wl.nrhs} + block-Jacobi")
        op = AimOperator.from_workload(wl)
        op.set_macromodels(wl.macromodels())
        op.set_dmatrix(*wl.d_matrix())
        op.build_preconditioner()
        _OPS[key] = (wl, op, OracleOperator(wl), opre.block_jacobi(wl))
    return _OPS[key]


def to_dev(torch, a, prec):
    dt = torch.complex128 if prec == 0 else torch.complex64
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dt)


def to_host(t):
    return t.detach().cpu().numpy().astype(np.complex128)


CASES = [(2, dict(px=5, py=3, nrhs=3)), (1, dict(px=4, py=3, nrhs=2))]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("case", CASES)
def test_precond_apply(torch, case, prec):
    wl, op, o, P = make(torch, case[0], **case[1])
    say(f"precond apply {wl.name} prec={prec}")
    X = wl.test_vectors()
    Y = to_host(op.precond_apply(to_dev(torch, X, prec), precision=prec))
    ref = np.stack([opre.apply(P, wl.elem_type, x) for x in X])
    assert rel(Y, ref) < TOL[prec]


def test_preconditioned_gmres_fp64_matches_oracle(torch):
    from paper_1712_02443_amd import AIM_PRECOND_BLOCK_JACOBI
    wl, op, o, P = make(torch, CASES[0][0], **CASES[0][1])
    say("preconditioned gmres fp64 vs oracle")
    b = op.plane_wave_rhs(wl.theta, wl.phi, wl.pol)
    x, st, code = op.gmres(b, restart=20, tol=1e-11, max_iters=2000, precond=AIM_PRECOND_BLOCK_JACOBI)
    assert code == 0
    B = to_host(b)
    pre = lambda v: opre.apply(P, wl.elem_type, v)  # noqa: E731
    for r in range(wl.nrhs):
        assert st[r]["converged"] and st[r]["true_relres"] <= 1e-11
        xo, info = oracle_gmres(o.matvec, B[r], restart=20, tol=1e-11, max_iters=2000, precond=pre)
        assert rel(to_host(x)[r], xo) < 1e-8
    # same Krylov process: iteration counts agree at the benchmark tolerance
    x6, st6, _ = op.gmres(b, restart=50, tol=1e-6, precond=AIM_PRECOND_BLOCK_JACOBI)
    for r in range(wl.nrhs):
        _, info6 = oracle_gmres(o.matvec, B[r], restart=50, tol=1e-6, precond=pre)
        assert abs(st6[r]["iters"] - info6["iters"]) <= 1, r


@pytest.mark.parametrize("case", CASES)
def test_preconditioned_mixed_solve(torch, case):
    """Mixed-precision preconditioned solve: FP64 true residual reached, solution within
    1e-5 of the unpreconditioned FP64 solve, in fewer iterations."""
    from paper_1712_02443_amd import AIM_MIXED, AIM_PRECOND_BLOCK_JACOBI
    wl, op, o, P = make(torch, case[0], **case[1])
    say(f"preconditioned mixed solve {wl.name}")
    b = op.plane_wave_rhs(wl.theta, wl.phi, wl.pol)
    x64, s64, c64 = op.gmres(b, restart=50, tol=1e-10, max_iters=3000)
    xm, sm, cm = op.gmres(b, restart=50, tol=1e-10, max_iters=3000, precision=AIM_MIXED,
                          precond=AIM_PRECOND_BLOCK_JACOBI)
    assert c64 == 0 and cm == 0
    assert rel(to_host(xm), to_host(x64)) < 1e-5
    X, B = to_host(xm), to_host(b)
    for r in range(wl.nrhs):
        assert sm[r]["converged"] and sm[r]["true_relres"] <= 1e-10
        assert sm[r]["iters"] < s64[r]["iters"]
        res = np.linalg.norm(B[r] - o.matvec(X[r])) / np.linalg.norm(B[r])
        assert res <= 1e-9


@pytest.mark.parametrize("prec", [0, 1])
def test_preconditioned_gmres_alone_equals_in_batch(torch, prec):
    from paper_1712_02443_amd import AIM_PRECOND_BLOCK_JACOBI
    wl, op, o, P = make(torch, CASES[0][0], **CASES[0][1])
    say(f"preconditioned gmres batch invariance prec={prec}")
    b = op.plane_wave_rhs(wl.theta, wl.phi, wl.pol)
    xb, sb, _ = op.gmres(b, restart=30, tol=1e-6, precision=prec, precond=AIM_PRECOND_BLOCK_JACOBI)
    x1, s1, _ = op.gmres(b[2:3].contiguous(), restart=30, tol=1e-6, precision=prec,
                         precond=AIM_PRECOND_BLOCK_JACOBI)
    assert torch.equal(xb[2], x1[0])
    assert sb[2]["iters"] == s1[0]["iters"]


def test_full_size_preconditioned_mixed_solve(torch):
    """The 32 x 32 Jerusalem-cross array at the benchmark's settings (GMRES(50), 1e-6):
    the preconditioned mixed solve converges in under half the iterations of the plain
    one, and its FP64 residual recomputed by the oracle over the whole vector meets the
    tolerance."""
    from paper_1712_02443_amd import AIM_MIXED, AIM_PRECOND_BLOCK_JACOBI, AimOperator
    wl = make_workload(1)
    say(f"full-size preconditioned solve {wl.name}")
    op = AimOperator.from_workload(wl)
    op.set_macromodels(wl.macromodels())
    op.set_dmatrix(*wl.d_matrix())
    op.build_preconditioner()
    b = op.plane_wave_rhs(wl.theta, wl.phi, wl.pol)
    xp, sp_, cp = op.gmres(b, restart=50, tol=1e-6, max_iters=3000, precision=AIM_MIXED, check_every=5,
                           precond=AIM_PRECOND_BLOCK_JACOBI)
    x0, s0, c0 = op.gmres(b, restart=50, tol=1e-6, max_iters=3000, precision=AIM_MIXED, check_every=5)
    assert cp == 0 and c0 == 0
    assert sp_[0]["true_relres"] <= 1e-6
    assert 2 * sp_[0]["iters"] < s0[0]["iters"]
    o = OracleOperator(wl)
    B = to_host(b)[0]
    relres = np.linalg.norm(B - o.matvec(to_host(xp)[0])) / np.linalg.norm(B)
    say(f"  oracle residual of the preconditioned mixed solve: {relres:.3e}")
    assert relres <= 1.01e-6
    op.close()
