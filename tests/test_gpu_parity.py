"""Parity of the HIP path (through the C ABI) with the CPU oracle, on seeded inputs.

Tolerances: FP64 path <= 1e-12 relative, mixed (complex FP32) path <= 1e-5 relative,
both measured as max |gpu - oracle| / max |oracle| over the compared outputs.
"""
import sys

import numpy as np
import pytest

from oracle import aim
from oracle.excitation import plane_wave_rhs
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


def make_pair(torch, idx, max_rhs=None, **kw):
    """Device op and oracle op for one workload (cached per module)."""
    key = (idx, tuple(sorted(kw.items())), max_rhs)
    if key not in _OPS:
        from paper_1712_02443_amd import AimOperator
        wl = make_workload(idx, **kw)
        say(f"build {wl.name} px={wl.px} py={wl.py} types={wl.n_types} rhs={wl.nrhs}")
        op = AimOperator.from_workload(wl, max_rhs=max_rhs)
        op.set_macromodels(wl.macromodels())
        op.set_dmatrix(*wl.d_matrix())
        _OPS[key] = (wl, op, OracleOperator(wl))
    return _OPS[key]


def to_dev(torch, a, prec):
    dt = torch.complex128 if prec == 0 else torch.complex64
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dt)


def to_host(t):
    return t.detach().cpu().numpy().astype(np.complex128)


CASES = [(0, {}), (2, dict(px=5, py=3, nrhs=3)), (1, dict(px=4, py=3, nrhs=2))]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("case", CASES)
def test_projection(torch, case, prec):
    wl, op, o = make_pair(torch, case[0], **case[1])
    say(f"project {wl.name} prec={prec}")
    u = wl.test_vectors(1)[0]
    Q = to_host(op.project(to_dev(torch, u, prec), precision=prec))[0]
    ref = aim.project(o.grid, o.W, u)
    assert rel(Q, ref) < TOL[prec]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("case", CASES)
def test_convolution(torch, case, prec):
    wl, op, o = make_pair(torch, case[0], **case[1])
    say(f"convolve {wl.name} prec={prec}")
    rng = np.random.default_rng(7)
    Q = rng.standard_normal((1, 4) + o.grid.shape) + 1j * rng.standard_normal((1, 4) + o.grid.shape)
    Phi = to_host(op.convolve(to_dev(torch, Q, prec), precision=prec))[0]
    ref = aim.convolve_fft(Q[0], o.Gs)
    assert rel(Phi, ref) < TOL[prec] * (3 if prec == 1 else 1)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("case", CASES)
def test_far_and_g_parts(torch, case, prec):
    from paper_1712_02443_amd import AIM_FAR_ONLY, AIM_G_ONLY
    wl, op, o = make_pair(torch, case[0], **case[1])
    say(f"far/G parts {wl.name} prec={prec}")
    u = wl.test_vectors(1)[0]
    far = to_host(op.matvec(to_dev(torch, u, prec), precision=prec, flags=AIM_FAR_ONLY))
    assert rel(far, o.far_field(u)) < TOL[prec]
    g = to_host(op.matvec(to_dev(torch, u, prec), precision=prec, flags=AIM_G_ONLY))
    assert rel(g, o.g_apply(u)) < TOL[prec]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("case", CASES)
def test_macro_apply(torch, case, prec):
    wl, op, o = make_pair(torch, case[0], **case[1])
    say(f"macro {wl.name} prec={prec}")
    X = wl.test_vectors()
    U = to_host(op.macro_apply(to_dev(torch, X, prec), precision=prec))
    ref = np.stack([o.macro_apply(x) for x in X])
    assert rel(U, ref) < TOL[prec]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("case", CASES)
def test_full_product(torch, case, prec):
    wl, op, o = make_pair(torch, case[0], **case[1])
    say(f"full product {wl.name} prec={prec} rhs={wl.nrhs}")
    X = wl.test_vectors()
    Y = to_host(op.matvec(to_dev(torch, X, prec), precision=prec))
    ref = o.matvec(X)
    assert rel(Y, ref) < TOL[prec]


@pytest.mark.parametrize("prec", [0, 1])
def test_kernel_timing_leaves_the_product(torch, prec):
    """aim_time_kernels times every kernel and still returns the full product."""
    wl, op, o = make_pair(torch, CASES[2][0], **CASES[2][1])
    say(f"kernel timing {wl.name} prec={prec} rhs={wl.nrhs}")
    X = wl.test_vectors()
    x = to_dev(torch, X, prec)
    y = torch.empty_like(x)
    t = op.time_kernels(x, precision=prec, reps=3, out=y)
    assert set(t) == set(op.KERNELS) and all(v > 0 for v in t.values())
    assert rel(to_host(y), o.matvec(X)) < TOL[prec]


@pytest.mark.parametrize("case", [CASES[0], CASES[2]])
def test_radix_stage_fft_path(torch, case, monkeypatch):
    """The radix-stage FFT passes (used for lengths without a register-DFT
    factorisation) against the oracle, forced on lengths that have one."""
    from paper_1712_02443_amd import AimOperator
    wl, op_fast, o = make_pair(torch, case[0], **case[1])
    assert op_fast.info()["paths"] & 1, "register-DFT FFT passes expected on these lengths"
    monkeypatch.setenv("AIMM_FFT4", "0")
    op = AimOperator.from_workload(wl)
    op.set_macromodels(wl.macromodels())
    op.set_dmatrix(*wl.d_matrix())
    assert not op.info()["paths"] & 1
    say(f"radix-stage FFT {wl.name}")
    rng = np.random.default_rng(7)
    Q = rng.standard_normal((1, 4) + o.grid.shape) + 1j * rng.standard_normal((1, 4) + o.grid.shape)
    for prec in (0, 1):
        Phi = to_host(op.convolve(to_dev(torch, Q, prec), precision=prec))[0]
        assert rel(Phi, aim.convolve_fft(Q[0], o.Gs)) < TOL[prec] * (3 if prec == 1 else 1)
        X = wl.test_vectors()
        assert rel(to_host(op.matvec(to_dev(torch, X, prec), precision=prec)), o.matvec(X)) < TOL[prec]
    op.close()


@pytest.mark.parametrize("case", [CASES[1], CASES[2]])
def test_fp32_gemm_path(torch, case, monkeypatch):
    """The mixed path's FP32-MFMA macromodel product (the alternative to the split-BF16
    one) against the oracle; the default op must be on the split-BF16 kernel."""
    from paper_1712_02443_amd import AIM_MIXED, AimOperator
    wl, op_fast, o = make_pair(torch, case[0], **case[1])
    assert op_fast.info()["paths"] & 4, "split-BF16 macromodel product expected"
    monkeypatch.setenv("AIMM_GEMM", "fp32")
    op = AimOperator.from_workload(wl)
    op.set_macromodels(wl.macromodels())
    op.set_dmatrix(*wl.d_matrix())
    assert not op.info()["paths"] & 4
    say(f"fp32 gemm {wl.name}")
    X = wl.test_vectors()
    U = to_host(op.macro_apply(to_dev(torch, X, AIM_MIXED), precision=AIM_MIXED))
    assert rel(U, np.stack([o.macro_apply(x) for x in X])) < TOL[1]
    assert rel(to_host(op.matvec(to_dev(torch, X, AIM_MIXED), precision=AIM_MIXED)), o.matvec(X)) < TOL[1]
    op.close()


def test_product_is_deterministic_and_batch_invariant(torch):
    wl, op, o = make_pair(torch, 2, px=5, py=3, nrhs=3)
    say("determinism")
    X = to_dev(torch, wl.test_vectors(), 0)
    a = op.matvec(X)
    b = op.matvec(X)
    assert torch.equal(a, b)
    one = op.matvec(X[1:2].contiguous())
    assert torch.equal(one[0], a[1])


def test_plane_wave_rhs(torch):
    wl, op, o = make_pair(torch, 2, px=5, py=3, nrhs=3)
    say("plane-wave rhs")
    b = to_host(op.plane_wave_rhs(wl.theta, wl.phi, wl.pol))
    for r in range(wl.nrhs):
        ref = plane_wave_rhs(o.geo, wl.elem_center(), wl.theta[r], wl.phi[r], wl.pol[r], wl.k)
        assert rel(b[r], ref) < 1e-13


def test_gmres_fp64_matches_oracle(torch):
    wl, op, o = make_pair(torch, 0)
    say("gmres fp64 vs oracle")
    b = op.plane_wave_rhs(wl.theta, wl.phi, wl.pol)
    x, st, code = op.gmres(b, restart=20, tol=1e-11, max_iters=2000)
    assert code == 0 and st[0]["converged"] and st[0]["true_relres"] <= 1e-11
    xo, info = oracle_gmres(o.matvec, to_host(b)[0], restart=20, tol=1e-11, max_iters=2000)
    assert rel(to_host(x)[0], xo) < 1e-8
    # same Krylov process: iteration counts agree closely at the benchmark tolerance
    x6, st6, _ = op.gmres(b, restart=50, tol=1e-6)
    _, info6 = oracle_gmres(o.matvec, to_host(b)[0], restart=50, tol=1e-6)
    assert abs(st6[0]["iters"] - info6["iters"]) <= 2


def test_gmres_mixed_reaches_fp64_residual(torch):
    from paper_1712_02443_amd import AIM_MIXED
    wl, op, o = make_pair(torch, 2, px=5, py=3, nrhs=3)
    say("gmres mixed")
    b = op.plane_wave_rhs(wl.theta, wl.phi, wl.pol)
    x64, s64, c64 = op.gmres(b, restart=50, tol=1e-10, max_iters=3000)
    xm, sm, cm = op.gmres(b, restart=50, tol=1e-10, max_iters=3000, precision=AIM_MIXED)
    assert c64 == 0 and cm == 0
    for s in sm:
        assert s["converged"] and s["true_relres"] <= 1e-10
    assert rel(to_host(xm), to_host(x64)) < 1e-5
    # the true residual of the mixed solution, recomputed by the oracle
    X = to_host(xm)
    B = to_host(b)
    for r in range(wl.nrhs):
        res = np.linalg.norm(B[r] - o.matvec(X[r])) / np.linalg.norm(B[r])
        assert res <= 1e-9


@pytest.mark.parametrize("case", [(0, {}), (1, dict(px=4, py=3, nrhs=1))])
def test_mixed_solve_rcs_matches_fp64_oracle(torch, case):
    """Bistatic RCS of the mixed-precision solve at the benchmark's tolerance (1e-6)
    within 0.05 dB of an FP64 oracle solve, over two cuts of 73 directions (directions
    within 40 dB of the cut's peak; deep nulls are excluded)."""
    from oracle.excitation import radiated_field, rcs_db
    from paper_1712_02443_amd import AIM_MIXED
    wl, op, o = make_pair(torch, case[0], **case[1])
    say(f"rcs {wl.name}")
    b = op.plane_wave_rhs(wl.theta, wl.phi, wl.pol)
    xm, sm, cm = op.gmres(b[:1].contiguous(), restart=50, tol=1e-6, max_iters=3000, precision=AIM_MIXED)
    assert cm == 0 and sm[0]["converged"]
    B = to_host(b)[0]
    xo, info = oracle_gmres(o.matvec, B, restart=50, tol=1e-10, max_iters=3000)
    assert info["converged"]
    th = np.linspace(0, np.pi, 73)
    rhat = np.concatenate([np.stack([np.sin(th), np.zeros_like(th), np.cos(th)], 1),
                           np.stack([np.zeros_like(th), np.sin(th), np.cos(th)], 1)])
    centers = wl.elem_center()
    db_m = rcs_db(radiated_field(o.geo, centers, -o.macro_apply(to_host(xm)[0]), rhat, wl.k, wl.eta))
    db_o = rcs_db(radiated_field(o.geo, centers, -o.macro_apply(xo), rhat, wl.k, wl.eta))
    keep = db_o > db_o.max() - 40.0
    assert keep.sum() > 60
    assert np.max(np.abs(db_m - db_o)[keep]) <= 0.05


@pytest.mark.parametrize("prec", [0, 1])
def test_gmres_alone_equals_in_batch(torch, prec):
    wl, op, o = make_pair(torch, 2, px=5, py=3, nrhs=3)
    say(f"gmres batch invariance prec={prec}")
    b = op.plane_wave_rhs(wl.theta, wl.phi, wl.pol)
    xb, sb, _ = op.gmres(b, restart=30, tol=1e-6, precision=prec)
    x1, s1, _ = op.gmres(b[2:3].contiguous(), restart=30, tol=1e-6, precision=prec)
    assert torch.equal(xb[2], x1[0])
    assert sb[2]["iters"] == s1[0]["iters"]


def test_gmres_reports_nonconvergence(torch):
    wl, op, o = make_pair(torch, 0)
    say("gmres max_iters")
    b = op.plane_wave_rhs(wl.theta, wl.phi, wl.pol)
    x, st, code = op.gmres(b, restart=5, tol=1e-12, max_iters=7)
    assert code == 1 and not st[0]["converged"] and st[0]["iters"] == 7


@pytest.fixture(scope="module")
def full1(torch):
    """The 32 x 32 Jerusalem-cross array (663,552 unknowns, 400 x 400 FFT) with the oracle's
    full product of one test vector (seeded operator data, as the product kernels' parity
    does not depend on the values)."""
    wl, op, o = make_pair(torch, 1)
    x = wl.test_vectors(1)[0]
    say("full-size oracle product")
    return wl, op, o, x, o.matvec(x)


@pytest.mark.parametrize("prec", [0, 1])
def test_full_size_full_vector(torch, full1, prec):
    """The full-size product in the launch configuration the benchmark times, every one of
    the 663,552 rows against the oracle."""
    wl, op, o, x, ref = full1
    say(f"full-size full vector prec={prec}")
    y = to_host(op.matvec(to_dev(torch, x[None], prec), precision=prec))[0]
    err = rel(y, ref)
    say(f"  max relative error over {y.size} rows: {err:.2e}")
    assert err < TOL[prec]


@pytest.mark.timeout(900)
def test_full_size_rcs_mixed_vs_oracle_fp64_solve(torch, full1):
    """Mixed device solve of the full 32 x 32 array against the oracle's FP64 GMRES solve of
    the same system: bistatic RCS on two principal cuts within 0.05 dB wherever within
    20 dB of the peak (the oracle solve takes about a minute)."""
    from oracle.excitation import radiated_field, rcs_db
    from paper_1712_02443_amd import AIM_MIXED
    wl, op, o, _, _ = full1
    b = op.plane_wave_rhs(wl.theta, wl.phi, wl.pol)
    xm, st, code = op.gmres(b, precision=AIM_MIXED, restart=50, tol=1e-6, check_every=5)
    assert code == 0
    say("oracle FP64 solve of the full array")
    xo, info = oracle_gmres(o.matvec, b.cpu().numpy()[0], restart=50, tol=1e-6)
    th = np.linspace(0.0, np.pi, 181)
    rh = np.concatenate([np.stack([np.sin(th), np.zeros_like(th), np.cos(th)], 1),
                         np.stack([np.zeros_like(th), np.sin(th), np.cos(th)], 1)])
    _, db_dev = op.far_field(xm, rh)
    db_dev = db_dev.cpu().numpy()[0]
    db_o = rcs_db(radiated_field(o.geo, wl.elem_center(), -o.macro_apply(xo), rh, wl.k, wl.eta))
    keep = db_o >= db_o.max() - 20.0
    err = float(np.max(np.abs(db_dev[keep] - db_o[keep])))
    say(f"  RCS max |difference| {err:.4f} dB over {int(keep.sum())} directions")
    assert err < 0.05


@pytest.mark.timeout(600)
@pytest.mark.parametrize("idx", [2, 4])
def test_full_size_multi_rhs_full_vectors(torch, idx):
    """The two multi-RHS workloads at full size, all right-hand sides in one launch:
    16 x 16 plates of three kinds with 64 RHS (73,728 unknowns each, 200 x 200 FFT) and
    the 64 x 64 two-kind array with 8 RHS (2,654,208 unknowns each, 800 x 800 FFT).
    First and last RHS checked over every row against the oracle, both precisions."""
    from paper_1712_02443_amd import AimOperator
    wl = make_workload(idx)
    say(f"full-size {wl.name}: {wl.nrhs} rhs x {wl.n_unknowns}")
    op = AimOperator.from_workload(wl)
    op.set_macromodels(wl.macromodels())
    op.set_dmatrix(*wl.d_matrix())
    o = OracleOperator(wl)
    X = wl.test_vectors()
    refs = {r: o.matvec(X[r]) for r in (0, wl.nrhs - 1)}
    for prec in (0, 1):
        Y = op.matvec(to_dev(torch, X, prec), precision=prec)
        for r, ref in refs.items():
            err = rel(to_host(Y[r]), ref)
            say(f"  prec={prec} rhs={r}: max relative error {err:.2e} over {ref.size} rows")
            assert err < TOL[prec]
        del Y
    op.close()
