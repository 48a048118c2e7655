"""Device far field (radiation pattern and bistatic RCS of the equivalent currents)
through the C ABI against the oracle's radiated field, FP64 (<= 1e-12 relative)."""
import sys

import numpy as np
import pytest

from oracle.excitation import radiated_field, rcs_db
from oracle.system import OracleOperator
from synth import make_workload

pytestmark = pytest.mark.gpu


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
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(np.asarray(b))))


def directions(n_random, seed=3):
    """Two principal cuts (37 directions each, the poles included) plus random directions."""
    th = np.linspace(0, np.pi, 37)
    cuts = np.concatenate([np.stack([np.sin(th), np.zeros_like(th), np.cos(th)], 1),
                           np.stack([np.zeros_like(th), np.sin(th), np.cos(th)], 1)])
    v = np.random.default_rng(seed).standard_normal((n_random, 3))
    return np.concatenate([cuts, v / np.linalg.norm(v, axis=1, keepdims=True)])


def make(idx, **kw):
    from paper_1712_02443_amd import AimOperator
    wl = make_workload(idx, **kw)
    say(f"build {wl.name} px={wl.px} py={wl.py} types={wl.n_types} rhs={wl.nrhs}")
    op = AimOperator.from_workload(wl)
    op.set_macromodels(wl.macromodels())
    op.set_dmatrix(*wl.d_matrix())
    return wl, op, OracleOperator(wl)


@pytest.mark.parametrize("case", [(0, {}), (2, dict(px=5, py=3, nrhs=3)), (1, dict(px=4, py=3, nrhs=2))])
def test_far_field_matches_oracle(torch, case):
    wl, op, o = make(case[0], **case[1])
    say(f"far field {wl.name}")
    X = wl.test_vectors()
    rh = directions(61)
    E, rcs = op.far_field(torch.from_numpy(X).to("cuda"), rh)
    E, rcs = E.cpu().numpy(), rcs.cpu().numpy()
    centers = wl.elem_center()
    for r in range(X.shape[0]):
        ref = radiated_field(o.geo, centers, -o.macro_apply(X[r]), rh, wl.k, wl.eta)
        assert rel(E[r], ref) < 1e-12
        keep = np.linalg.norm(ref, axis=1) > 1e-6 * np.abs(ref).max()
        assert np.max(np.abs(rcs[r][keep] - rcs_db(ref)[keep])) < 1e-9
    op.close()


def test_far_field_workspace_grows_and_shrinks(torch):
    """Calls with more, then fewer directions than before give the same values."""
    wl, op, o = make(0)
    x = torch.from_numpy(wl.test_vectors()).to("cuda")
    rh = directions(200)
    E_small, _ = op.far_field(x, rh[:5])
    E_big, _ = op.far_field(x, rh)
    E_again, _ = op.far_field(x, rh[:5])
    assert torch.equal(E_small, E_again)
    assert torch.equal(E_big[:, :5], E_small)
    op.close()


def test_full_size_far_field(torch):
    """The 32 x 32 array (1,024 elements) at 24 directions, one solution-sized vector."""
    wl, op, o = make(1)
    say("full-size far field")
    x = wl.test_vectors(1)
    rh = directions(0)[::3]
    E, rcs = op.far_field(torch.from_numpy(x).to("cuda"), rh)
    ref = radiated_field(o.geo, wl.elem_center(), -o.macro_apply(x[0]), rh, wl.k, wl.eta)
    assert rel(E.cpu().numpy()[0], ref) < 1e-12
    op.close()


@pytest.mark.parametrize("case", [(0, {}), (1, dict(px=4, py=3, nrhs=1))])
def test_device_rcs_of_mixed_solve_matches_fp64_oracle(torch, case):
    """Solve and RCS both on the device (mixed-precision GMRES to 1e-6, FP64 far field)
    within 0.05 dB of the FP64 oracle solve's RCS, over two cuts of 73 directions
    (directions within 40 dB of the cut's peak)."""
    from oracle.gmres import gmres as oracle_gmres
    from paper_1712_02443_amd import AIM_MIXED
    wl, op, o = make(case[0], **case[1])
    say(f"device rcs {wl.name}")
    b = op.plane_wave_rhs(wl.theta, wl.phi, wl.pol)
    xm, sm, cm = op.gmres(b[:1].contiguous(), restart=50, tol=1e-6, max_iters=3000, precision=AIM_MIXED)
    assert cm == 0 and sm[0]["converged"]
    xo, info = oracle_gmres(o.matvec, b.cpu().numpy()[0], restart=50, tol=1e-10, max_iters=3000)
    assert info["converged"]
    th = np.linspace(0, np.pi, 73)
    rh = np.concatenate([np.stack([np.sin(th), np.zeros_like(th), np.cos(th)], 1),
                         np.stack([np.zeros_like(th), np.sin(th), np.cos(th)], 1)])
    _, db_dev = op.far_field(xm, rh)
    db_o = rcs_db(radiated_field(o.geo, wl.elem_center(), -o.macro_apply(xo), rh, wl.k, wl.eta))
    keep = db_o > db_o.max() - 40.0
    assert keep.sum() > 60
    assert np.max(np.abs(db_dev.cpu().numpy()[0] - db_o)[keep]) <= 0.05
    op.close()
