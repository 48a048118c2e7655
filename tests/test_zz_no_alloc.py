"""aim_far_field_noalloc (library scratch array, no device allocation) through the C ABI
against aim_far_field (op workspace) on the same inputs: two calls in a row, the second
with fewer directions and right-hand sides, then a call too large for the scratch array."""
import sys

import numpy as np
import pytest

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


def directions(n, seed):
    v = np.random.default_rng(seed).standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def test_noalloc_far_field_matches_workspace_path(torch):
    from paper_1712_02443_amd import AIM_FULL, AIM_G_ONLY, AimError, AimOperator
    from paper_1712_02443_amd._lib import AIM_EINVAL
    wl = make_workload(2, px=5, py=4, nrhs=3)
    say(f"build {wl.name} px={wl.px} py={wl.py} rhs={wl.nrhs}")
    op = AimOperator.from_workload(wl)
    op.set_macromodels(wl.macromodels())
    op.set_dmatrix(*wl.d_matrix())
    X = torch.from_numpy(wl.test_vectors()).to("cuda")
    for system in (AIM_FULL, AIM_G_ONLY):
        for step, (nr, nd, seed) in enumerate(((3, 150, 1), (2, 37, 2))):
            say(f"far field system={system} call={step} nrhs={nr} ndir={nd}")
            rh = directions(nd, seed)
            x = X[:nr].contiguous()
            E_ref, db_ref = op.far_field(x, rh, system=system)
            # outputs pre-filled with garbage: the no-allocation call must write all of them
            E = torch.full_like(E_ref, complex(np.nan, np.nan))
            db = torch.full_like(db_ref, np.nan)
            op.far_field(x, rh, system=system, out=(E, db), noalloc=True)
            torch.cuda.synchronize()
            Eh, Er = E.cpu().numpy(), E_ref.cpu().numpy()
            assert np.all(np.isfinite(Eh))
            err = float(np.max(np.abs(Eh - Er)) / np.max(np.abs(Er)))
            say(f"  max relative difference {err:.2e}")
            assert err <= 1e-12
            assert np.max(np.abs(db.cpu().numpy() - db_ref.cpu().numpy())) <= 1e-9
    # more than the 16 MiB scratch array holds: rejected, outputs untouched
    big = directions(40000, 5)
    E = torch.zeros((3, big.shape[0], 3), dtype=torch.complex128, device="cuda")
    db = torch.zeros((3, big.shape[0]), dtype=torch.float64, device="cuda")
    with pytest.raises(AimError) as ei:
        op.far_field(X, big, out=(E, db), noalloc=True)
    assert ei.value.code == AIM_EINVAL
    assert "scratch" in str(ei.value)
    assert not bool(E.abs().max()) and not bool(db.abs().max())
    op.close()
