"""GMRES inner iterations captured as HIP graphs (one per iteration index, replayed in
later cycles and solves, gmres(graphs=True)) against the same solves launched kernel
by kernel: every replay gives bit-identical solutions and iteration counts, with
the program's own eager work and synchronisations between replays, after the element
kinds change (the captured graphs must be dropped), and with preconditioning."""
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


def solve(op, b, graphs, **kw):
    x, st, code = op.gmres(b, graphs=graphs, **kw)
    assert code == 0
    return x.cpu().numpy(), [s["iters"] for s in st]


@pytest.mark.parametrize("prec,pc", [(1, 0), (0, 0), (1, 1)])
def test_graph_replays_match_eager_solves(torch, prec, pc):
    from paper_1712_02443_amd import AimOperator
    wl = make_workload(2, px=6, py=5, nrhs=3)
    op = AimOperator.from_workload(wl)
    op.build_macromodels(wl.element_meshes())
    if pc:
        op.build_preconditioner()
    b = op.plane_wave_rhs(wl.theta, wl.phi, wl.pol)
    kw = dict(restart=20, tol=1e-8, max_iters=2000, precision=prec, precond=pc, check_every=3)
    say(f"eager solve prec={prec} precond={pc}")
    xe, ie = solve(op, b, False, **kw)
    say(f"  iterations {ie}")
    y = torch.empty_like(b)
    for rep in range(3):
        xg, ig = solve(op, b, True, **kw)
        assert ig == ie
        assert np.array_equal(xg, xe), f"replay {rep}: max diff {np.abs(xg - xe).max()}"
        # eager work and a synchronisation between replays
        op.matvec(b, out=y)
        torch.cuda.synchronize()
    # new element kinds: captured launches carry the old kind counts and must be rebuilt
    et = np.roll(wl.elem_type, 7)
    op.set_elem_type(et)
    xe2, ie2 = solve(op, b, False, **kw)
    xg2, ig2 = solve(op, b, True, **kw)
    assert ig2 == ie2 and np.array_equal(xg2, xe2)
    assert not np.array_equal(xe2, xe)
    op.close()
