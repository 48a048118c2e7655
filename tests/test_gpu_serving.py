"""The request loop (paper_1712_02443_amd.serving) on a short seeded trace of the serving
workload (square plate arrays of random size, kinds and right-hand sides): every
request's solution is the same when it runs alone and when it runs in the mix of
concurrent requests on several streams, with operators admitted under a memory budget
small enough to force waiting and eviction."""
import sys

import numpy as np
import pytest

from synth import make_workload, serving_trace

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


def server(workers, budget, keep=True):
    from paper_1712_02443_amd.serving import ArrayServer
    wl = make_workload(2, px=2, py=2, nrhs=1)
    return ArrayServer(wl.surface, wl.element_meshes(), k=wl.k, eta=wl.eta, h=wl.h, r_near=wl.r_near,
                       order=wl.order, pitch_cells=wl.pitch_cells, max_rhs=4, workers=workers,
                       mem_budget_bytes=budget, keep_solutions=keep)


def test_results_alone_and_in_the_mix(torch):
    from paper_1712_02443_amd.serving import summarize
    trace = serving_trace(seed=3, n_requests=12, side_range=(4, 7), rhs_range=(1, 4))
    say(f"trace: sides {[r.side for r in trace]}, rhs {[len(r.theta) for r in trace]}")
    alone = server(1, 64 << 30)
    xs = []
    for i, req in enumerate(trace):
        x, st, code, _ = alone.solve(req)
        torch.cuda.synchronize()
        assert code == 0
        xs.append(x.cpu().numpy())
    alone.close()
    # the mix: four workers, arrivals 200x faster than the trace, a budget of about two of
    # the largest operators (so requests wait for memory and idle operators are evicted)
    big = server(4, 1)._footprint(7)
    mix = server(4, int(2.2 * big))
    recs = mix.run(trace, speed=200.0)
    say(f"mix: built {mix.ops_built} ops, evicted {mix.ops_evicted}; {summarize(recs)}")
    assert not mix.errors, mix.errors
    assert mix.ops_evicted > 0
    bitwise = True
    for rec, xa in zip(recs, xs):
        assert rec.converged
        err = float(np.max(np.abs(rec.x - xa)) / np.max(np.abs(xa)))
        bitwise = bitwise and err == 0.0
        assert err <= 1e-5, (rec.index, err)
    say(f"solutions identical bit for bit: {bitwise}")
    mix.close()


def test_operator_too_large_for_the_budget_is_refused(torch):
    srv = server(1, 1 << 20)
    req = serving_trace(seed=1, n_requests=1, side_range=(4, 4), rhs_range=(1, 1))[0]
    with pytest.raises(MemoryError):
        srv.solve(req)
    srv.close()
