"""The launch-configuration autotuner (paper_1712_02443_amd.autotune) and aim_set_tuning:
the tuned product still matches the oracle, the JSON cache is written and reused by a
second op of the same shape, and configurations the op cannot run are refused with
nothing changed."""
import sys

import numpy as np
import pytest

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


def make(wl):
    from paper_1712_02443_amd import AimOperator
    op = AimOperator.from_workload(wl)
    op.set_macromodels(wl.macromodels())
    op.set_dmatrix(*wl.d_matrix())
    return op


@pytest.mark.parametrize("prec", [1, 0])
def test_tuned_product_matches_oracle_and_cache_is_reused(torch, tmp_path, prec):
    from paper_1712_02443_amd.autotune import tune
    wl = make_workload(1, px=5, py=4, nrhs=2)
    cache = str(tmp_path / "tuning.json")
    op = make(wl)
    res = tune(op, nrhs=2, precision=prec, cache_path=cache, reps=3)
    say(f"tuned {res['key']}: {res['tuning']} {res['us']:.1f} us, tried {res['tried']}, rejected {res['rejected']}")
    assert not res["cached"] and res["tried"] > 1
    X = wl.test_vectors(2)
    o = OracleOperator(wl)
    ref = np.stack([o.matvec(x) for x in X])
    dt = torch.complex128 if prec == 0 else torch.complex64
    y = op.matvec(torch.from_numpy(X).to("cuda", dt), precision=prec).cpu().numpy()
    assert np.max(np.abs(y - ref)) / np.max(np.abs(ref)) < (1e-12 if prec == 0 else 1e-5)
    op2 = make(wl)
    res2 = tune(op2, nrhs=2, precision=prec, cache_path=cache)
    assert res2["cached"] and res2["tuning"] == res["tuning"]
    t1, t2 = op.tuning(), op2.tuning()
    assert t1 == t2
    op.close()
    op2.close()


def test_unusable_cache_entry_is_searched_again(torch, tmp_path):
    """A cached choice the library refuses (here a near-field blocking it does not offer)
    leaves the op's configuration alone, and the tuner searches again and replaces it."""
    import json
    from paper_1712_02443_amd.autotune import shape_key, tune
    wl = make_workload(1, px=5, py=4, nrhs=1)
    op = make(wl)
    cache = str(tmp_path / "tuning.json")
    bad = {"fft_b": 1, "interp_tile": [1, 1], "gemm_bf16": 1, "fft_register": 1, "near_block": 7}
    with open(cache, "w") as f:
        json.dump({shape_key(op, 1, 1): {"tuning": bad, "us": 1.0}}, f)
    res = tune(op, nrhs=1, precision=1, cache_path=cache, reps=2)
    say(f"re-tuned {res['key']}: {res['tuning']}, tried {res['tried']}")
    assert not res["cached"] and res["tried"] > 1 and res["tuning"]["near_block"] in (1, 2)
    with open(cache) as f:
        assert json.load(f)[res["key"]]["tuning"] == res["tuning"]
    op.close()


def test_invalid_tuning_is_refused(torch):
    from paper_1712_02443_amd import AimError
    wl = make_workload(0)
    op = make(wl)
    before = op.tuning()
    inf = op.info()
    bad_b = next(b for b in range(2, 50) if inf["ly"] % b)
    for kw in (dict(fft_b=(bad_b, 0)), dict(interp_tile=(3, 2)), dict(fft_b=(0, -1)), dict(near_block=(3, 0)),
               dict(near_block=(0, -1)), dict(near_fork=(3, -1)), dict(near_fork=(-1, -2))):
        with pytest.raises(AimError):
            op.set_tuning(**kw)
        assert op.tuning() == before
    op.close()


@pytest.mark.parametrize("idx", [0, 1])
def test_every_accepted_line_block_launches(torch, idx):
    """Each FFT line block / pass kind that aim_set_tuning accepts must launch and give
    the product of the default configuration (to rounding); the rest are refused."""
    from paper_1712_02443_amd import AimError
    wl = make_workload(idx, px=4, py=3, nrhs=1) if idx == 1 else make_workload(idx)
    op = make(wl)
    inf = op.info()
    x64 = torch.from_numpy(wl.test_vectors(1)).to("cuda")
    x32 = x64.to(torch.complex64)
    ref = op.matvec(x64, precision=0).cpu().numpy()
    scale = np.abs(ref).max()
    accepted = refused = 0
    for f4 in ([0, 1] if op.tuning()["fft_register"] else [0]):
        for b in range(1, inf["ly"] + 1):
            if inf["ly"] % b:
                continue
            try:
                op.set_tuning(fft_b=(b, b), fft_register=f4)
            except AimError:
                refused += 1
                continue
            accepted += 1
            y64 = op.matvec(x64, precision=0).cpu().numpy()
            y32 = op.matvec(x32, precision=1).cpu().numpy()
            assert np.abs(y64 - ref).max() / scale < 1e-12, (f4, b)
            assert np.abs(y32 - ref).max() / scale < 1e-5, (f4, b)
    say(f"ly={inf['ly']}: {accepted} line blocks accepted, {refused} refused")
    assert accepted >= 1 and refused >= 1
    op.close()


@pytest.mark.parametrize("idx", [0, 4])
def test_near_blocks_give_identical_products(torch, idx):
    """One or two blocks of 16 elements per near-field workgroup do the same sums per
    element in the same order, and the fork point of the near field's stream only moves
    when it runs: the products are bit-identical, in both precisions, on a 2 x 2 array
    and on a ragged 5 x 3 slice of the two-kind 648-RWG array."""
    wl = make_workload(idx, px=5, py=3, nrhs=2) if idx == 4 else make_workload(idx)
    op = make(wl)
    X = torch.from_numpy(wl.test_vectors(wl.nrhs)).to("cuda")
    for prec, x in ((0, X), (1, X.to(torch.complex64))):
        ys = []
        for nb in (1, 2):
            for fork in (0, 1, 2):
                op.set_tuning(near_block=(nb, nb), near_fork=(fork, fork))
                assert op.tuning()["near_block"] == [nb, nb] and op.tuning()["near_fork"] == [fork, fork]
                ys.append(op.matvec(x, precision=prec).cpu().numpy())
        for y in ys[1:]:
            assert np.array_equal(ys[0], y), f"precision {prec}: max diff {np.abs(ys[0] - y).max()}"
    op.close()
