"""Host logic of the launch-configuration tuner (paper_1712_02443_amd.autotune), on a
stand-in op that records the configurations it is given (no device): candidates cover
the kernels' launch choices with the fork point at its first value, a configuration is
applied to one precision only (the other precision's fields keep their values), and a
cache entry the op refuses does not stop the tuner."""
import json

import pytest

from paper_1712_02443_amd import AIM_FP64, AIM_MIXED, AimError
from paper_1712_02443_amd import autotune


class FakeOp:
    def __init__(self, ly=400, n_rwg=648, refuse=None):
        self.calls = []
        self.refuse = refuse or (lambda kw: False)
        self._info = {"nx": 200, "ny": 200, "nz": 9, "lx": 400, "ly": ly, "n_rwg": n_rwg, "n_elem": 1024,
                      "paths": 1}

    def info(self):
        return dict(self._info)

    def tuning(self):
        return {"fft_b": [1, 1], "interp_tile": [1, 1], "gemm_bf16": 1, "fft_register": 1, "near_block": [1, 1],
                "near_fork": [0, 0]}

    def set_tuning(self, **kw):
        if self.refuse(kw):
            raise AimError(-1, "refused")
        self.calls.append(kw)


def test_candidates_cover_the_launch_choices():
    op = FakeOp()
    mixed = list(autotune._candidates(op, AIM_MIXED))
    fp64 = list(autotune._candidates(op, AIM_FP64))
    assert {c["near_block"] for c in mixed} == {1, 2}
    assert {c["near_fork"] for c in mixed} == {0}  # the other fork points are tried on the best one
    assert {c["gemm_bf16"] for c in mixed} == {0, 1} and {c["gemm_bf16"] for c in fp64} == {1}
    assert all(400 % c["fft_b"] == 0 for c in mixed)
    assert {tuple(c["interp_tile"]) for c in mixed} == {(1, 1), (2, 1), (1, 2), (2, 2)}
    assert {c["gemm_bf16"] for c in autotune._candidates(FakeOp(n_rwg=650), AIM_MIXED)} == {0}


@pytest.mark.parametrize("prec", [AIM_FP64, AIM_MIXED])
def test_apply_sets_one_precision(prec):
    op = FakeOp()
    cand = {"fft_b": 2, "interp_tile": [1, 2], "gemm_bf16": 1, "fft_register": 1, "near_block": 2, "near_fork": 1}
    autotune._apply(op, cand, prec)
    kw = op.calls[-1]
    mine, other = (0, 1) if prec == AIM_FP64 else (1, 0)
    assert kw["fft_b"][mine] == 2 and kw["fft_b"][other] == 0
    assert kw["near_block"][mine] == 2 and kw["near_block"][other] == 0
    assert kw["near_fork"][mine] == 1 and kw["near_fork"][other] == -1
    # an entry written before the fork point was a tuning field applies with the default point
    old = {k: v for k, v in cand.items() if k != "near_fork"}
    autotune._apply(op, old, prec)
    assert op.calls[-1]["near_fork"][mine] == 0


def test_refused_cache_entry_falls_through_to_the_search(tmp_path, monkeypatch):
    op = FakeOp(refuse=lambda kw: kw["near_block"][1] == 7)
    cache = tmp_path / "tuning.json"
    key = autotune.shape_key(op, 1, AIM_MIXED)
    bad = {"fft_b": 1, "interp_tile": [1, 1], "gemm_bf16": 1, "fft_register": 1, "near_block": 7}
    cache.write_text(json.dumps({key: {"tuning": bad, "us": 1.0}}))
    reached = []

    class Stop(Exception):
        pass

    def no_device(*a, **k):  # the search needs the device: stop where it would start
        reached.append(True)
        raise Stop

    monkeypatch.setattr(autotune.np.random, "default_rng", no_device)
    with pytest.raises(Stop):
        autotune.tune(op, nrhs=1, precision=AIM_MIXED, cache_path=str(cache))
    assert reached


def test_usable_cache_entry_is_applied(tmp_path):
    op = FakeOp()
    cache = tmp_path / "tuning.json"
    key = autotune.shape_key(op, 4, AIM_FP64)
    good = {"fft_b": 2, "interp_tile": [2, 1], "gemm_bf16": 1, "fft_register": 1, "near_block": 2, "near_fork": 2}
    cache.write_text(json.dumps({key: {"tuning": good, "us": 12.5}}))
    res = autotune.tune(op, nrhs=4, precision=AIM_FP64, cache_path=str(cache))
    assert res["cached"] and res["tuning"] == good and res["us"] == 12.5
    assert op.calls[-1]["near_fork"] == [2, -1] and op.calls[-1]["interp_tile"] == [2, 1]
