"""Autotuner of the product's launch configuration (aim_set_tuning): x-pass FFT line
block, interpolation element tile, macromodel GEMM kernel, FFT pass kind, near-field
element blocks per workgroup and the point where the near field forks to the op's second
stream.

For one op, right-hand-side count and precision it times every admissible candidate
with HIP events around back-to-back products, keeps only candidates whose product
agrees with the op's FP64 product within the precision's tolerance (1e-12 FP64, 1e-5
mixed; the candidates differ only in rounding order), applies the fastest, and records
the choice in a JSON cache keyed by grid, padded FFT lengths, N, element count,
right-hand sides and precision, so later ops of the same shape skip the search.
The products themselves run in the library's kernels; this module only chooses.
"""
from __future__ import annotations

import itertools
import json
import os
import time

import numpy as np

from . import AIM_FP64, AIM_MIXED, AimError

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "aimm", "tuning.json")


def shape_key(op, nrhs: int, precision: int) -> str:
    inf = op.info()
    return (f"grid{inf['nx']}x{inf['ny']}x{inf['nz']}-L{inf['lx']}x{inf['ly']}-N{inf['n_rwg']}-"
            f"elems{inf['n_elem']}-R{nrhs}-{'fp64' if precision == AIM_FP64 else 'mixed'}")


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _candidates(op, precision):
    cur = op.tuning()
    inf = op.info()
    fft_b = sorted({1, 2, 3, 4, 5} & {b for b in range(1, 6) if inf["ly"] % b == 0})
    tiles = [(1, 1), (2, 1), (1, 2), (2, 2)]
    gemm = [cur["gemm_bf16"]] if precision == AIM_FP64 else ([0, 1] if inf["n_rwg"] % 8 == 0 else [0])
    fftk = [0, 1] if cur["fft_register"] or (inf["paths"] & 1) else [0]
    for b, t, g, f, nb in itertools.product(fft_b, tiles, gemm, fftk, (1, 2)):
        yield {"fft_b": b, "interp_tile": list(t), "gemm_bf16": g, "fft_register": f, "near_block": nb,
               "near_fork": 0}


def _apply(op, cand, precision):
    fb = [cand["fft_b"], 0] if precision == AIM_FP64 else [0, cand["fft_b"]]
    nb = cand.get("near_block", 0)
    nf = cand.get("near_fork", 0)
    op.set_tuning(fft_b=fb, interp_tile=cand["interp_tile"], gemm_bf16=cand["gemm_bf16"],
                  fft_register=cand["fft_register"], near_block=[nb, 0] if precision == AIM_FP64 else [0, nb],
                  near_fork=[nf, -1] if precision == AIM_FP64 else [-1, nf])


def tune(op, nrhs: int = 1, precision: int = AIM_MIXED, cache_path: str | None = DEFAULT_CACHE, reps: int = 10,
         seed: int = 0) -> dict:
    """Choose, apply and cache the fastest admissible launch configuration.
    Returns {"key", "tuning", "us", "cached", "tried", "rejected"}, and on a search also
    "start_us" (the configuration the op had) and "best5"."""
    import torch
    key = shape_key(op, nrhs, precision)
    cache = _load(cache_path) if cache_path else {}
    if key in cache:
        try:
            _apply(op, cache[key]["tuning"], precision)
            return {"key": key, "tuning": cache[key]["tuning"], "us": cache[key]["us"], "cached": True,
                    "tried": 0, "rejected": 0}
        except (AimError, KeyError, TypeError):
            pass  # an entry this library refuses (or an older format): search again and replace it
    rng = np.random.default_rng(seed)
    xh = rng.standard_normal((nrhs, op.n)) + 1j * rng.standard_normal((nrhs, op.n))
    x64 = torch.from_numpy(xh).to("cuda")
    ref = op.matvec(x64, precision=AIM_FP64).cpu().numpy()
    scale = np.abs(ref).max()
    tol = 1e-12 if precision == AIM_FP64 else 1e-5
    x = x64 if precision == AIM_FP64 else x64.to(torch.complex64)
    y = torch.empty_like(x)
    start = op.tuning()

    def timed():
        op.matvec(x, precision=precision, out=y)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            op.matvec(x, precision=precision, out=y)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e3

    start_us = timed()
    best, results, rejected = None, [], 0

    def trial(cand):
        nonlocal best, rejected
        try:
            _apply(op, cand, precision)
        except AimError:
            return
        op.matvec(x, precision=precision, out=y)
        err = float(np.abs(y.cpu().numpy() - ref).max() / scale)
        if not err <= tol:
            rejected += 1
            return
        us = timed()
        results.append((us, cand, err))
        if best is None or us < best[0]:
            best = (us, cand, err)

    for cand in _candidates(op, precision):
        trial(cand)
    if best is not None:  # the fork point, on the best configuration of the kernels
        base = best[1]
        for nf in (1, 2):
            trial(dict(base, near_fork=nf))
    if best is None:
        op.set_tuning(fft_b=start["fft_b"], interp_tile=start["interp_tile"], gemm_bf16=start["gemm_bf16"],
                      fft_register=start["fft_register"], near_block=start["near_block"],
                      near_fork=start["near_fork"])
        raise RuntimeError("no candidate launch configuration passed the accuracy check")
    _apply(op, best[1], precision)
    if cache_path:
        cache = _load(cache_path)
        cache[key] = {"tuning": best[1], "us": best[0], "err": best[2], "tried": len(results) + rejected,
                      "when": time.strftime("%Y-%m-%dT%H:%M:%S")}
        os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return {"key": key, "tuning": best[1], "us": best[0], "start_us": start_us, "cached": False,
            "tried": len(results) + rejected, "rejected": rejected,
            "best5": [(round(u, 2), c) for u, c, _ in sorted(results, key=lambda r: r[0])[:5]]}
