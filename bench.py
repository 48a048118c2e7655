#!/usr/bin/env python3
"""Benchmark of the solve-time path on one MI355X.

Workload: 32 x 32 array of Jerusalem-cross elements in 0.55-wavelength equivalent
boxes (6 x 6 squares per face, 648 RWG per box, 663,552 unknowns), AIM grid
h = 0.1 wavelength, order 2 (195 x 195 x 9 nodes, FFT lengths 400 x 400), one
plane wave at theta = 30 deg, phi = 45 deg.  Seeded synthetic data (see synth/).

One step = one GMRES(50) solve to 1e-6 relative residual in mixed precision
(complex FP32 products and basis, FP64 Gram-Schmidt sums, Hessenberg, Givens and
a FP64 residual product at every restart).  `value` = AIM matrix-vector products
per second over the timed solves (every product counts, FP64 restart products
included).  The FP64 solve, the same solves right-preconditioned with the per-kind
block-Jacobi inverses ("block_jacobi"), the standalone products, per-kernel times
and the oracle's CPU rate are reported beside it.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
COPY_BYTES = 536870912  # the plain device copy that calibrates the byte counters
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_jc32x32_fp32_product.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1712_02443_amd", "csrc", "aim_kernels.hip")
# device kernel name prefixes (FP32 product) -> per-kernel keys of this benchmark
KERNEL_KEYS = [("k_gemm_bf16x3", "macro_gemm"), ("k_gemm_f32", "macro_gemm"), ("k_project<float>", "project"), ("k_fft4_y_fwd<float", "fft_y_fwd"),
               ("k_fft_y_fwd<float>", "fft_y_fwd"), ("k_fft4_x<float", "fft_x_conv"), ("k_fft_x<float, 0>", "fft_x_conv"),
               ("k_fft4_y_inv<float", "fft_y_inv"), ("k_fft_y_inv<float>", "fft_y_inv"),
               ("k_near_mfma<float>", "near_field"), ("k_near<float>", "near_field"), ("k_interp<float, 0", "interp_d")]
FP32_MFMA_PEAK_TFLOPS = 157.3
BF16_MFMA_PEAK_TFLOPS = 2500.0  # dense
AIM_PATH_GEMM_BF16X3 = 4
# split-BF16 macromodel product: three real products per complex step (6 flop per
# complex multiply-add against the algorithmic 8), each as six bf16 products
BF16X3_EXECUTED_PER_ALGORITHMIC = 3 * 6 * 2 / 8
# FP32 vector FMA without packed (two-wide) instructions, which this build disables:
# 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
FP32_VALU_PEAK_TFLOPS = 78.6
FP64_VALU_PEAK_TFLOPS = 78.6
METRIC = "AIM matvecs/s and solve time to 1e-6 residual, mixed vs FP64; p50/p99 latency"


def kernel_model(info: dict, R: int, bytes_per: int) -> dict:
    """Algorithmic HBM bytes (flops for the two arithmetic-bound kernels) per launch."""
    nx, ny, nz, lx, ly = info["nx"], info["ny"], info["nz"], info["lx"], info["ly"]
    n = info["n_rwg"] * info["n_elem"]
    grid = 4 * R * nx * ny * nz * bytes_per
    spec = 4 * R * nx * ly * nz * bytes_per
    gt = (lx // 2 + 1) * (ly // 2 + 1) * nz * bytes_per
    vec = n * R * bytes_per
    return {
        "macro_gemm": {"flops": 8.0 * info["n_rwg"] ** 2 * info["n_elem"] * R, "bytes": 2 * vec},
        "project": {"bytes": vec + grid},
        "fft_y_fwd": {"bytes": grid + spec},
        "fft_x_conv": {"bytes": 2 * spec + gt},
        "fft_y_inv": {"bytes": spec + grid},
        "near_field": {"flops": 8.0 * info["near_nnz"] * info["n_elem"] * R, "bytes": 2 * vec},
        "interp_d": {"bytes": grid + 3 * vec},
    }


def source_sha256() -> str:
    import hashlib
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def summarize_counters(fetch_csv: str, write_csv: str, out_md: str, command: str) -> None:
    """Per-launch HBM bytes of the FP32 product kernels from two rocprofv3 --pmc runs
    (FETCH_SIZE, WRITE_SIZE; KiB per dispatch), scaled by what the same counters read
    for the plain 536,870,912-byte device copy of --profile-products."""
    import csv

    def load(path, counter):
        per, copy = {}, []
        for row in csv.DictReader(open(path)):
            if row["Counter_Name"] != counter:
                continue
            name = row["Kernel_Name"].replace("void ", "").replace("aimm::", "")
            val = float(row["Counter_Value"]) * 1024.0
            if "copyBuffer" in name:
                copy.append(val)
                continue
            for prefix, key in KERNEL_KEYS:
                if name.startswith(prefix):
                    per.setdefault(key, []).append(val)
        return per, max(copy)

    fetch, copy_f = load(fetch_csv, "FETCH_SIZE")
    write, copy_w = load(write_csv, "WRITE_SIZE")
    kf, kw = COPY_BYTES / copy_f, COPY_BYTES / copy_w
    lines = ["# HBM traffic per launch, FP32 product kernels, 32x32 Jerusalem-cross array", "",
             "Commands (from the repository root, libaimm.so built):", "", "```", command, "```", "",
             f"Calibration: the {COPY_BYTES}-byte device copy read FETCH_SIZE {copy_f:.0f} B and WRITE_SIZE "
             f"{copy_w:.0f} B, so fetch counts are scaled by {kf:.4f} and write counts by {kw:.4f}.", "",
             "| kernel | launches | fetch bytes | write bytes | total bytes |", "|---|---|---|---|---|"]
    for _, key in KERNEL_KEYS:
        if key in fetch and key in write and f"| {key} |" not in "\n".join(lines):
            f = sum(fetch[key]) / len(fetch[key]) * kf
            w = sum(write[key]) / len(write[key]) * kw
            lines.append(f"| {key} | {len(fetch[key])} | {f:.0f} | {w:.0f} | {f + w:.0f} |")
    lines += ["", f"source-sha256 aim_kernels.hip: {source_sha256()}", ""]
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines))


def measured_traffic(kernel: str):
    """Bytes per launch of `kernel` from the committed counter summary, or None when
    the summary is missing or was taken from another version of the kernel source."""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    if f"source-sha256 aim_kernels.hip: {source_sha256()}" not in text:
        return None
    for line in text.splitlines():
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) == 5 and cells[0] == kernel:
            return float(cells[4])
    return None


def cpu_baseline(wl, budget_s: float = 20.0) -> dict:
    """The CPU oracle's full product on the same workload, single thread."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle.system import OracleOperator
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        op = OracleOperator(wl)
        setup = time.perf_counter() - t0
        x = wl.test_vectors(1)[0]
        times = []
        t_start = time.perf_counter()
        while True:
            t = time.perf_counter()
            op.matvec(x)
            times.append(time.perf_counter() - t)
            if time.perf_counter() - t_start > budget_s * 0.5 or len(times) >= 5:
                break
    per = float(np.median(times))
    return {"value": 1.0 / per, "unit": "matvecs/s", "cores": 1, "kind": "oracle",
            "sample": f"{len(times)} full FP64 products of the same 663,552-unknown workload "
                      f"(median {per:.2f} s each; {setup:.1f} s untimed setup), numpy/scipy, 1 thread"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--restart", type=int, default=50)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison solves")
    ap.add_argument("--no-precond", action="store_true", help="skip the block-Jacobi preconditioned solves")
    ap.add_argument("--no-standard-mom", action="store_true",
                    help="skip the standard AIM-MoM solves on the original Jerusalem-cross surfaces")
    ap.add_argument("--no-multi-rhs", action="store_true",
                    help="skip the multi-RHS solves (16x16 plates with 64 RHS, 64x64 crosses with 8 RHS)")
    ap.add_argument("--profile-products", type=int, default=0,
                    help="only run this many FP32 and FP64 products and a 512 MiB device copy "
                         "(the copy calibrates hardware byte counters), then exit")
    ap.add_argument("--summarize-counters", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "OUT_MD"),
                    help="write the per-launch HBM traffic summary from two rocprofv3 --pmc runs and exit")
    ap.add_argument("--counter-command", default="", help="command line recorded in the summary")
    args = ap.parse_args()
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters, command=args.counter_command)
        return 0
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the path would shard over "
              "right-hand sides, or over x-slabs of the grid with all-to-all exchanges around the x FFT pass)",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1712_02443_amd import AIM_FP64, AIM_G_ONLY, AIM_MIXED, AIM_PRECOND_BLOCK_JACOBI, AimOperator
    from synth import make_workload, standard_mom_workload

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 1
    wl = make_workload(1)
    print(f"[bench] building {wl.name}: {wl.n_unknowns} unknowns", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    op = AimOperator.from_workload(wl)
    op.set_macromodels(wl.macromodels())
    op.set_dmatrix(*wl.d_matrix())
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    info = op.info()
    if args.profile_products:
        x64 = torch.from_numpy(wl.test_vectors(1)).to("cuda")
        x32 = x64.to(torch.complex64)
        for xv, prec in ((x32, AIM_MIXED), (x64, AIM_FP64)):
            y = torch.empty_like(xv)
            for _ in range(args.profile_products):
                op.matvec(xv, precision=prec, out=y)
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device="cuda")  # 512 MiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] profiled {args.profile_products} products per precision and a 536870912-byte copy",
              file=sys.stderr, flush=True)
        return 0
    b = op.plane_wave_rhs(wl.theta, wl.phi, wl.pol)
    # convergence flags are read by the host every 5 iterations (the result does not
    # depend on it: each right-hand side stops at its own first converged column)
    solve_kw = dict(restart=args.restart, tol=args.tol, max_iters=5000, check_every=5)

    last_x = {}

    def solve(prec):
        x, st, code = op.gmres(b, precision=prec, **solve_kw)
        last_x[prec] = x
        return st[0], code

    for _ in range(args.warmup):
        solve(AIM_MIXED)
    print("[bench] warm-up done", file=sys.stderr, flush=True)

    # timed region: exactly `steps` mixed-precision solves
    lat = []
    matvecs = 0
    stats = None
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        t = time.perf_counter()
        stats, code = solve(AIM_MIXED)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t)
        matvecs += stats["matvecs"]
        if code != 0:
            print(f"[bench] mixed solve did not converge: {stats}", file=sys.stderr)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    value = matvecs / elapsed
    print(f"[bench] mixed: {elapsed / args.steps * 1e3:.2f} ms/solve, {stats}", file=sys.stderr, flush=True)

    out = {}
    if not args.no_fp64:
        solve(AIM_FP64)
        torch.cuda.synchronize()
        t = time.perf_counter()
        mv64 = 0
        for _ in range(args.steps):
            st64, _ = solve(AIM_FP64)
            mv64 += st64["matvecs"]
        torch.cuda.synchronize()
        e64 = time.perf_counter() - t
        out["fp64_solve_ms"] = e64 / args.steps * 1e3
        out["fp64_matvecs_per_s"] = mv64 / e64
        out["fp64_iters"] = st64["iters"]
        out["fp64_true_relres"] = st64["true_relres"]
        out["mixed_vs_fp64_solve_speedup"] = (e64 / args.steps) / (elapsed / args.steps)
        print(f"[bench] fp64: {out['fp64_solve_ms']:.2f} ms/solve, {st64}", file=sys.stderr, flush=True)

    if not args.no_precond:
        # the same solves right-preconditioned with the per-kind block-Jacobi inverses
        t = time.perf_counter()
        op.build_preconditioner()
        torch.cuda.synchronize()
        bj = {"setup_s": time.perf_counter() - t}
        pkw = dict(solve_kw, precond=AIM_PRECOND_BLOCK_JACOBI)

        def psolve(prec):
            x, st, code = op.gmres(b, precision=prec, **pkw)
            return st[0], code

        for prec, tag in ((AIM_MIXED, "mixed"), (AIM_FP64, "fp64")):
            if prec == AIM_FP64 and args.no_fp64:
                continue
            psolve(prec)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(args.steps):
                stp, cp = psolve(prec)
            torch.cuda.synchronize()
            ep = time.perf_counter() - t
            bj[f"{tag}_solve_ms"] = ep / args.steps * 1e3
            bj[f"{tag}_iters"] = stp["iters"]
            bj[f"{tag}_matvecs_per_solve"] = stp["matvecs"]
            bj[f"{tag}_true_relres"] = stp["true_relres"]
            bj[f"{tag}_converged"] = bool(stp["converged"])
        bj["mixed_speedup_vs_unpreconditioned_mixed"] = (elapsed / args.steps * 1e3) / bj["mixed_solve_ms"]
        if "fp64_solve_ms" in bj:
            bj["mixed_vs_fp64_solve_speedup"] = bj["fp64_solve_ms"] / bj["mixed_solve_ms"]
        out["block_jacobi"] = bj
        print(f"[bench] block-Jacobi: {bj}", file=sys.stderr, flush=True)

    # far field of the mixed solution along two principal cuts (0.5 degree steps)
    th = np.linspace(0.0, math.pi, 361)
    rh = np.concatenate([np.stack([np.sin(th), np.zeros_like(th), np.cos(th)], 1),
                         np.stack([np.zeros_like(th), np.sin(th), np.cos(th)], 1)])
    xs = last_x[AIM_MIXED]
    op.far_field(xs, rh)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        op.far_field(xs, rh)
    torch.cuda.synchronize()
    ff_s = (time.perf_counter() - t) / args.steps
    out["far_field"] = {"directions": int(rh.shape[0]), "ms": ff_s * 1e3,
                        "element_sum_gflop": 8.0 * rh.shape[0] * info["n_rwg"] * info["n_elem"] / 1e9}
    print(f"[bench] far field: {out['far_field']}", file=sys.stderr, flush=True)

    if not args.no_standard_mom:
        # the same array solved as a standard AIM-MoM on each element's own PEC surface
        # (1,196 RWG per cross instead of the 648 of its equivalent box): G J = V
        ws = standard_mom_workload()
        t = time.perf_counter()
        ops = AimOperator.from_workload(ws)
        torch.cuda.synchronize()
        sm = {"workload": f"{ws.name}: 32x32 PEC Jerusalem crosses, {ws.n_rwg} RWG each", "unknowns": ws.n_unknowns,
              "macromodel_unknowns": wl.n_unknowns, "build_s": time.perf_counter() - t}
        bs = ops.plane_wave_rhs(ws.theta, ws.phi, ws.pol)
        skw = dict(restart=args.restart, tol=args.tol, max_iters=5000, check_every=5, precision=AIM_MIXED,
                   system=AIM_G_ONLY)
        ops.gmres(bs, **skw)
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, sts, cs = ops.gmres(bs, **skw)
        torch.cuda.synchronize()
        sm.update({"mixed_solve_ms": (time.perf_counter() - t) * 1e3, "iters": sts[0]["iters"],
                   "converged": bool(sts[0]["converged"]), "true_relres": sts[0]["true_relres"]})
        # block-Jacobi on the crosses: blocks G_self^-1 (built with M = -I, empty D)
        t = time.perf_counter()
        ops.set_macromodels(-np.eye(ws.n_rwg, dtype=np.complex128)[None])
        ops.set_dmatrix(np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.complex128))
        ops.build_preconditioner()
        torch.cuda.synchronize()
        sm["block_jacobi_setup_s"] = time.perf_counter() - t
        skw["precond"] = AIM_PRECOND_BLOCK_JACOBI
        ops.gmres(bs, **skw)
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, sts, cs = ops.gmres(bs, **skw)
        torch.cuda.synchronize()
        sm.update({"block_jacobi_mixed_solve_ms": (time.perf_counter() - t) * 1e3,
                   "block_jacobi_iters": sts[0]["iters"], "block_jacobi_converged": bool(sts[0]["converged"])})
        ops.close()
        del ops
        out["standard_mom"] = sm
        print(f"[bench] standard MoM: {sm}", file=sys.stderr, flush=True)

    if not args.no_multi_rhs:
        # many incidences as one block: every right-hand side in every launch
        mr = {}
        for idx in (2, 4):
            wm = make_workload(idx)
            opm = AimOperator.from_workload(wm)
            opm.set_macromodels(wm.macromodels())
            opm.set_dmatrix(*wm.d_matrix())
            bm = opm.plane_wave_rhs(wm.theta, wm.phi, wm.pol)
            ent = {"unknowns_per_rhs": wm.n_unknowns, "nrhs": wm.nrhs, "restart": wm.restart}
            for prec, tag in ((AIM_MIXED, "mixed"), (AIM_FP64, "fp64")):
                mkw = dict(restart=wm.restart, tol=args.tol, max_iters=5000, check_every=5, precision=prec)
                opm.gmres(bm, **mkw)
                torch.cuda.synchronize()
                t = time.perf_counter()
                _, stm, cm = opm.gmres(bm, **mkw)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t
                ent[f"{tag}_solve_ms"] = dt * 1e3
                ent[f"{tag}_rhs_matvecs_per_s"] = sum(q["matvecs"] for q in stm) / dt
                ent[f"{tag}_max_iters"] = max(q["iters"] for q in stm)
                ent[f"{tag}_all_converged"] = cm == 0
            ent["mixed_vs_fp64_solve_speedup"] = ent["fp64_solve_ms"] / ent["mixed_solve_ms"]
            mr[wm.name] = ent
            opm.close()
            del opm
            torch.cuda.empty_cache()
        out["multi_rhs"] = mr
        print(f"[bench] multi-RHS: {mr}", file=sys.stderr, flush=True)

    # standalone products
    x64 = torch.from_numpy(wl.test_vectors(1)).to("cuda")
    x32 = x64.to(torch.complex64)
    for name, xv, prec in (("product_fp32_us", x32, AIM_MIXED), ("product_fp64_us", x64, AIM_FP64)):
        y = torch.empty_like(xv)
        for _ in range(3):
            op.matvec(xv, precision=prec, out=y)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.kernel_reps):
            op.matvec(xv, precision=prec, out=y)
        e1.record()
        torch.cuda.synchronize()
        out[name] = e0.elapsed_time(e1) / args.kernel_reps * 1e3

    # per-kernel times of the mixed product, roofline of the dominant kernel
    kt = op.time_kernels(x32, precision=AIM_MIXED, reps=args.kernel_reps)
    kt64 = op.time_kernels(x64, precision=AIM_FP64, reps=args.kernel_reps)
    model = kernel_model(info, 1, 8)
    dom = max(kt, key=kt.get)
    traffic = measured_traffic(dom)
    if "flops" in model[dom]:
        # the near field runs on the FP32 matrix cores; the mixed macromodel product on the
        # FP32 matrix cores or, by default, as split-BF16 with FP32 accumulation, which takes
        # FP32 operands to an FP32-accurate result and is priced at the FP32 peak: its
        # executed bf16 rate against the bf16 dense peak is reported beside it
        ach = model[dom]["flops"] / (kt[dom] * 1e-3) / 1e12
        roof = {"kernel": dom, "bound": "mfma", "achieved": ach, "peak": FP32_MFMA_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": ach / FP32_MFMA_PEAK_TFLOPS, "traffic": traffic,
                "algorithmic_bytes": model[dom]["bytes"]}
        if dom == "macro_gemm" and info["paths"] & AIM_PATH_GEMM_BF16X3:
            ex = ach * BF16X3_EXECUTED_PER_ALGORITHMIC
            roof.update({"mfma_dtype": "bf16, three-term split of FP32 operands, FP32 accumulation",
                         "executed_bf16_tflops": ex, "executed_bf16_frac": ex / BF16_MFMA_PEAK_TFLOPS})
    else:
        ach = model[dom]["bytes"] / (kt[dom] * 1e-3) / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBS, "traffic": traffic}
    per_kernel = {}
    for k, ms in kt.items():
        m = model[k]
        ent = {"us": ms * 1e3}
        if "flops" in m:
            ent["tflops"] = m["flops"] / (ms * 1e-3) / 1e12
        else:
            ent["gbs"] = m["bytes"] / (ms * 1e-3) / 1e9
        per_kernel[k] = ent
    out["kernels_fp32"] = per_kernel
    out["kernels_fp64_us"] = {k: v * 1e3 for k, v in kt64.items()}

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "matvecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 products + f64 Krylov sums",
        "data": "synthetic (seeded meshes, macromodel blocks and D; plane-wave excitation)",
        "config": {"workload": "jc-32x32-mixed: 32x32 array, 648 RWG/box, 663552 unknowns, grid 195x195x9, "
                               "FFT 400x400, 1 RHS, GMRES(50) to 1e-6",
                   "unknowns": wl.n_unknowns, "nrhs": 1, "restart": args.restart, "tol": args.tol},
        "solve_ms_p50": float(np.percentile(lat, 50) * 1e3),
        "solve_ms_p99": float(np.percentile(lat, 99) * 1e3),
        "iters": stats["iters"], "restarts": stats["restarts"], "matvecs_per_solve": stats["matvecs"],
        "true_relres": stats["true_relres"],
        "build_s": build_s,
        "roofline": roof,
    }
    line.update(out)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(wl)
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
