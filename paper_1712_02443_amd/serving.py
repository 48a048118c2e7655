"""Request loop for array solves: many arrays of different sizes and right-hand-side
counts arriving over time, served concurrently on one GPU.

The reuse the paper builds on (section III: the macromodel of a distinct element is
computed once and shared by every copy of it) extends across requests here:
  * the macromodel blocks M_t and D of the element kinds are generated once, on the
    device, and copied to every operator;
  * an operator (AIM grid, Green's-function spectrum, near field, block-Jacobi blocks,
    Krylov workspace) is built once per array size and kept; a request of that size
    only re-assigns the element kinds (aim_set_elem_type) and solves;
  * operators are admitted by their device footprint (aim_footprint_bytes) against a
    memory budget; an idle operator of another size is evicted when a new one does not
    fit, and a request waits when nothing can be evicted;
  * requests are taken in arrival order by a fixed number of workers, each with its own
    default-priority stream, so a request that arrives while others run starts as soon
    as a worker and the memory for its operator are free, and the solves overlap on the
    device.
Each request is solved with its own Krylov spaces (one per right-hand side), so a
result does not depend on which other requests ran beside it.

This module only schedules: every arithmetic step runs in the library's kernels.
"""
from __future__ import annotations

import collections
import queue
import threading
import time
from dataclasses import dataclass, field

import numpy as np

from . import AIM_MIXED, AIM_PRECOND_BLOCK_JACOBI, AimOperator, footprint_bytes


@dataclass
class Record:
    index: int
    side: int
    nrhs: int
    arrival_s: float
    start_s: float = 0.0
    end_s: float = 0.0
    iters: int = 0
    converged: bool = False
    built_op: bool = False
    x: object = None

    @property
    def latency_s(self) -> float:
        return self.end_s - self.arrival_s


@dataclass
class _Slot:
    op: AimOperator
    bytes: int
    busy: bool = False
    last_used: float = 0.0


class ArrayServer:
    """Serves plane-wave solves of square arrays of one equivalent surface with a few
    element kinds (see the module docstring)."""

    def __init__(self, box_mesh, kind_meshes, *, k, eta, h=0.1, r_near=0.3, order=2, pitch_cells=6,
                 max_rhs=16, workers=4, mem_budget_bytes=64 << 30, restart=50, tol=1e-6, precision=AIM_MIXED,
                 precond=True, max_iters=5000, keep_solutions=False):
        import torch
        self._torch = torch
        self.box = box_mesh
        self.n_types = len(kind_meshes)
        self.params = dict(k=k, eta=eta, h=h, r_near=r_near, order=order, pitch_cells=pitch_cells)
        self.max_rhs = int(max_rhs)
        self.workers = int(workers)
        self.budget = int(mem_budget_bytes)
        self.solve_kw = dict(restart=restart, tol=tol, max_iters=max_iters, check_every=5, precision=precision,
                             precond=AIM_PRECOND_BLOCK_JACOBI if precond else 0)
        self.precond = precond
        self.keep = keep_solutions
        # the kinds' macromodels, generated once on the device (on a one-element op)
        gen = AimOperator(box_mesh.vert, box_mesh.tri, box_mesh.rwg, px=1, py=1,
                          elem_type=np.zeros(1, np.int32), n_types=self.n_types, max_rhs=1, **self.params)
        t0 = time.perf_counter()
        gen.build_macromodels(kind_meshes)
        self.M, self.d_rows, self.d_cols, self.d_vals = gen.macromodel_data()
        gen.close()
        self.generation_s = time.perf_counter() - t0
        self._lock = threading.Condition()
        self._pool: dict[int, list[_Slot]] = collections.defaultdict(list)
        self._used = 0
        self.ops_built = 0
        self.ops_evicted = 0

    # ---- operators --------------------------------------------------------------
    def _footprint(self, side: int) -> int:
        return footprint_bytes(self.box.vert, self.box.tri, self.box.rwg, px=side, py=side,
                               elem_type=np.zeros(side * side, np.int32), n_types=self.n_types,
                               max_rhs=self.max_rhs, nrhs=self.max_rhs, restart=self.solve_kw["restart"],
                               precision=self.solve_kw["precision"], **self.params)

    def _build(self, side: int, stream) -> AimOperator:
        op = AimOperator(self.box.vert, self.box.tri, self.box.rwg, px=side, py=side,
                         elem_type=np.zeros(side * side, np.int32), n_types=self.n_types, max_rhs=self.max_rhs,
                         stream=stream, **self.params)
        op.set_macromodels(self.M)
        op.set_dmatrix(self.d_rows, self.d_cols, self.d_vals)
        if self.precond:
            op.build_preconditioner()
        return op

    def _acquire(self, side: int, stream):
        """An idle operator of this size, or a new one once its footprint fits the budget
        (evicting idle operators of other sizes, least recently used first)."""
        need = self._footprint(side)
        if need > self.budget:
            raise MemoryError(f"an operator for a {side} x {side} array needs {need} bytes, over the budget")
        with self._lock:
            while True:
                for slot in self._pool[side]:
                    if not slot.busy:
                        slot.busy = True
                        return slot, False
                if self._used + need <= self.budget:
                    self._used += need
                    break
                idle = [(s.last_used, sd, s) for sd, lst in self._pool.items() for s in lst if not s.busy]
                if idle:
                    _, sd, victim = min(idle, key=lambda t: t[0])
                    self._pool[sd].remove(victim)
                    self._used -= victim.bytes
                    victim.op.close()
                    self.ops_evicted += 1
                    continue
                self._lock.wait()
        try:
            op = self._build(side, stream)
        except Exception:
            with self._lock:
                self._used -= need
                self._lock.notify_all()
            raise
        slot = _Slot(op, need, busy=True)
        with self._lock:
            self._pool[side].append(slot)
            self.ops_built += 1
        return slot, True

    def _release(self, slot: _Slot):
        with self._lock:
            slot.busy = False
            slot.last_used = time.perf_counter()
            self._lock.notify_all()

    # ---- one request ------------------------------------------------------------
    def solve(self, req, stream=None):
        """Solve one request on an operator of its size; returns (x, stats, code, built)."""
        torch = self._torch
        slot, built = self._acquire(int(req.side), stream)
        try:
            op = slot.op
            op.set_elem_type(req.elem_type, stream=stream)
            with torch.cuda.stream(stream) if stream is not None else _null():
                b = op.plane_wave_rhs(req.theta, req.phi, req.pol, stream=stream)
                x, st, code = op.gmres(b, stream=stream, **self.solve_kw)
                if stream is not None:
                    stream.synchronize()
        finally:
            self._release(slot)
        return x, st, code, built

    # ---- the loop -----------------------------------------------------------------
    def run(self, trace, speed: float = 1.0) -> list[Record]:
        """Replay a trace: request i is released at its arrival time (divided by speed)
        and taken by the first free worker; returns one record per request."""
        torch = self._torch
        recs = [Record(i, int(r.side), int(len(r.theta)), float(r.arrival_s) / speed) for i, r in enumerate(trace)]
        work: queue.Queue = queue.Queue()
        errors = []
        t0 = time.perf_counter()

        def worker():
            stream = torch.cuda.Stream()  # default priority
            while True:
                item = work.get()
                if item is None:
                    return
                i, req = item
                rec = recs[i]
                rec.start_s = time.perf_counter() - t0
                try:
                    x, st, code, built = self.solve(req, stream)
                    rec.iters = max(s["iters"] for s in st)
                    rec.converged = code == 0
                    rec.built_op = built
                    if self.keep:
                        rec.x = x.cpu().numpy()
                except Exception as e:  # recorded; the loop goes on
                    errors.append((i, repr(e)))
                rec.end_s = time.perf_counter() - t0

        threads = [threading.Thread(target=worker, daemon=True) for _ in range(self.workers)]
        for th in threads:
            th.start()
        for i, req in enumerate(trace):
            wait = recs[i].arrival_s - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
            work.put((i, req))
        for _ in threads:
            work.put(None)
        for th in threads:
            th.join()
        self.errors = errors
        return recs

    def close(self):
        with self._lock:
            for lst in self._pool.values():
                for slot in lst:
                    slot.op.close()
            self._pool.clear()
            self._used = 0


class _null:
    def __enter__(self):
        return None

    def __exit__(self, *a):
        return False


def summarize(recs: list[Record]) -> dict:
    lat = np.array([r.latency_s for r in recs])
    span = max(r.end_s for r in recs) - min(r.arrival_s for r in recs)
    return {
        "requests": len(recs),
        "rhs": int(sum(r.nrhs for r in recs)),
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "mean_service_ms": float(np.mean([r.end_s - r.start_s for r in recs]) * 1e3),
        "requests_per_s": len(recs) / span,
        "rhs_solves_per_s": sum(r.nrhs for r in recs) / span,
        "all_converged": all(r.converged for r in recs),
        "max_iters": max(r.iters for r in recs),
        "span_s": span,
    }
