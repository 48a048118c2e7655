"""MI355X-native solve-time path of the macromodel + AIM method (arXiv:1712.02443).

`AimOperator` wraps one array problem held by libaimm.so: the AIM-accelerated
final-system product (D - G T A^-1 B) x (section V, eq. MV_product1), its parts,
the plane-wave excitation (eq. V1) and the restarted GMRES solve of
eq. finalsystem.  Tensors must live on the GPU; complex128 for AIM_FP64 and
complex64 for AIM_MIXED products, complex128 for solves.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import (AIM_FAR_ONLY, AIM_FP64, AIM_FULL, AIM_G_ONLY, AIM_MIXED, AIM_PRECOND_BLOCK_JACOBI,
                   AIM_PRECOND_NONE, AimError, GmresOpts, GmresStat, check, load)

__all__ = ["AimOperator", "AIM_FP64", "AIM_MIXED", "AIM_FULL", "AIM_G_ONLY", "AIM_FAR_ONLY",
           "AIM_PRECOND_NONE", "AIM_PRECOND_BLOCK_JACOBI", "AimError", "footprint_bytes", "load"]


def _stream(torch, stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def footprint_bytes(vert, tri, rwg, *, k, eta, h, r_near, order, px, py, pitch_cells, elem_type, n_types,
                    max_rhs, nrhs, restart, precision) -> int:
    st = _lib.Structs(vert, tri, rwg, k, eta, h, r_near, order, px, py, pitch_cells, elem_type, n_types, max_rhs)
    return int(load().aim_footprint_bytes(ctypes.byref(st.surface), ctypes.byref(st.array), nrhs, restart,
                                          precision))


class AimOperator:
    """One array problem on the current GPU (see include/aimm.h for the conventions)."""

    def __init__(self, vert, tri, rwg, *, k, eta, h, r_near, order, px, py, pitch_cells, elem_type, n_types,
                 max_rhs=1, host_only=False, stream=None):
        self.lib = load()
        self._op = None
        self._st = _lib.Structs(vert, tri, rwg, k, eta, h, r_near, order, px, py, pitch_cells, elem_type,
                                n_types, max_rhs)
        if not host_only:
            import torch
            self._torch = torch
        h_op = ctypes.c_void_p()
        if host_only:
            check(self.lib.aim_build_host(ctypes.byref(self._st.surface), ctypes.byref(self._st.array),
                                          ctypes.byref(h_op)))
        else:
            check(self.lib.aim_build_grid(ctypes.byref(self._st.surface), ctypes.byref(self._st.array),
                                          _stream(self._torch, stream), ctypes.byref(h_op)))
        self._op = h_op
        self.max_rhs = int(max_rhs)
        inf = self.info()
        self.n_rwg, self.n_elem = inf["n_rwg"], inf["n_elem"]
        self.n = self.n_rwg * self.n_elem
        self.grid = (inf["nx"], inf["ny"], inf["nz"])

    @classmethod
    def from_workload(cls, wl, max_rhs=None, host_only=False):
        m = wl.surface
        return cls(m.vert, m.tri, m.rwg, k=wl.k, eta=wl.eta, h=wl.h, r_near=wl.r_near, order=wl.order,
                   px=wl.px, py=wl.py, pitch_cells=wl.pitch_cells, elem_type=wl.elem_type, n_types=wl.n_types,
                   max_rhs=wl.nrhs if max_rhs is None else max_rhs, host_only=host_only)

    def close(self):
        if getattr(self, "_op", None):
            self.lib.aim_destroy(self._op)
            self._op = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- data ---------------------------------------------------------------------
    def set_macromodels(self, M: np.ndarray):
        """M: (n_types, N, N) complex; stored column-major as the library expects."""
        Mc = np.ascontiguousarray(np.transpose(np.asarray(M, dtype=np.complex128), (0, 2, 1)))
        check(self.lib.aim_set_macromodels(self._op, Mc.view(np.float64).ctypes.data_as(_lib._f64p)))
        self._M = Mc

    def set_dmatrix(self, rows, cols, vals):
        r = np.ascontiguousarray(rows, dtype=np.int32)
        c = np.ascontiguousarray(cols, dtype=np.int32)
        v = np.ascontiguousarray(vals, dtype=np.complex128)
        check(self.lib.aim_set_dmatrix(self._op, r.shape[0], r.ctypes.data_as(_lib._i32p),
                                       c.ctypes.data_as(_lib._i32p), v.view(np.float64).ctypes.data_as(_lib._f64p)))

    def tuning(self) -> dict:
        t = _lib.AimTuning()
        check(self.lib.aim_get_tuning(self._op, ctypes.byref(t)))
        return {"fft_b": [int(t.fft_b[0]), int(t.fft_b[1])], "interp_tile": [int(t.interp_tx), int(t.interp_ty)],
                "gemm_bf16": int(t.gemm_bf16), "fft_register": int(t.fft_register),
                "near_block": [int(t.near_block[0]), int(t.near_block[1])],
                "near_fork": [int(t.near_fork[0]), int(t.near_fork[1])]}

    def set_tuning(self, fft_b=(0, 0), interp_tile=(0, 0), gemm_bf16=-1, fft_register=-1, near_block=(0, 0),
                   near_fork=(-1, -1)):
        t = _lib.AimTuning((ctypes.c_int32 * 2)(*fft_b), int(interp_tile[0]), int(interp_tile[1]), int(gemm_bf16),
                           int(fft_register), (ctypes.c_int32 * 2)(*near_block), (ctypes.c_int32 * 2)(*near_fork))
        check(self.lib.aim_set_tuning(self._op, ctypes.byref(t)))

    def set_elem_type(self, elem_type, stream=None):
        """Re-assign the element kinds of this op (same lattice), keeping everything else."""
        et = np.ascontiguousarray(elem_type, dtype=np.int32)
        if et.shape[0] != self.n_elem:
            raise ValueError("one kind per element is needed")
        check(self.lib.aim_set_elem_type(self._op, et.ctypes.data_as(_lib._i32p), _stream(self._torch, stream)))
        self._st.elem_type[:] = et

    def macromodel_data(self):
        """(M blocks (n_types, N, N), D rows, cols, values) as generated by build_macromodels,
        for reuse on other ops of the same surface (set_macromodels / set_dmatrix)."""
        nt = self.info()["n_types"]
        Ms, D = [], None
        for t in range(nt):
            M, _, D = self.macromodel(t)
            Ms.append(M)
        r, c = np.nonzero(D)
        return np.stack(Ms), r.astype(np.int32), c.astype(np.int32), D[r, c].astype(np.complex128)

    def build_macromodels(self, meshes, stream=None):
        """Generate every kind's M_t, R_t = A_t^-1 B_t and D on the device from the PEC
        scatterer meshes (one per kind: objects with vert, tri, rwg), and set M and D."""
        if len(meshes) != self.info()["n_types"]:
            raise ValueError("one scatterer mesh per element kind is needed")
        keep = []
        surfs = (_lib.AimSurface * len(meshes))()
        for i, m in enumerate(meshes):
            v = np.ascontiguousarray(m.vert, dtype=np.float64)
            t = np.ascontiguousarray(m.tri, dtype=np.int32)
            r = np.ascontiguousarray(m.rwg, dtype=np.int32)
            keep += [v, t, r]
            surfs[i] = _lib.AimSurface(v.shape[0], t.shape[0], r.shape[0], v.ctypes.data_as(_lib._f64p),
                                       t.ctypes.data_as(_lib._i32p), r.ctypes.data_as(_lib._i32p))
        check(self.lib.aim_build_macromodels(self._op, surfs, _stream(self._torch, stream)))
        self._n_scat = [int(self.lib.aim_scatterer_unknowns(self._op, t)) for t in range(len(meshes))]

    def macromodel(self, kind: int):
        """Generated blocks of one kind: M (N, N), R (N_t, N) complex128 and D (N, N) real."""
        N = self.n_rwg
        Nt = self._n_scat[kind]
        M = np.empty((N, N), np.complex128)
        R = np.empty((N, Nt), np.complex128)
        D = np.empty((N, N), np.float64)
        check(self.lib.aim_get_macromodel(self._op, int(kind), M.view(np.float64).ctypes.data_as(_lib._f64p),
                                          R.view(np.float64).ctypes.data_as(_lib._f64p),
                                          D.ctypes.data_as(_lib._f64p)))
        # column-major storage read back as row-major is the transpose
        return M.T.copy(), R.T.copy(), D.T.copy()

    def recover_currents(self, x, stream=None):
        """J = -R_t E^ on every element's scatterer (device complex128 (nrhs, total scatterer unknowns))."""
        R = self._check_vec(x, AIM_FP64)
        ntot = int(self.lib.aim_scatterer_unknowns(self._op, -1))
        J = self._torch.empty((R, ntot), dtype=self._torch.complex128, device=x.device)
        check(self.lib.aim_recover_currents(self._op, _dev_ptr(x), _dev_ptr(J), R, _stream(self._torch, stream)))
        return J

    def build_preconditioner(self):
        """Per-kind block-Jacobi blocks P_t = (D - G_self M_t)^-1 (host FP64, then the device)."""
        check(self.lib.aim_build_preconditioner(self._op))

    def preconditioner(self) -> np.ndarray:
        """The blocks P_t as (n_types, N, N) complex128."""
        inf = self.info()
        nt, N = inf["n_types"], inf["n_rwg"]
        P = np.empty((nt, N, N), np.complex128)  # column-major per block: [t][col][row]
        check(self.lib.aim_get_preconditioner(self._op, P.view(np.float64).ctypes.data_as(_lib._f64p)))
        return np.ascontiguousarray(np.transpose(P, (0, 2, 1)))

    def precond_apply(self, x, precision=AIM_FP64, out=None, stream=None):
        R = self._check_vec(x, precision)
        y = self._torch.empty_like(x) if out is None else out
        check(self.lib.precond_apply(self._op, _dev_ptr(x), _dev_ptr(y), R, precision, _stream(self._torch, stream)))
        return y

    def info(self) -> dict:
        inf = _lib.AimInfo()
        check(self.lib.aim_get_info(self._op, ctypes.byref(inf)))
        return {name: getattr(inf, name) for name, _ in inf._fields_}

    def near(self):
        """Pre-corrected near field: rows, offset index, cols, values, offsets (dx, dy)."""
        inf = self.info()
        nnz = inf["near_nnz"]
        rows = np.empty(nnz, np.int32)
        offs = np.empty(nnz, np.int32)
        cols = np.empty(nnz, np.int32)
        vals = np.empty(nnz, np.complex128)
        offsets = np.empty(2 * max(inf["n_offsets"], 1), np.int32)
        check(self.lib.aim_get_near(self._op, rows.ctypes.data_as(_lib._i32p), offs.ctypes.data_as(_lib._i32p),
                                    cols.ctypes.data_as(_lib._i32p), vals.view(np.float64).ctypes.data_as(_lib._f64p),
                                    offsets.ctypes.data_as(_lib._i32p)))
        return rows, offs, cols, vals, offsets[:2 * inf["n_offsets"]].reshape(-1, 2)

    # ---- device work ------------------------------------------------------------------
    def _check_vec(self, x, prec):
        torch = self._torch
        want = torch.complex128 if prec == AIM_FP64 else torch.complex64
        if x.dtype != want or not x.is_cuda or not x.is_contiguous():
            raise ValueError(f"expected a contiguous {want} CUDA tensor")
        if x.numel() % self.n:
            raise ValueError("tensor size is not a multiple of the unknown count")
        return x.numel() // self.n

    def matvec(self, x, precision=AIM_FP64, flags=AIM_FULL, out=None, stream=None):
        R = self._check_vec(x, precision)
        y = self._torch.empty_like(x) if out is None else out
        check(self.lib.aim_matvec(self._op, _dev_ptr(x), _dev_ptr(y), R, precision, flags, _stream(self._torch, stream)))
        return y

    KERNELS = ("macro_gemm", "project", "fft_y_fwd", "fft_x_conv", "fft_y_inv", "near_field", "interp_d")

    def time_kernels(self, x, precision=AIM_FP64, reps=20, stream=None, out=None) -> dict:
        """Mean per-kernel duration (ms) of the full product: each kernel launched reps
        times back to back between HIP events on the stream.  out (optional) receives
        the product."""
        R = self._check_vec(x, precision)
        y = self._torch.empty_like(x) if out is None else out
        ms = np.zeros(7)
        check(self.lib.aim_time_kernels(self._op, _dev_ptr(x), _dev_ptr(y), R, precision, int(reps),
                                        ms.ctypes.data_as(_lib._f64p), _stream(self._torch, stream)))
        return dict(zip(self.KERNELS, ms.tolist()))

    def macro_apply(self, x, precision=AIM_FP64, out=None, stream=None):
        R = self._check_vec(x, precision)
        u = self._torch.empty_like(x) if out is None else out
        check(self.lib.macro_apply(self._op, _dev_ptr(x), _dev_ptr(u), R, precision, _stream(self._torch, stream)))
        return u

    def project(self, u, precision=AIM_FP64, stream=None):
        R = self._check_vec(u, precision)
        nx, ny, nz = self.grid
        Q = self._torch.empty((R, 4, nx, ny, nz), dtype=u.dtype, device=u.device)
        check(self.lib.aim_project(self._op, _dev_ptr(u), _dev_ptr(Q), R, precision, _stream(self._torch, stream)))
        return Q

    def convolve(self, Q, precision=AIM_FP64, stream=None):
        R = Q.shape[0]
        Phi = self._torch.empty_like(Q)
        check(self.lib.aim_convolve(self._op, _dev_ptr(Q), _dev_ptr(Phi), R, precision, _stream(self._torch, stream)))
        return Phi

    def plane_wave_rhs(self, theta, phi, pol, stream=None):
        th = np.ascontiguousarray(theta, dtype=np.float64)
        ph = np.ascontiguousarray(phi, dtype=np.float64)
        po = np.ascontiguousarray(pol, dtype=np.int32)
        R = th.shape[0]
        b = self._torch.empty((R, self.n), dtype=self._torch.complex128, device="cuda")
        check(self.lib.aim_plane_wave_rhs(self._op, th.ctypes.data_as(_lib._f64p), ph.ctypes.data_as(_lib._f64p),
                                          po.ctypes.data_as(_lib._i32p), R, _dev_ptr(b), _stream(self._torch, stream)))
        return b

    def far_field(self, x, rhat, system=AIM_FULL, stream=None, out=None, noalloc=False):
        """Far-zone field (nrhs, ndir, 3) complex128 and RCS in dB (nrhs, ndir) of the
        solutions x (device complex128) along the unit directions rhat (ndir, 3); the
        currents are -M x (AIM_FULL) or x (AIM_G_ONLY).  out = (E, rcs) reuses output
        tensors; noalloc calls aim_far_field_noalloc (library scratch, no allocation)."""
        R = self._check_vec(x, AIM_FP64)
        rh = np.ascontiguousarray(rhat, dtype=np.float64).reshape(-1, 3)
        D = rh.shape[0]
        if out is None:
            E = self._torch.empty((R, D, 3), dtype=self._torch.complex128, device=x.device)
            rcs = self._torch.empty((R, D), dtype=self._torch.float64, device=x.device)
        else:
            E, rcs = out
            if tuple(E.shape) != (R, D, 3) or tuple(rcs.shape) != (R, D):
                raise ValueError("out tensors have the wrong shape")
        fn = self.lib.aim_far_field_noalloc if noalloc else self.lib.aim_far_field
        check(fn(self._op, _dev_ptr(x), R, D, rh.ctypes.data_as(_lib._f64p), _dev_ptr(E), _dev_ptr(rcs),
                 int(system), _stream(self._torch, stream)))
        return E, rcs

    def gmres(self, b, x=None, *, restart=50, tol=1e-6, max_iters=1000, precision=AIM_FP64, check_every=1,
              precond=0, system=AIM_FULL, graphs=False, stream=None):
        R = self._check_vec(b, AIM_FP64)
        x0_given = x is not None
        if x is None:
            x = self._torch.empty_like(b)
        opts = GmresOpts(int(restart), int(max_iters), int(precision), int(x0_given), int(check_every), int(precond),
                         int(system), int(bool(graphs)), float(tol))
        stats = (GmresStat * R)()
        code = check(self.lib.gmres_solve(self._op, _dev_ptr(b), _dev_ptr(x), R, ctypes.byref(opts), stats,
                                          _stream(self._torch, stream)))
        st = [{name: getattr(s, name) for name, _ in s._fields_} for s in stats]
        return x, st, code
