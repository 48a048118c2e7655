"""ctypes binding of libaimm.so: argument marshalling only.

Every step of the product and of the solve runs in the library's HIP kernels;
PyTorch supplies device memory (tensors) and the current HIP stream.  If the
library is missing or fails to load, every entry point raises: there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libaimm.so")

AIM_OK, AIM_ENOCONV, AIM_EINVAL, AIM_ENOMEM, AIM_EDEVICE, AIM_ESTATE = 0, 1, -1, -2, -3, -4
AIM_FP64, AIM_MIXED = 0, 1
AIM_FULL, AIM_G_ONLY, AIM_FAR_ONLY = 0, 1, 2
AIM_PRECOND_NONE, AIM_PRECOND_BLOCK_JACOBI = 0, 1

_i32p = ctypes.POINTER(ctypes.c_int32)
_f64p = ctypes.POINTER(ctypes.c_double)


class AimSurface(ctypes.Structure):
    _fields_ = [("n_vert", ctypes.c_int32), ("n_tri", ctypes.c_int32), ("n_rwg", ctypes.c_int32),
                ("vert", _f64p), ("tri", _i32p), ("rwg", _i32p)]


class AimArray(ctypes.Structure):
    _fields_ = [("k", ctypes.c_double), ("eta", ctypes.c_double), ("h", ctypes.c_double),
                ("r_near", ctypes.c_double), ("order", ctypes.c_int32), ("px", ctypes.c_int32),
                ("py", ctypes.c_int32), ("pitch_cells", ctypes.c_int32), ("n_types", ctypes.c_int32),
                ("elem_type", _i32p), ("max_rhs", ctypes.c_int32)]


class AimInfo(ctypes.Structure):
    _fields_ = [("n_rwg", ctypes.c_int32), ("n_elem", ctypes.c_int32), ("n_types", ctypes.c_int32),
                ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("lx", ctypes.c_int32), ("ly", ctypes.c_int32), ("n_offsets", ctypes.c_int32),
                ("near_nnz", ctypes.c_int64), ("d_nnz", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("paths", ctypes.c_int32)]


class AimTuning(ctypes.Structure):
    _fields_ = [("fft_b", ctypes.c_int32 * 2), ("interp_tx", ctypes.c_int32), ("interp_ty", ctypes.c_int32),
                ("gemm_bf16", ctypes.c_int32), ("fft_register", ctypes.c_int32),
                ("near_block", ctypes.c_int32 * 2), ("near_fork", ctypes.c_int32 * 2)]


class GmresOpts(ctypes.Structure):
    _fields_ = [("restart", ctypes.c_int32), ("max_iters", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("x0_given", ctypes.c_int32), ("check_every", ctypes.c_int32), ("precond", ctypes.c_int32),
                ("system", ctypes.c_int32), ("graphs", ctypes.c_int32), ("tol", ctypes.c_double)]


class GmresStat(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("restarts", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("matvecs", ctypes.c_int32), ("true_relres", ctypes.c_double)]


_LIB = None

EXPORTS = {
    "aim_build_grid": (ctypes.c_int, [ctypes.POINTER(AimSurface), ctypes.POINTER(AimArray), ctypes.c_void_p,
                                      ctypes.POINTER(ctypes.c_void_p)]),
    "aim_build_host": (ctypes.c_int, [ctypes.POINTER(AimSurface), ctypes.POINTER(AimArray),
                                      ctypes.POINTER(ctypes.c_void_p)]),
    "aim_set_macromodels": (ctypes.c_int, [ctypes.c_void_p, _f64p]),
    "aim_set_elem_type": (ctypes.c_int, [ctypes.c_void_p, _i32p, ctypes.c_void_p]),
    "aim_get_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(AimTuning)]),
    "aim_set_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(AimTuning)]),
    "aim_set_dmatrix": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, _i32p, _i32p, _f64p]),
    "macro_apply": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                   ctypes.c_int32, ctypes.c_void_p]),
    "aim_matvec": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                  ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]),
    "aim_time_kernels": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.c_int32, _f64p, ctypes.c_void_p]),
    "aim_project": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                   ctypes.c_int32, ctypes.c_void_p]),
    "aim_convolve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                    ctypes.c_int32, ctypes.c_void_p]),
    "aim_plane_wave_rhs": (ctypes.c_int, [ctypes.c_void_p, _f64p, _f64p, _i32p, ctypes.c_int32,
                                          ctypes.c_void_p, ctypes.c_void_p]),
    "gmres_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                   ctypes.POINTER(GmresOpts), ctypes.POINTER(GmresStat), ctypes.c_void_p]),
    "aim_build_preconditioner": (ctypes.c_int, [ctypes.c_void_p]),
    "aim_get_preconditioner": (ctypes.c_int, [ctypes.c_void_p, _f64p]),
    "precond_apply": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                     ctypes.c_int32, ctypes.c_void_p]),
    "aim_far_field": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, _f64p,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "aim_far_field_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                             _f64p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                             ctypes.c_void_p]),
    "aim_build_macromodels": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(AimSurface), ctypes.c_void_p]),
    "aim_get_macromodel": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _f64p, _f64p, _f64p]),
    "aim_scatterer_unknowns": (ctypes.c_int64, [ctypes.c_void_p, ctypes.c_int32]),
    "aim_recover_currents": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                            ctypes.c_void_p]),
    "aim_get_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(AimInfo)]),
    "aim_get_near": (ctypes.c_int, [ctypes.c_void_p, _i32p, _i32p, _i32p, _f64p, _i32p]),
    "aim_footprint_bytes": (ctypes.c_size_t, [ctypes.POINTER(AimSurface), ctypes.POINTER(AimArray),
                                              ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "aim_destroy": (None, [ctypes.c_void_p]),
    "aim_last_error": (ctypes.c_char_p, []),
}


def load() -> ctypes.CDLL:
    """Load libaimm.so once; raise if it is missing (run the package build first)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1712_02443_amd.build.build()")
    # torch ships its own HIP runtime under the same soname; loading torch first makes
    # the library bind to that one runtime, so torch streams and pointers are valid here
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


class AimError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"aimm error {code}: {msg}")
        self.code = code


def check(code: int) -> int:
    if code < 0:
        raise AimError(code, load().aim_last_error().decode())
    return code


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


class Structs:
    """Host copies of the C structs plus the numpy arrays they point into."""

    def __init__(self, vert, tri, rwg, k, eta, h, r_near, order, px, py, pitch_cells, elem_type, n_types,
                 max_rhs):
        self.vert = np.ascontiguousarray(vert, dtype=np.float64)
        self.tri = np.ascontiguousarray(tri, dtype=np.int32)
        self.rwg = np.ascontiguousarray(rwg, dtype=np.int32)
        self.elem_type = np.ascontiguousarray(elem_type, dtype=np.int32)
        self.surface = AimSurface(self.vert.shape[0], self.tri.shape[0], self.rwg.shape[0],
                                  _ptr(self.vert, ctypes.c_double), _ptr(self.tri, ctypes.c_int32),
                                  _ptr(self.rwg, ctypes.c_int32))
        self.array = AimArray(float(k), float(eta), float(h), float(r_near), int(order), int(px), int(py),
                              int(pitch_cells), int(n_types), _ptr(self.elem_type, ctypes.c_int32), int(max_rhs))
