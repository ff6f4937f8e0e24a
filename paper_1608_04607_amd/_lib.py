"""ctypes declarations of libdfm.so (the C ABI in include/dfm.h).

Loading fails loudly when the library has not been built: there is no
fallback implementation behind these names.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdfm.so")

DFM_OK = 0
STATUS_NAMES = {
    -1: "DFM_E_INVALID", -2: "DFM_E_MESH", -3: "DFM_E_NOMEM", -4: "DFM_E_HIP",
    -5: "DFM_E_NOCONV", -6: "DFM_E_UNSUPPORTED", -7: "DFM_E_NUMERIC",
}


class Basis(C.Structure):
    _fields_ = [("pos_order", C.c_int), ("mom_family", C.c_int), ("mom_degree", C.c_int),
                ("quad_n", C.c_int), ("rule", C.c_int), ("dtype", C.c_int)]


class SolveOpts(C.Structure):
    _fields_ = [("method", C.c_int), ("restart", C.c_int), ("max_iter", C.c_int),
                ("rtol", C.c_double), ("precision", C.c_int), ("warm_start", C.c_int)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("restarts", C.c_int), ("relres", C.c_double)]


# (name, restype, argtypes)
_P = C.c_void_p
_I64 = C.c_int64
_PROTOS = [
    ("dfm_mesh_build", C.c_int, [_P, _I64, _P, _I64, _P, _P, _P, _P, C.POINTER(_P)]),
    ("dfm_mesh_destroy", None, [_P]),
    ("dfm_mesh_info", C.c_int, [_P, C.POINTER(_I64), C.POINTER(_I64)]),
    ("dfm_mesh_export", C.c_int, [_P, _P, _P, _P, _P, _P]),
    ("dfm_assemble", C.c_int, [_P, C.POINTER(Basis), _P, _P, C.POINTER(_P)]),
    ("dfm_op_destroy", None, [_P]),
    ("dfm_op_info", C.c_int, [_P, C.POINTER(_I64), C.POINTER(_I64), C.POINTER(_I64), C.POINTER(_I64),
                              C.POINTER(_I64)]),
    ("dfm_op_export", C.c_int, [_P, _P, _P, _P]),
    ("dfm_op_export_tets", C.c_int, [_P, _P, _I64, _P, _P, _P]),
    ("dfm_apply", C.c_int, [_P, _P, _P, C.c_int, C.c_int, _P]),
    ("dfm_apply_f32", C.c_int, [_P, _P, _P, C.c_int, _P]),
    ("dfm_solve", C.c_int, [_P, _P, _P, C.c_int, C.POINTER(SolveOpts), C.POINTER(SolveInfo), _P]),
    ("dfm_solve_groups", C.c_int, [_P, _P, _P, C.c_int, C.POINTER(SolveOpts), C.POINTER(_I64), C.c_int,
                                   C.POINTER(SolveInfo), _P]),
    ("dfm_source_points", C.c_int, [_P, _P, _I64, C.c_double, _P, _P]),
    ("dfm_source_points_sum", C.c_int, [_P, _P, _I64, _P, C.c_int, C.c_double, _P, _P]),
    ("dfm_source_points_noalloc", C.c_int, [_P, _P, _I64, C.c_double, _P, _P]),
    ("dfm_source_plane", C.c_int, [_P, C.c_int, C.c_double, C.c_int, C.POINTER(C.c_double), C.c_double, _P, _P]),
    ("dfm_receiver_functional", C.c_int, [_P, _P, C.POINTER(C.c_double), _P, _P]),
    ("dfm_adjoint", C.c_int, [_P, _P, C.POINTER(C.c_double), _P, _P, C.c_int, C.POINTER(SolveOpts), _P, _P, _P,
                              C.POINTER(SolveInfo), _P]),
    ("dfm_receiver_energy", C.c_int, [_P, _P, C.POINTER(C.c_double), _P, C.c_int, _P, _P]),
    ("dfm_weighted_sum", C.c_int, [_P, _I64, C.c_int, _P, _P, _P]),
    ("dfm_residual", C.c_int, [_P, _P, _P, _P, C.c_int, _P]),
    ("dfm_apply_f16", C.c_int, [_P, _P, _P, C.c_int, _P]),
    ("dfm_product_timing", C.c_int, [_P, C.c_int, _P, _P, _P]),
    ("dfm_last_error", C.c_char_p, []),
]

EXPORTED = [name for name, _, _ in _PROTOS]

_lib = None


def load(path=LIB_PATH):
    """Load libdfm.so and declare every entry point (raises if it is missing).

    torch is imported first: it brings its own HIP runtime, and the library must
    bind to that same runtime (one process, one HIP runtime) instead of loading
    a second copy from the system."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1608_04607_amd.build` "
                          "(or __graft_entry__.build())")
    lib = C.CDLL(path)
    for name, res, args in _PROTOS:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class DFMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def check(code):
    if code != DFM_OK:
        raise DFMError(code, load().dfm_last_error().decode())
