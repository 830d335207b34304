"""ctypes view of libmls.so (the C ABI declared in include/mls.h).

Argument marshalling only. Loading fails loudly when the library has not been
built: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libmls.so")

MLS_OK, MLS_ERR_INVALID_ARGUMENT, MLS_ERR_TOO_FEW_POINTS = 0, 1, 2
MLS_ERR_UNSUPPORTED, MLS_ERR_WORKSPACE_TOO_SMALL, MLS_ERR_OUT_OF_MEMORY, MLS_ERR_HIP = 3, 4, 5, 6
MLS_F32, MLS_F64 = 0, 1
MLS_MAX_K = 64
NOALLOC_SCRATCH_BYTES = 64 << 20
MLS_MAX_PLANE_ITERS = 16
MLS_PREC_FP64, MLS_PREC_FP32_MOMENTS = 0, 1
MLS_STAGE_ALL, MLS_STAGE_SEARCH, MLS_STAGE_FIT, MLS_STAGE_REFRESH = 0, 1, 2, 4
PT_OK, PT_OUTLIER, PT_PLANE_ONLY, PT_NONFINITE, PT_FLAG_AMBIGUOUS = 0, 1, 2, 3, 0x10
PT_NO_MINIMUM = 4
PT_FLAG_TRUNCATED = 0x20
MAX_K = 64

# Every function the header declares, with (restype, argtypes).
_P = ctypes.c_void_p
_I32, _I64, _F64, _SZ = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
_ST = ctypes.c_int


MLS_SLOT_QUERIES = 1
MLS_SLOT_OUTPUTS = 2
MLS_SLOT_OWN_POINTS = 4


class MlsParams(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("support_radius_h", ctypes.c_double), ("min_support", ctypes.c_int32),
                ("stages", ctypes.c_int32), ("search_extra", ctypes.c_int32),
                ("plane_iters", ctypes.c_int32), ("ball", ctypes.c_int32),
                ("levin", ctypes.c_int32), ("slot_order", ctypes.c_int32)]


class MlsGridInfo(ctypes.Structure):
    _fields_ = [("n_points", ctypes.c_int64), ("n_clouds", ctypes.c_int32),
                ("key_bits", ctypes.c_int32), ("n_cells", ctypes.c_int64),
                ("hash_capacity", ctypes.c_int64), ("n_nonfinite", ctypes.c_int64),
                ("min_cloud_finite", ctypes.c_int64)]


SIGNATURES = {
    "mls_version": (ctypes.c_char_p, []),
    "mls_status_string": (ctypes.c_char_p, [_ST]),
    "mls_last_error": (ctypes.c_char_p, []),
    "mls_grid_workspace_bytes": (_SZ, [_I64, _I32]),
    "mls_build_grid": (_ST, [_P, _I64, _P, _I32, _P, _P, _P, _SZ, _P, ctypes.POINTER(_P)]),
    "mls_grid_destroy": (_ST, [_P]),
    "mls_rebuild_grid": (_ST, [_P, _P, _P]),
    "mls_get_grid_info": (_ST, [_P, ctypes.POINTER(MlsGridInfo)]),
    "mls_get_cloud_grid": (_ST, [_P, _I32, _P, _P, _P]),
    "mls_grid_sorted_points": (_ST, [_P, ctypes.POINTER(_P), ctypes.POINTER(_P)]),
    "mls_grid_cell_table": (_ST, [_P, ctypes.POINTER(_P), ctypes.POINTER(ctypes.c_int64),
                                  ctypes.POINTER(_P)]),
    "mls_project_workspace_bytes": (_SZ, [_P, _I32, _I64]),
    "mls_project_backward_workspace_bytes": (_SZ, [_P, _I32, _I64, _I32]),
    "mls_autotune_workspace_bytes": (_SZ, [_I64, _I32, _I32, _I32]),
    "mls_autotune_cell": (_ST, [_P, _I64, _P, _I32, _P, _I32, _P, _I32, _I32, _P, _SZ, _P, _P,
                                _P]),
    "mls_knn": (_ST, [_P, _I32, _P, _ST, _I64, _P, _P, _P, _P, _SZ, _P]),
    "mls_project": (_ST, [_P, ctypes.POINTER(MlsParams), _P, _ST, _I64, _P, _P, _P, _P, _P,
                          _SZ, _P]),
    "mls_project_backward": (_ST, [_P, ctypes.POINTER(MlsParams), _P, _ST, _I64, _P, _P, _P,
                                   _P, _P, _P, _SZ, _P]),
    "mls_project_geometry": (_ST, [_P, ctypes.POINTER(MlsParams), _P, _ST, _I64, _P, _P, _P, _P,
                                   _P, _P, _P, _SZ, _P]),
    "mls_project_noalloc": (_ST, [_P, ctypes.POINTER(MlsParams), _P, _ST, _I64, _P, _P, _P, _P,
                                  _P]),
}

_lib = None


class MLSError(RuntimeError):
    def __init__(self, code, where, detail=""):
        self.code = code
        msg = "%s failed: %s (%d)" % (where, status_string(code), code)
        if detail:
            msg += ": " + detail
        super().__init__(msg)


def load(path: str = LIB_PATH):
    """Load libmls.so; raises if it is missing (build it with
    ``python -m paper_2401_03365_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError("libmls.so not found at %s: build the HIP library first "
                               "(python -m paper_2401_03365_amd.build)" % path)
        lib = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def status_string(code):
    try:
        return load().mls_status_string(code).decode()
    except Exception:  # pragma: no cover - message only
        return "status %d" % code


def check(code, where):
    if code != MLS_OK:
        detail = load().mls_last_error().decode() if code == MLS_ERR_HIP else ""
        raise MLSError(code, where, detail)
