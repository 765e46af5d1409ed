"""ctypes declarations of include/plss.h and loading of libplss.so.

The library is loaded from this package directory only; if it is missing the
import fails (there is no fallback implementation)."""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libplss.so")

PLSS_OK, PLSS_NOT_CONVERGED, PLSS_BREAKDOWN, PLSS_PENDING = 0, 1, 2, 3
PLSS_EINVAL, PLSS_ENOMEM, PLSS_EDEVICE, PLSS_ECANCELLED = -1, -2, -3, -4
SKETCH = {"residual": 0, "identity": 1, "mixed": 2, "block_identity": 3, "block_mixed": 4, "randproj": 5}
DTYPE = {"f64": 0, "float64": 0, "f32": 1, "float32": 1}


class plss_csr(C.Structure):
    _fields_ = [("m", C.c_int64), ("n", C.c_int64), ("nnz", C.c_int64),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("values", C.c_void_p)]


class plss_opts(C.Structure):
    _fields_ = [("sketch", C.c_int), ("tol", C.c_double), ("maxit", C.c_int64),
                ("tol_absolute", C.c_int32), ("refine", C.c_int32), ("inner_tol", C.c_double),
                ("max_outer", C.c_int64), ("x0", C.c_void_p), ("wi_diag", C.c_void_p),
                ("row_perm", C.c_void_p), ("hist_cap", C.c_int64), ("chunk", C.c_int32),
                ("timing", C.c_int32), ("engine", C.c_int32), ("block", C.c_int32),
                ("seed", C.c_uint64)]


class plss_info(C.Structure):
    _fields_ = [("iters", C.c_int64), ("outer_iters", C.c_int64), ("relres", C.c_double),
                ("relres_true", C.c_double), ("status", C.c_int32), ("ms", C.c_double)]


class plss_layout(C.Structure):
    _fields_ = [("a_stripes", C.c_int32), ("t_stripes", C.c_int32), ("unit_rows", C.c_int32)]


ENGINE = {"auto": 0, "multi": 1, "single": 2}


EXPORTS = {
    # name: (restype, argtypes)
    "plss_opts_default": (None, [C.POINTER(plss_opts)]),
    "plss_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int]),
    "plss_destroy": (C.c_int, [C.c_void_p]),
    "plss_matrix_create": (C.c_int, [C.c_void_p, C.POINTER(plss_csr), C.c_int, C.POINTER(C.c_void_p)]),
    "plss_matrix_destroy": (C.c_int, [C.c_void_p]),
    "plss_matrix_info": (C.c_int, [C.c_void_p] + [C.POINTER(C.c_int64)] * 4),
    "plss_matrix_csc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "plss_matrix_autotune": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "plss_matrix_layout": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(plss_layout), C.POINTER(plss_layout)]),
    "plss_spmv": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    "plss_spmv_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    "plss_release_workspace": (C.c_int, [C.c_void_p]),
    "plss_residual_pair": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.POINTER(C.c_double)]),
    "plss_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(plss_opts), C.c_void_p,
                             C.c_void_p, C.c_int64, C.POINTER(plss_info)]),
    "plss_solve_batch": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                   C.POINTER(plss_opts), C.POINTER(C.c_void_p), C.POINTER(plss_info)]),
    "plss_solve_multi": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(plss_opts),
                                   C.c_void_p, C.POINTER(plss_info)]),
    "plss_kernel_times": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "plss_server_create": (C.c_int, [C.c_void_p, C.c_size_t, C.c_int32, C.POINTER(C.c_void_p)]),
    "plss_server_submit": (C.c_int, [C.c_void_p, C.POINTER(plss_csr), C.c_int, C.c_void_p,
                                     C.POINTER(plss_opts), C.POINTER(C.c_uint64)]),
    "plss_server_poll": (C.c_int, [C.c_void_p, C.c_uint64, C.c_void_p, C.POINTER(plss_info)]),
    "plss_server_drain": (C.c_int, [C.c_void_p]),
    "plss_server_cancel": (C.c_int, [C.c_void_p, C.c_uint64]),
    "plss_server_stats": (C.c_int, [C.c_void_p] + [C.POINTER(C.c_int64)] * 4),
    "plss_server_destroy": (C.c_int, [C.c_void_p]),
    "plss_status_string": (C.c_char_p, [C.c_int]),
    "plss_last_error": (C.c_char_p, []),
}

_lib = None


def _single_runtime():
    """PyTorch ships its own HIP runtime (same SONAME as ROCm's).  Importing
    torch before libplss.so makes the library bind to that runtime, so torch
    device pointers and library pointers live in one runtime; loading
    libplss.so first would map a second runtime once torch is imported."""
    import importlib.util
    if importlib.util.find_spec("torch") is not None:
        import torch  # noqa: F401


def load() -> C.CDLL:
    global _lib
    if _lib is None:
        _single_runtime()
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2207_07615_amd.build`")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib
