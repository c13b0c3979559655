"""ctypes declarations of libmde.so (the C ABI in include/mde.h).

Loading fails loudly when the library has not been built: there is no
fallback implementation anywhere in this package.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmde.so")

MDE_OK, MDE_INVALID, MDE_NOMEM, MDE_DEVICE, MDE_STATE, MDE_UNSUPPORTED = range(6)
STATUS_NAMES = {0: "OK", 1: "INVALID", 2: "NOMEM", 3: "DEVICE", 4: "STATE", 5: "UNSUPPORTED"}
MDE_FP64, MDE_MIXED, MDE_MIXED_GEMM, MDE_MIXED_GEMM_KSUM64 = 0, 1, 2, 3
ST_SINGULAR_REF, ST_SMALL_RATIO, ST_NONFINITE, ST_ZERO_PSI, ST_REF_ILLCOND = 1, 2, 4, 8, 16


class MdeDesc(C.Structure):
    _fields_ = [("n_elec", C.c_int32 * 2), ("n_orb", C.c_int32 * 2),
                ("max_walkers", C.c_int32), ("max_order", C.c_int32),
                ("refresh_every", C.c_int32), ("precision", C.c_int32)]


class MdeError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libmde {STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None

_P = C.c_void_p
_I = C.c_int32
_SIGS = {
    "mde_version": ([], C.c_char_p),
    "mde_error_string": ([_P], C.c_char_p),
    "mde_group_error_string": ([_P], C.c_char_p),
    "mde_create": ([C.POINTER(MdeDesc), _P, C.POINTER(_P)], C.c_int),
    "mde_destroy": ([_P], C.c_int),
    "mde_set_excitations": ([_P, _I, _I, _P, _P, _P], C.c_int),
    "mde_set_ci": ([_P, C.c_int64, _P, _P, _P], C.c_int),
    "mde_set_reference": ([_P, _I, _I], C.c_int),
    "mde_workspace_bytes": ([_P, _I, C.POINTER(C.c_size_t)], C.c_int),
    "mde_bind_workspace": ([_P, _I, _P, C.c_size_t], C.c_int),
    "mde_init": ([_P, _I, _P, _P, _P, _P, _P], C.c_int),
    "mde_refresh": ([_P, _P, _P, _P], C.c_int),
    "mde_propose": ([_P, _I, _P, _P, _P, _P, _P], C.c_int),
    "mde_grad_lap": ([_P, _I, _P, _P, _P, _P], C.c_int),
    "mde_accept": ([_P, _I, _P], C.c_int),
    "mde_local_derivs": ([_P, _P, _P, _P, _P, _P], C.c_int),
    "mde_local_derivs_noalloc": ([_P, _P, _P, _P, _P, _P], C.c_int),
    "mde_vmc": ([_P, _I, C.c_double, _P, _P, _P, _P, _P], C.c_int),
    "mde_export": ([_P, _I, _I, _P], C.c_int),
    "mde_eval_tables": ([_P, _I, _P, _P, _P, _P, _P, _P], C.c_int),
    "mde_backward": ([_P, _P, _P, _P, _P, _P], C.c_int),
    "mde_set_plan": ([_P, _I, _I, _I, _I], C.c_int),
    "mde_get_plan": ([_P, _I, C.POINTER(_I), C.POINTER(_I), C.POINTER(_I)], C.c_int),
    "mde_debug_items": ([_P, _I, _I, _I, _I, _I, _P, _I, C.POINTER(_I), _P, _I, C.POINTER(_I), _P],
                        C.c_int),
    "mde_autotune": ([_P, _P, _P, C.c_char_p], C.c_int),
    "mde_profile_enable": ([_P, _I, _I], C.c_int),
    "mde_profile_read": ([_P, C.POINTER(C.c_double), C.POINTER(_I)], C.c_int),
    "mde_profile_disable": ([_P], C.c_int),
    "mde_capture_begin": ([_P], C.c_int),
    "mde_capture_end": ([_P, C.POINTER(_P)], C.c_int),
    "mde_graph_launch": ([_P, _P], C.c_int),
    "mde_graph_destroy": ([_P], C.c_int),
    "mde_group_workspace_bytes": ([_P, _I, C.POINTER(C.c_size_t)], C.c_int),
    "mde_group_create": ([_P, _I, _P, C.c_size_t, C.POINTER(_P)], C.c_int),
    "mde_group_destroy": ([_P], C.c_int),
    "mde_group_propose": ([_P, _P, _P, _P, _P, _P, _P], C.c_int),
    "mde_group_accept": ([_P, _P, _P], C.c_int),
    "mde_group_tune": ([_P, _P, _P], C.c_int),
    "mde_group_capture_begin": ([_P], C.c_int),
    "mde_group_capture_end": ([_P, C.POINTER(_P)], C.c_int),
    "mde_sgauss_set_basis": ([_P, _I, _I, _P, _P, _P], C.c_int),
    "mde_sgauss_eval": ([_P, _I, _I, _P, _P], C.c_int),
}


def exported_symbols():
    return sorted(_SIGS)


def lib():
    """Load libmde.so (raises if it is missing or incomplete)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} not found: build it with `python -m paper_1106_2456_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)          # AttributeError if a symbol is missing
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib
