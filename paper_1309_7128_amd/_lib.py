"""ctypes view of libism.so (the C ABI of include/ism.h).

Argument marshalling only: no arithmetic of the solver happens here.  The library is
loaded from this package's directory; if it is missing the import of the binding fails
loudly (there is no fallback path).
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libism.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "ism.h")

ISM_OK = 0
ISM_NOT_CONVERGED = 1
ISM_ERR_INVALID = -1
ISM_ERR_UNSUPPORTED = -2
ISM_ERR_HIP = -3
ISM_ERR_NONFINITE = -4

ISM_BC_NEUMANN = 0
ISM_BC_PERIODIC = 1
ISM_BC_DIRICHLET = 2
ISM_BC_NEUMANN_DIRICHLET = 3
ISM_BC_DIRICHLET_NEUMANN = 4
ISM_PREC_FP64 = 0
ISM_PREC_MIXED = 1
ISM_COARSE_ISM = 0
ISM_COARSE_GMG5 = 1
ISM_COARSE_ACM = 2
ISM_CYCLE_REPEAT = 0
ISM_CYCLE_ONESHOT = 1
ISM_COARSE_GS_BLOCK = 0
ISM_COARSE_GS_MULTICOLOUR = 1
ISM_FUSED_OFF = 0
ISM_FUSED_AUTO = 1
ISM_FUSED_WALK = 2
ISM_FUSED_TILE = 3
ISM_F64 = 0
ISM_F32 = 1
KERNEL_CLASSES = {"cycle": 0, "smooth": 1, "restrict": 2, "prolong": 3, "coarse": 4, "outer": 5}


class IsmConfig(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("batch", ctypes.c_int32),
        ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32), ("coarsen", ctypes.c_int32),
        ("lx", ctypes.c_double), ("ly", ctypes.c_double),
        ("precision", ctypes.c_int32), ("nu", ctypes.c_int32),
        ("rtol", ctypes.c_double), ("inner_rtol", ctypes.c_double),
        ("max_cycles", ctypes.c_int32), ("max_outer", ctypes.c_int32),
        ("check_every", ctypes.c_int32), ("fused", ctypes.c_int32),
        ("stall_window", ctypes.c_int32), ("stall_drop", ctypes.c_double),
        ("coarse_stencil", ctypes.c_int32), ("cycling", ctypes.c_int32),
        ("coarse_tol", ctypes.c_double), ("fine_tol", ctypes.c_double),
        ("coarse_gs", ctypes.c_int32),
    ]


class IsmStats(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32), ("outer_iters", ctypes.c_int32),
        ("cycles", ctypes.c_int32), ("sweeps", ctypes.c_int32),
        ("launches", ctypes.c_int64), ("host_syncs", ctypes.c_int64),
        ("rel_res_l2", ctypes.c_double), ("rel_res_max", ctypes.c_double),
        ("seconds", ctypes.c_double),
        ("coarse_iters", ctypes.c_int32), ("fine_iters", ctypes.c_int32),
        ("coarse_syncs", ctypes.c_int32),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_P = ctypes.c_void_p
_I = ctypes.c_int32
_SIGNATURES = {
    "ism_config_init": (ctypes.c_int, [ctypes.POINTER(IsmConfig), _I, _I, _I]),
    "ism_create": (ctypes.c_int, [ctypes.POINTER(IsmConfig), _P, ctypes.POINTER(_P)]),
    "ism_destroy": (ctypes.c_int, [_P]),
    "ism_workspace_bytes": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_size_t)]),
    "ism_solve": (ctypes.c_int, [_P, _P, _P, ctypes.POINTER(IsmStats)]),
    "ism_solve_adjoint": (ctypes.c_int, [_P, _P, _P, ctypes.POINTER(IsmStats)]),
    "ism_solve_static": (ctypes.c_int, [ctypes.POINTER(IsmConfig), _P, _P,
                                        ctypes.POINTER(IsmStats), _P]),
    "ism_div": (ctypes.c_int, [_P, _P, _P, _P]),
    "ism_grad": (ctypes.c_int, [_P, _P, _P, _P]),
    "ism_div_adjoint": (ctypes.c_int, [_P, _P, _P, _P]),
    "ism_grad_adjoint": (ctypes.c_int, [_P, _P, _P, _P]),
    "ism_smooth": (ctypes.c_int, [_P, _I, _P, _P, _I]),
    "ism_restrict": (ctypes.c_int, [_P, _I, _P, _P, _P, _P]),
    "ism_prolong": (ctypes.c_int, [_P, _I, _P, _P]),
    "ism_coarse_solve": (ctypes.c_int, [_P, _P, _P]),
    "ism_cycle": (ctypes.c_int, [_P, _I, _P, _P, _P, _I, _P]),
    "ism_coarse_stencil": (ctypes.c_int, [_P, _P]),
    "ism_coarse_gs": (ctypes.c_int, [_P, _P, _P, ctypes.c_double, _I, ctypes.POINTER(_I)]),
    "ism_predict": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_double, ctypes.c_double, _P, _P, _P]),
    "ism_correct": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "ism_outer_residual": (ctypes.c_int, [_P, _P, _P, _P]),
    "ism_profile": (ctypes.c_int, [_P, _I]),
    "ism_profile_read": (ctypes.c_int, [_P, _I, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_int64)]),
    "ism_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "ism_last_error": (ctypes.c_char_p, [_P]),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load libism.so once; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python -m paper_1309_7128_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def exported_names():
    return sorted(_SIGNATURES)
