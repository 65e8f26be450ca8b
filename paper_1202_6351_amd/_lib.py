"""ctypes declarations of liblbm.so (the C ABI in include/lbm.h).

Argument marshalling only.  Loading fails loudly if the library has not been
built: there is no CPU fallback anywhere in this package.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_EDEVICE, LBM_ESTATE, LBM_EUNSUPPORTED, LBM_EUNSTABLE = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_EDEVICE", -3: "LBM_ESTATE",
                -4: "LBM_EUNSUPPORTED", -5: "LBM_EUNSTABLE"}
STORAGE = {"fp64": 0, "fp32": 1, "fp16": 2, "bf16": 3}
BC = {"periodic": 0, "wall": 1}
ROUNDING = {"nearest": 0, "stochastic": 1}


class LbmParams(ctypes.Structure):
    """Mirror of lbm_params."""
    _fields_ = [
        ("nx", ctypes.c_int32),
        ("ny", ctypes.c_int32),
        ("omega_nu", ctypes.c_double),
        ("omega3", ctypes.c_double),
        ("omega6", ctypes.c_double),
        ("omega7", ctypes.c_double),
        ("omega8", ctypes.c_double),
        ("fx", ctypes.c_double),
        ("fy", ctypes.c_double),
        ("bc", ctypes.c_int32 * 4),
        ("wall_u", ctypes.c_double * 4),
        ("rho0", ctypes.c_double),
        ("storage", ctypes.c_int32),
        ("rounding", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
    ]


# Every exported symbol of include/lbm.h with its (restype, argtypes).
_vp = ctypes.c_void_p
_st = ctypes.c_int
SIGNATURES = {
    "lbm_lattice_layout": (_st, [ctypes.POINTER(LbmParams), ctypes.POINTER(ctypes.c_int64),
                                 ctypes.POINTER(ctypes.c_int64)]),
    "lbm_create": (_st, [ctypes.POINTER(LbmParams), _vp, _vp, _vp, _vp, ctypes.POINTER(_vp)]),
    "lbm_destroy": (None, [_vp]),
    "lbm_last_error": (ctypes.c_char_p, [_vp]),
    "lbm_set_stream": (_st, [_vp, _vp]),
    "lbm_time": (ctypes.c_int64, [_vp]),
    "lbm_current_lattice": (_vp, [_vp]),
    "lbm_init_equilibrium": (_st, [_vp, _vp, _vp, _vp]),
    "lbm_set_populations": (_st, [_vp, _vp]),
    "lbm_get_populations": (_st, [_vp, _vp]),
    "lbm_step": (_st, [_vp, ctypes.c_int64]),
    "lbm_step_between": (_st, [_vp, _vp, _vp]),
    "lbm_step_sequence": (_st, [_vp, _vp, ctypes.POINTER(_vp), ctypes.c_int64]),
    "lbm_snapshot": (_st, [_vp, _vp]),
    "lbm_restore": (_st, [_vp, _vp, ctypes.c_int64]),
    "lbm_macroscopic": (_st, [_vp] * 7),
    "lbm_diagnostics": (_st, [_vp, ctypes.POINTER(ctypes.c_double)]),
    "lbm_diagnostics_noalloc": (_st, [_vp, _vp]),
    "lbm_adjoint_step": (_st, [_vp] * 5),
    "lbm_adjoint_sequence": (_st, [_vp, ctypes.POINTER(_vp), ctypes.c_int64, _vp, _vp, _vp,
                                   ctypes.POINTER(ctypes.c_int)]),
    "lbm_adjoint_macroscopic": (_st, [_vp] * 7),
    "lbm_adjoint_init": (_st, [_vp] * 9),
}

_lib = None


class LbmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        # PyTorch supplies the device memory and streams: its HIP runtime must
        # be the one in the process before liblbm.so resolves libamdhip64, or
        # the library would start a second runtime that sees no device.
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build the HIP library first "
                "(python paper_1202_6351_amd/build.py, or __graft_entry__.build()).")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def check(status: int, ctx=None) -> None:
    if status != LBM_OK:
        msg = lib().lbm_last_error(ctx)
        raise LbmError(status, msg.decode() if msg else "")
