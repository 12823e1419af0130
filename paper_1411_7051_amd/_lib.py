"""ctypes declarations of the C ABI in ``include/lbk.h``.

Argument marshalling only: every step of the method runs in the HIP
library.  Loading fails loudly when ``liblbk.so`` has not been built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# LBK_LIB points the binding at another build of the same library (the
# host-sanitizer build of the tests)
LIB_PATH = os.environ.get("LBK_LIB", os.path.join(HERE, "liblbk.so"))

LBK_OK = 0
STATUS = {
    0: "LBK_OK",
    -1: "LBK_ERR_INVALID_ARG",
    -2: "LBK_ERR_DEVICE",
    -3: "LBK_ERR_OOM",
    -4: "LBK_ERR_NONFINITE",
    -5: "LBK_ERR_UNSUPPORTED",
}
STORAGE = {"f32": 0, "f16": 1, "bf16": 2}
OBJECTIVE = {"k_app": 0, "q_out": 1}
CORRELATION = {"bkc": 0, "klinkenberg": 1, "none": 2}
PASS_MODE = {"auto": 0, "two_step": 1, "single": 2, "three_step": 3}


class LbkError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class Desc(ctypes.Structure):
    """``lbk_desc``."""

    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32),
        ("storage", ctypes.c_int32), ("kn_local", ctypes.c_int32),
        ("init", ctypes.c_int32), ("check_every", ctypes.c_int32),
        ("tau", ctypes.c_double),
        ("gx", ctypes.c_double), ("gy", ctypes.c_double),
        ("f_eps", ctypes.c_double),
        ("rho_in", ctypes.c_double), ("rho_out", ctypes.c_double),
        ("rho0", ctypes.c_double), ("rho_ref", ctypes.c_double),
        ("slip_b", ctypes.c_double),
        ("correlation", ctypes.c_int32), ("pass_mode", ctypes.c_int32),
        ("band", ctypes.c_int32),
    ]


class Desc3(ctypes.Structure):
    """``lbk_desc3``."""

    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32), ("bc_z", ctypes.c_int32),
        ("storage", ctypes.c_int32), ("kn_local", ctypes.c_int32),
        ("init", ctypes.c_int32), ("check_every", ctypes.c_int32),
        ("correlation", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("tau", ctypes.c_double),
        ("gx", ctypes.c_double), ("gy", ctypes.c_double), ("gz", ctypes.c_double),
        ("f_eps", ctypes.c_double),
        ("rho_in", ctypes.c_double), ("rho_out", ctypes.c_double),
        ("rho0", ctypes.c_double), ("rho_ref", ctypes.c_double),
        ("slip_b", ctypes.c_double),
    ]


# Every symbol include/lbk.h declares, with (restype, argtypes).
_P = ctypes.c_void_p
_SIG = {
    "lbk_desc_default": (ctypes.c_int, [ctypes.POINTER(Desc)]),
    "lbk_workspace_size": (ctypes.c_int, [ctypes.POINTER(Desc), ctypes.POINTER(ctypes.c_size_t)]),
    "lbk_create": (ctypes.c_int, [ctypes.POINTER(Desc), _P, _P, _P, _P, ctypes.c_size_t, _P,
                                  ctypes.POINTER(_P)]),
    "lbk_destroy": (ctypes.c_int, [_P]),
    "lbk_step": (ctypes.c_int, [_P, ctypes.c_int64]),
    "lbk_time": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64)]),
    "lbk_steps_per_launch": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32)]),
    "lbk_read_macroscopic": (ctypes.c_int, [_P, _P, _P, _P]),
    "lbk_read_populations": (ctypes.c_int, [_P, _P]),
    "lbk_apparent_permeability": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double)]),
    "lbk_apparent_permeability_noalloc": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double)]),
    "lbk_diagnostics": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_double)]),
    "lbk_state_size": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_size_t)]),
    "lbk_save_state": (ctypes.c_int, [_P, _P]),
    "lbk_load_state": (ctypes.c_int, [_P, _P]),
    "lbk_adjoint_workspace_size": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int64,
                                                  ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)]),
    "lbk_adjoint_plan": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int64, ctypes.c_size_t,
                                        ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_size_t)]),
    "lbk_adjoint_forward": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int64, ctypes.c_int64,
                                           ctypes.c_int64, _P, ctypes.c_size_t,
                                           ctypes.POINTER(ctypes.c_double)]),
    "lbk_adjoint_backward": (ctypes.c_int, [_P, _P, ctypes.c_size_t, _P, _P]),
    "lbk_batch_workspace_size": (ctypes.c_int, [_P, ctypes.c_int32,
                                                ctypes.POINTER(ctypes.c_size_t)]),
    "lbk_batch_create": (ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_size_t,
                                        ctypes.POINTER(_P)]),
    "lbk_batch_destroy": (ctypes.c_int, [_P]),
    "lbk_batch_step": (ctypes.c_int, [_P, ctypes.c_int64]),
    "lbk_batch_set_launch": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.c_int32]),
    "lbk_batch_get_launch": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32),
                                            ctypes.POINTER(ctypes.c_int32),
                                            ctypes.POINTER(ctypes.c_int32),
                                            ctypes.POINTER(ctypes.c_int32)]),
    "lbk_batch_set_graph_readout": (ctypes.c_int, [_P, ctypes.c_int32]),
    "lbk_batch_set_pass_mode": (ctypes.c_int, [_P, ctypes.c_int32]),
    "lbk_batch_get_pass_mode": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32),
                                               ctypes.POINTER(ctypes.c_int32)]),
    "lbk_batch_autotune": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]),
    "lbk_batch_apparent_permeability": (ctypes.c_int, [_P, _P]),
    "lbk_batch_check": (ctypes.c_int, [_P]),
    "lbk_batch_adjoint_workspace_size": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int64,
                                                        ctypes.c_int64,
                                                        ctypes.POINTER(ctypes.c_size_t)]),
    "lbk_batch_adjoint_plan": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int64,
                                              ctypes.c_size_t, ctypes.POINTER(ctypes.c_int64),
                                              ctypes.POINTER(ctypes.c_size_t)]),
    "lbk_batch_adjoint_forward": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int64,
                                                 ctypes.c_int64, ctypes.c_int64, _P,
                                                 ctypes.c_size_t, _P]),
    "lbk_batch_adjoint_backward": (ctypes.c_int, [_P, _P, ctypes.c_size_t, _P, _P]),
    "lbk_correction_factor": (ctypes.c_int, [ctypes.c_int32, ctypes.c_double, _P, _P,
                                             ctypes.c_size_t]),
    "lbk3_desc_default": (ctypes.c_int, [ctypes.POINTER(Desc3)]),
    "lbk3_workspace_size": (ctypes.c_int, [ctypes.POINTER(Desc3),
                                           ctypes.POINTER(ctypes.c_size_t)]),
    "lbk3_create": (ctypes.c_int, [ctypes.POINTER(Desc3), _P, _P, _P, _P, ctypes.c_size_t, _P,
                                   ctypes.POINTER(_P)]),
    "lbk3_destroy": (ctypes.c_int, [_P]),
    "lbk3_step": (ctypes.c_int, [_P, ctypes.c_int64]),
    "lbk3_time": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64)]),
    "lbk3_scale_exponent": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32)]),
    "lbk3_read_macroscopic": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "lbk3_read_populations": (ctypes.c_int, [_P, _P]),
    "lbk3_apparent_permeability": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double)]),
    "lbk3_diagnostics": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double)]),
    "lbk_last_error": (ctypes.c_char_p, []),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load ``liblbk.so`` (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"HIP library {LIB_PATH} is not built; run __graft_entry__.build() "
                "(hipcc --offload-arch=gfx950)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIG.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def symbols():
    return list(_SIG)


def check(status: int) -> None:
    if status != LBK_OK:
        msg = load().lbk_last_error()
        raise LbkError(status, msg.decode() if msg else "")
