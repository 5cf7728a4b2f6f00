"""ctypes loader and prototypes for libsv.so (the C-ABI declared in include/sv.h).

The library is built in-tree by ``paper_1805_00988_amd/build.py``; nothing
here computes anything, and there is no fallback: if the shared library is
missing or fails to load, every call raises.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsv.so")

SV_C64, SV_C128 = 1, 2
SV_OK, SV_EINVAL, SV_ENOMEM, SV_EDEVICE, SV_EUNSUPPORTED = 0, -1, -2, -3, -4
SV_PREC_NATIVE, SV_PREC_FP32, SV_PREC_SPLIT_BF16 = 0, 1, 2
SV_RUN_PER_GATE, SV_RUN_TILED = 0, 1
GATE_KINDS = {"H": 1, "X": 2, "Y": 3, "Z": 4, "S": 5, "T": 6,
              "RX": 7, "RY": 8, "RZ": 9, "U1": 10, "U": 11}

EXPORTED = ("sv_state_bytes", "sv_alloc", "sv_free", "sv_set_basis", "sv_set_stream", "sv_sync",
            "sv_data", "sv_apply_gate", "sv_apply_fused", "sv_probabilities", "sv_expectation",
            "sv_expectation_noalloc", "sv_marginals", "sv_collapse", "sv_measure", "sv_sample",
            "sv_run", "sv_schedule", "sv_fuse", "sv_run_fused", "sv_fused_tune", "sv_adjoint_grad", "sv_batch_create",
            "sv_batch_run", "sv_batch_results", "sv_batch_output", "sv_batch_state",
            "sv_batch_tune", "sv_batch_config", "sv_batch_free", "sv_timing", "sv_timing_read", "sv_last_error",
            "sv_version")
SV_BATCH_KEEP_STATES = 1


class sv_op(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n_targets", ctypes.c_int32),
                ("targets", ctypes.c_int32 * 2), ("ctrl_mask", ctypes.c_uint64),
                ("param_index", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("theta", ctypes.c_double), ("matrix", ctypes.c_double * 32)]


class sv_kernel_stat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 24), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double), ("bytes", ctypes.c_double), ("flops", ctypes.c_double)]


class SVError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libsv error {code}: {msg}")
        self.code = code


_lib = None

_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_DP = ctypes.POINTER(ctypes.c_double)
_IP = ctypes.POINTER(ctypes.c_int)
_U64 = ctypes.c_uint64
_U64P = ctypes.POINTER(ctypes.c_uint64)
_OPP = ctypes.POINTER(sv_op)

_PROTOS = {
    "sv_state_bytes": (ctypes.c_size_t, [_I, _I]),
    "sv_alloc": (_I, [_I, _I, _P, _P, ctypes.POINTER(_P)]),
    "sv_free": (_I, [_P]),
    "sv_set_basis": (_I, [_P, _U64]),
    "sv_set_stream": (_I, [_P, _P]),
    "sv_sync": (_I, [_P]),
    "sv_data": (_P, [_P]),
    "sv_apply_gate": (_I, [_P, _I, _IP, _U64, _DP]),
    "sv_apply_fused": (_I, [_P, _I, _IP, _DP, _I]),
    "sv_probabilities": (_I, [_P, _P, _DP]),
    "sv_expectation": (_I, [_P, _I, _U64P, _DP, _DP]),
    "sv_expectation_noalloc": (_I, [_P, _I, _I, _I, _U64P, _DP, _P, _P]),
    "sv_marginals": (_I, [_P, _U64, _DP]),
    "sv_collapse": (_I, [_P, _U64, _U64, _DP]),
    "sv_measure": (_I, [_P, _U64, ctypes.c_double, _U64P, _DP]),
    "sv_sample": (_I, [_P, _I, _DP, _U64P]),
    "sv_run": (_I, [_P, _OPP, _I, _DP, _I, _I]),
    "sv_schedule": (_I, [_I, _I, _OPP, _I, _DP, _I, _I, _I, _IP, _U64P, _IP]),
    "sv_fuse": (_I, [_I, _OPP, _I, _DP, _I, _I, _I, _IP, _IP, _DP, _IP, _IP]),
    "sv_fused_tune": (_I, [_P, _OPP, _I, _DP, _I, _I, _I, _I, _IP, _IP, _DP]),
    "sv_run_fused": (_I, [_P, _OPP, _I, _DP, _I, _I, _I, _IP]),
    "sv_adjoint_grad": (_I, [_P, _P, _OPP, _I, _DP, _I, _I, _U64P, _DP, _DP, _DP]),
    "sv_batch_create": (_I, [_I, _IP, ctypes.POINTER(ctypes.c_int64), _OPP, _DP, _I, _I, _U64, _I,
                             _P, ctypes.POINTER(_P)]),
    "sv_batch_run": (_I, [_P]),
    "sv_batch_results": (_I, [_P, _DP]),
    "sv_batch_output": (_P, [_P]),
    "sv_batch_state": (_I, [_P, _I, _P]),
    "sv_batch_tune": (_I, [_P, _I, _IP, _IP, _IP, _IP, _DP]),
    "sv_batch_config": (_I, [_P, _I, _I, _I, _I]),
    "sv_batch_free": (_I, [_P]),
    "sv_timing": (_I, [_P, _I]),
    "sv_timing_read": (_I, [_P, ctypes.POINTER(sv_kernel_stat), _I, _IP]),
    "sv_last_error": (ctypes.c_char_p, []),
    "sv_version": (ctypes.c_char_p, []),
}


def lib_path() -> str:
    return LIB_PATH


def load():
    """Load libsv.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python __graft_entry__.py build` "
                               "(or paper_1805_00988_amd/build.py) first")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _PROTOS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(code: int) -> None:
    if code != SV_OK:
        raise SVError(code, load().sv_last_error().decode())
