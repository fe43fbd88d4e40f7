"""ctypes binding of the C ABI in include/lbm.h (argument marshalling only).

Loads the in-tree ``liblbm_hip.so``.  There is no fallback: if the library is
missing every call raises, so nothing can silently run elsewhere.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm_hip.so")

D2Q9 = 0
D3Q19 = 1

STORE_F64 = 0
STORE_F32 = 1
STORE_F16 = 2
STORE_BF16 = 3

FLAG_SHIFTED = 1

OK = 0
ERR_ARG = -1
ERR_GEOMETRY = -2
ERR_UNSUPPORTED = -3
ERR_HIP = -4
ERR_STATE = -5
ERR_NONFINITE = -6

# Every symbol declared in include/lbm.h with (argtypes, restype).
_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_U = ctypes.c_uint
_SZ = ctypes.c_size_t
_PSZ = ctypes.POINTER(ctypes.c_size_t)
_PP = ctypes.POINTER(ctypes.c_void_p)
_PLL = ctypes.POINTER(ctypes.c_longlong)
_PI = ctypes.POINTER(ctypes.c_int)
_PD = ctypes.POINTER(ctypes.c_double)

SIGNATURES = {
    "lbm_required_bytes": ([_I, _I, _I, _I, _I, _PSZ, _PSZ], _I),
    "lbm_lattice_create": ([_PP, _I, _I, _I, _I, _D, _I, _U, _P, _SZ, _P, _SZ, _P], _I),
    "lbm_validate_geometry": ([_I, _I, _I, _I, _P, _U], _I),
    "lbm_set_geometry": ([_P, _P, _U], _I),
    "lbm_set_wall_velocity": ([_P, _P], _I),
    "lbm_set_body_force": ([_P, _P], _I),
    "lbm_set_tau": ([_P, _D], _I),
    "lbm_init_equilibrium": ([_P, _P, _P], _I),
    "lbm_set_populations": ([_P, _P], _I),
    "lbm_get_populations": ([_P, _P], _I),
    "lbm_step": ([_P, _I], _I),
    "lbm_set_graph_steps": ([_P, _I], _I),
    "lbm_moments": ([_P, _P, _P], _I),
    "lbm_moments_device": ([_P, _P, _P], _I),
    "lbm_totals": ([_P, _P, _P, _P], _I),
    "lbm_totals_noalloc": ([_P, _P, _P, _P], _I),
    "lbm_get_info": ([_P, _PLL, _PLL], _I),
    "lbm_lattice_destroy": ([_P], _I),
    "lbm_status_string": ([_I], ctypes.c_char_p),
    "lbm_last_error": ([_P], ctypes.c_char_p),
    "lbm_batch_required_bytes": ([_I, _I, _P, _I, _PSZ, _PSZ], _I),
    "lbm_batch_create": ([_PP, _I, _I, _P, _P, _I, _U, _P, _SZ, _P, _SZ, _P], _I),
    "lbm_batch_lattice": ([_P, _I, _PP], _I),
    "lbm_batch_step": ([_P, _I], _I),
    "lbm_batch_set_graph_steps": ([_P, _I], _I),
    "lbm_batch_set_launch": ([_P, _I, _I], _I),
    "lbm_batch_set_phase_launch": ([_P, _I, _I, _I], _I),
    "lbm_batch_get_phase_launch": ([_P, _I, _PI, _PI], _I),
    "lbm_batch_autotune": ([_P, _I, _PI, _PI, _PD], _I),
    "lbm_batch_get_info": ([_P, _PI, _PLL, _PI, _PI], _I),
    "lbm_batch_destroy": ([_P], _I),
    "lbm_batch_last_error": ([_P], ctypes.c_char_p),
    "lbm_porous_required_bytes": ([_I, _I, _I, _I, _I, _PSZ], _I),
    "lbm_porous_create": ([_PP, _I, _I, _I, _D, _P, _U, _P, _I, _I, _I, _P, _SZ, _P], _I),
    "lbm_porous_forward": ([_P, _P, _PD], _I),
    "lbm_porous_backward": ([_P, _P], _I),
    "lbm_porous_get_final": ([_P, _P], _I),
    "lbm_porous_generation": ([_P, _PLL], _I),
    "lbm_porous_destroy": ([_P], _I),
    "lbm_porous_last_error": ([_P], ctypes.c_char_p),
}

_lib = None


class LBMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def load():
    """Load liblbm_hip.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2307_11752_amd.build` "
            "(or __graft_entry__.build()) before using the GPU path")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (args, res) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def check(status, handle=None):
    if status != OK:
        lib = load()
        msg = lib.lbm_last_error(handle).decode() or lib.lbm_status_string(status).decode()
        raise LBMError(status, msg)
    return status


def check_porous(status, handle):
    if status != OK:
        lib = load()
        msg = (lib.lbm_porous_last_error(handle).decode() if handle else "") or \
            lib.lbm_last_error(None).decode() or lib.lbm_status_string(status).decode()
        raise LBMError(status, msg)
    return status


def check_batch(status, batch):
    if status != OK:
        lib = load()
        msg = lib.lbm_batch_last_error(batch).decode() or lib.lbm_last_error(None).decode() or \
            lib.lbm_status_string(status).decode()
        raise LBMError(status, msg)
    return status
