"""ctypes view of libpamd (include/pamd.h).  Argument marshalling only.

The shared library is built in-tree by ``paper_1907_09529_amd.build_lib``;
loading fails loudly when it is missing - there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_size_t, c_uint64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpamd.so")

PAMD_OK = 0
PAMD_EINVAL = -1
PAMD_EUNSUPPORTED = -2
PAMD_EWORKSPACE = -3
PAMD_EHIP = -4

PAMD_HARMONIC = 0
PAMD_LJ = 1
PAMD_FP64 = 0
PAMD_FP32_FORCE = 1
PAMD_ALGO_AUTO = 0
PAMD_ALGO_FUSED = 1
PAMD_ALGO_PLAIN = 2
PAMD_LIST_AUTO = 0
PAMD_LIST_FULL = 1
PAMD_LIST_HALF = 2
PAMD_NOALLOC_SCRATCH_BYTES = 128 << 20

ERROR_NAMES = {PAMD_EINVAL: "PAMD_EINVAL", PAMD_EUNSUPPORTED: "PAMD_EUNSUPPORTED",
               PAMD_EWORKSPACE: "PAMD_EWORKSPACE", PAMD_EHIP: "PAMD_EHIP"}


class PamdPotential(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("reserved0", c_int32), ("k", c_double), ("eps", c_double),
                ("sigma", c_double), ("rc", c_double), ("box", c_double)]


class PamdPath(ctypes.Structure):
    _fields_ = [("n_steps", c_int64), ("n_atoms", c_int32), ("n_dim", c_int32),
                ("dt", c_double), ("D", c_double), ("gamma", c_double),
                ("precision", c_int32), ("reserved0", c_int32)]


class PamdTuning(ctypes.Structure):
    _fields_ = [("algo", c_int32), ("block", c_int32), ("tile", c_int32),
                ("max_neighbours", c_int32), ("skin", c_double), ("neighbour_list", c_int32),
                ("slot_arrays", c_int32)]


class PamdLaunch(ctypes.Structure):
    _fields_ = [("algo", c_int32), ("block", c_int32), ("tile", c_int32), ("n_tiles", c_int32),
                ("grid", c_int32), ("cells", c_int32), ("reach", c_int32),
                ("max_neighbours", c_int32), ("neighbour_list", c_int32), ("lds_bytes", c_int32),
                ("slot_arrays", c_int32), ("exact_lists", c_int32), ("skin", c_double)]


class PamdError(RuntimeError):
    def __init__(self, code: int, func: str, msg: str):
        super().__init__(f"{func}: {ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


_DP = POINTER(c_double)
_PATH = POINTER(PamdPath)
_POT = POINTER(PamdPotential)
_TUNE = POINTER(PamdTuning)

_SIGNATURES = {
    "pamd_workspace_size": (c_int32, [_PATH, _POT, _TUNE, POINTER(c_size_t)]),
    "pamd_launch_info": (c_int32, [_PATH, _POT, _TUNE, POINTER(PamdLaunch)]),
    "pamd_action": (c_int32, [_PATH, _POT, _TUNE, c_void_p, c_void_p, c_void_p, c_void_p,
                              c_size_t, c_void_p]),
    "pamd_action_grad": (c_int32, [_PATH, _POT, _TUNE, c_void_p, c_void_p, c_void_p, c_void_p,
                                   c_void_p, c_void_p, c_size_t, c_void_p]),
    "pamd_action_grad_noalloc": (c_int32, [_PATH, _POT, _TUNE, c_void_p, c_void_p, c_void_p,
                                           c_void_p, c_void_p, c_void_p]),
    "pamd_excess_action": (c_int32, [_PATH, _POT, _TUNE, c_void_p, c_void_p, c_void_p,
                                     c_void_p, c_size_t, c_void_p]),
    "pamd_log_norm": (c_double, [_PATH]),
    "pamd_last_error": (c_char_p, []),
    "pamd_version": (c_char_p, []),
    "pamd_batch_create": (c_int32, [c_int32, _PATH, _POT, _TUNE, POINTER(c_void_p)]),
    "pamd_batch_destroy": (None, [c_void_p]),
    "pamd_batch_layout": (c_int32, [c_void_p, POINTER(c_int64), POINTER(c_int64),
                                    POINTER(c_size_t)]),
    "pamd_batch_prepare": (c_int32, [c_void_p, c_void_p, c_size_t, c_void_p]),
    "pamd_batch_run": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                 c_void_p, c_void_p, c_size_t, c_void_p]),
    "pamd_batch_workspace_size": (c_int32, [c_int32, _PATH, _POT, POINTER(c_size_t)]),
    "pamd_batch_autotune_workspace_size": (c_int32, [c_void_p, POINTER(c_size_t)]),
    "pamd_batch_autotune": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p,
                                      POINTER(c_double), POINTER(c_double)]),
    "pamd_batch_action_grad": (c_int32, [c_int32, _PATH, _POT, POINTER(c_void_p), c_void_p,
                                         POINTER(c_void_p), c_void_p, c_size_t, c_void_p]),
    "pamd_mh_workspace_size": (c_int32, [_PATH, _POT, _TUNE, POINTER(c_size_t)]),
    "pamd_mh_step": (c_int32, [_PATH, _POT, _TUNE, c_uint64, c_int32, c_int32, c_void_p,
                               c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                               c_void_p, c_size_t, c_void_p]),
    "pamd_shift": (c_int32, [_PATH, c_uint64, c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                             c_void_p, c_void_p, c_void_p]),
    "pamd_run_workspace_size": (c_int32, [_PATH, _POT, _TUNE, c_int32, POINTER(c_size_t)]),
    "pamd_run": (c_int32, [_PATH, _POT, _TUNE, c_uint64, c_int32, c_int32, c_int32, c_int32,
                           c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                           c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "pamd_langevin_workspace_size": (c_int32, [_PATH, _POT, _TUNE, POINTER(c_size_t)]),
    "pamd_langevin_step": (c_int32, [_PATH, _POT, _TUNE, c_uint64, c_double, c_void_p, c_void_p,
                                     c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                     c_void_p, c_size_t, c_void_p]),
    "pamd_em_workspace_size": (c_int32, [_PATH, _POT, _TUNE, POINTER(c_size_t)]),
    "pamd_em_integrate": (c_int32, [_PATH, _POT, _TUNE, c_void_p, c_void_p, c_void_p, c_void_p,
                                    c_size_t, c_void_p]),
    "pamd_autotune": (c_int32, [_PATH, _POT, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p,
                                _TUNE]),
    "pamd_profile_events": (c_int32, [c_void_p, c_void_p]),
    "pamd_graph_begin": (c_int32, [c_void_p]),
    "pamd_graph_end": (c_int32, [c_void_p, POINTER(c_void_p)]),
    "pamd_graph_launch": (c_int32, [c_void_p, c_void_p]),
    "pamd_graph_destroy": (None, [c_void_p]),
}

EXPORTED = tuple(_SIGNATURES)

_lib = None


def load(path: str = LIB_PATH):
    """Loads libpamd.so once; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libpamd.so not found at {path}; build it with "
                          "`python -m paper_1907_09529_amd.build_lib` or __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(code: int, func: str) -> None:
    if code != PAMD_OK:
        msg = load().pamd_last_error()
        raise PamdError(code, func, msg.decode() if msg else "")


def call(name: str, *args) -> int:
    """Calls a C entry point and raises PamdError on a nonzero return."""
    fn = getattr(load(), name)
    code = fn(*args)
    check(code, name)
    return code
