"""ctypes binding of the C ABI in include/flare.h (argument marshalling only).

Device buffers are torch tensors; their data_ptr() and torch's current HIP stream are
passed straight through. torch is imported before the library is loaded so that both
resolve the same HIP runtime (the loader matches libamdhip64 by its soname).
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime the library will share)

LIB_NAME = "libflare_mi355x.so"
LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), LIB_NAME)

OK, E_ARG, E_SPECIES, E_BOX, E_CAPACITY, E_NONFINITE, E_STALE, E_OOM, E_HIP, E_UNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6, -7, -8, -9
FP32, BF16_SPLIT, FP8_SPLIT, BF16X6_SPLIT = 0, 1, 2, 3
VAR_FP32 = 16          # with a split form: the variance through the FP32 factor
FLAG_NONFINITE, FLAG_SPECIES, FLAG_DISPLACED, FLAG_UNCERTAIN = 1, 2, 4, 8


class FlareError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(msg)
        self.code = code


_p = ctypes.c_void_p
_i = ctypes.c_int
_d = ctypes.c_double
_ll = ctypes.c_longlong

# name -> (restype, argtypes); the same names as include/flare.h
SIGNATURES = {
    "flare_last_error": (ctypes.c_char_p, []),
    "flare_strerror": (ctypes.c_char_p, [_i]),
    "flare_model_create": (_i, [ctypes.POINTER(_p), _i, _i, _i, _d, _p, _p, _i]),
    "flare_model_from_sparse_set": (_i, [ctypes.POINTER(_p), _i, _i, _i, _d, _p, _p, _p, _d, _d, _i, _p, _p]),
    "flare_model_destroy": (_i, [_p]),
    "flare_descriptor_dim": (_i, [_p, ctypes.POINTER(_i)]),
    "flare_state_create": (_i, [ctypes.POINTER(_p), _p, _i, _ll, _p]),
    "flare_state_destroy": (_i, [_p]),
    "flare_neighbors": (_i, [_p, _i, _p, _p, _p, _p, _i, _p, _p, _d]),
    "flare_list_info": (_i, [_p, ctypes.POINTER(_ll), _p]),
    "flare_neighbors_export": (_i, [_p, _p, _p, _p]),
    "flare_descriptors": (_i, [_p, _p, _p, _p, _p, _p]),
    "flare_energy_forces": (_i, [_p, _p, _p, _p, _p, _p, _p, _p]),
    "flare_forces": (_i, [_p, _p, _p, _p, _p]),
    "flare_virial": (_i, [_p, _p]),
    "flare_virial_noalloc": (_i, [_p, _p]),
    "flare_model_info": (_i, [_p, ctypes.POINTER(_i), ctypes.POINTER(_i)]),
    "flare_variance": (_i, [_p, _p, _p, _p]),
    "flare_quadratic_forms": (_i, [_p, _i, _i, _p, _p, _p]),
    "flare_memory_bytes": (_i, [_p, _p, ctypes.POINTER(_ll)]),
    "flare_md_first_half": (_i, [_p, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p, _d]),
    "flare_md_second_half": (_i, [_p, _p, _p, _p, _p, _p, _p, _p, _p, _d]),
    "flare_md_step": (_i, [_p, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p, _d, _i, _p, _p, _p, _p]),
    "flare_nvt_first_half": (_i, [_p, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p, _d, _d, _d, _p]),
    "flare_nvt_second_half": (_i, [_p, _p, _p, _p, _p, _p, _p, _p, _p, _d, _d, _d, _p]),
    "flare_kinetic": (_i, [_p, _p, _p, _p, _p, _p, _p]),
    "flare_coordination": (_i, [_p, _p, _p, _p, _p, _p, _p]),
    "flare_timers_enable": (_i, [_p, _i]),
    "flare_timers_read": (_i, [_p, _p, _p, _i]),
    "flare_status": (_i, [_p, _p]),
    "flare_interval_status": (_i, [_p, _p]),
    "flare_uncertainty_monitor": (_i, [_p, _d, _p, _p]),
}

TIMER_NAMES = ["list", "desc144", "desc544", "qform144", "qform544", "force144", "force544",
               "outputs", "md"]

_LIB = None


def load():
    """Load the built library (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise FlareError(E_ARG, f"{LIB_NAME} is not built; run `python -m paper_2204_12573_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib
    return _LIB


def check(rc):
    if rc != OK:
        lib = load()
        raise FlareError(rc, f"{lib.flare_strerror(rc).decode()}: {lib.flare_last_error().decode()}")


def ptr(t):
    """Device (or host) address of a tensor / numpy array, or None."""
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        return t.data_ptr()
    return t.ctypes.data


def stream_handle(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream
