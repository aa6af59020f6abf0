"""ctypes view of libbeagle.so (the C ABI declared in include/beagle.h).

Loading fails loudly when the library has not been built: there is no
fallback implementation of any entry point.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_float, c_int, c_int8, c_int32, c_int64, c_size_t, c_uint32, \
    c_uint64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
# BEAGLE_LIBRARY selects another build of the same library (e.g. a variant
# with different tile parameters)
LIB_PATH = os.environ.get("BEAGLE_LIBRARY") or os.path.join(HERE, "libbeagle.so")

# return codes
OK = 0
E_INVALID_ARG = -1
E_HIP = -2
E_NOMEM = -3
E_UNSUPPORTED = -4

FIT_MSE = 0
FIT_CORR = 1
FIT_POINT = 2
FIT_R4 = 3
DECODE_WAVE = 0
DECODE_THREAD = 1
TUNE_AUTO = 0
TUNE_WIDE = 1
TUNE_NARROW = 2

# per-program status codes
PROG_STATUS = {0: "ok", 1: "empty", 2: "bad_opcode", 3: "underflow", 4: "bad_final_depth",
               5: "bad_var", 6: "bad_const", 7: "too_long", 8: "bad_layout"}


class Programs(ctypes.Structure):
    _fields_ = [("tokens", c_void_p), ("n_tokens", c_int64), ("tok_offset", c_void_p),
                ("tok_len", c_void_p), ("consts", c_void_p), ("n_consts", c_int64),
                ("const_offset", c_void_p), ("const_count", c_void_p), ("n_programs", c_int32)]


class Dataset(ctypes.Structure):
    _fields_ = [("X", c_void_p), ("y", c_void_p), ("M", c_int64), ("D", c_int32)]


class GenParams(ctypes.Structure):
    _fields_ = [("tournament", c_int32), ("p_crossover", c_float), ("p_mutation", c_float),
                ("max_len", c_int32), ("max_consts", c_int32), ("const_lo", c_float), ("const_hi", c_float),
                ("init_depth_min", c_int32), ("init_depth_max", c_int32), ("op_set", c_int32)]


# (name, restype, argtypes) of every exported entry point
SIGNATURES = [
    ("beagle_abi_version", c_int, []),
    ("beagle_last_error", c_char_p, []),
    ("beagle_ctx_create", c_int, [POINTER(c_void_p), c_int, c_size_t]),
    ("beagle_ctx_destroy", None, [c_void_p]),
    ("beagle_ctx_enable_timing", c_int, [c_void_p, c_int]),
    ("beagle_ctx_kernel_time", c_int, [c_void_p, POINTER(c_double), POINTER(c_int64)]),
    ("beagle_ctx_set_tuning", c_int, [c_void_p, c_int]),
    ("beagle_ctx_set_decoder", c_int, [c_void_p, c_int]),
    ("beagle_ctx_graph_stats", c_int, [c_void_p, POINTER(c_int64), POINTER(c_int64)]),
    ("beagle_ctx_tile_width", c_int, [c_void_p, c_int, c_int32, c_int64, c_int64, c_int32, POINTER(c_int32)]),
    ("beagle_eval", c_int, [c_void_p, POINTER(Programs), POINTER(Dataset), c_int, c_void_p, c_void_p, c_void_p]),
    ("beagle_eval_static", c_int, [POINTER(Programs), POINTER(Dataset), c_int, c_void_p, c_void_p, c_void_p]),
    ("beagle_eval_batched", c_int, [c_void_p, POINTER(Programs), POINTER(Dataset), c_int32, c_int,
                                    POINTER(c_void_p), POINTER(c_void_p), c_void_p]),
    ("beagle_eval_workspace_size", c_int, [POINTER(Programs), POINTER(Dataset), c_int, POINTER(c_size_t)]),
    ("beagle_eval_score", c_int, [c_void_p, POINTER(Programs), POINTER(Dataset), c_int, c_double, c_void_p,
                                  c_void_p, c_void_p]),
    ("beagle_predict", c_int, [c_void_p, POINTER(Programs), POINTER(Dataset), c_void_p, c_void_p, c_void_p]),
    ("beagle_eval_grad", c_int, [c_void_p, POINTER(Programs), POINTER(Dataset), c_int, c_void_p, c_void_p,
                                 c_void_p, c_void_p]),
    ("beagle_init_population", c_int, [c_void_p, POINTER(GenParams), c_int32, c_int32, c_uint64, c_uint32,
                                       c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    ("beagle_generation", c_int, [c_void_p, POINTER(Programs), c_void_p, POINTER(GenParams), c_int32, c_uint64,
                                  c_uint64, c_uint32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    ("beagle_generation_microcosm", c_int, [c_void_p, POINTER(Programs), c_void_p, POINTER(GenParams), c_int32,
                                            c_int32, c_float, c_uint64, c_uint64, c_uint32, c_int32, c_void_p,
                                            c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
]

_lib = None
HEADER = os.path.join(os.path.dirname(HERE), "include", "beagle.h")
# the layout of the structures above (beagle_gen_params grew op_set in 2)
ABI_VERSION = 2


def load():
    """The loaded library (raises ImportError when it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2603_12292_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name, None)
        if fn is None:
            raise ImportError(f"{LIB_PATH} does not export {name}: rebuild it")
        fn.restype = res
        fn.argtypes = args
    if lib.beagle_abi_version() != ABI_VERSION:
        raise ImportError(f"{LIB_PATH} has ABI version {lib.beagle_abi_version()}, these bindings {ABI_VERSION}: "
                          "rebuild it")
    _lib = lib
    return lib


def declared_symbols():
    """Names of the functions include/beagle.h declares (parsed from the header)."""
    import re
    with open(HEADER) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(beagle_[a-z_]+)\s*\(", text)))
