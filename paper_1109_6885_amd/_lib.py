"""ctypes declarations for libcolmerge.so (the C ABI of include/colmerge.h).

Only argument marshalling lives here; every step of the merge runs in the
library's HIP kernels.  Loading fails loudly if the library is not built:
there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcolmerge.so")

MC_U32, MC_U64, MC_STR16 = 0, 1, 2
TYPE_CODES = {"u32": MC_U32, "u64": MC_U64, "str16": MC_STR16}
VALUE_LEN = {"u32": 4, "u64": 8, "str16": 16}

STATUS = {0: "MC_OK", -1: "MC_E_ARG", -2: "MC_E_CAP", -3: "MC_E_NOMEM", -4: "MC_E_HIP",
          -5: "MC_E_DATA"}

MC_DEVERR_CODE_RANGE = 1
MC_DEVERR_DELTA_RANGE = 2
MC_DEVERR_SPIN = 4
MC_DEVERR_ORDER = 8

EXPORTS = [
    "mc_ctx_create", "mc_ctx_destroy", "mc_last_error", "mc_merge_bounds", "mc_merge_column",
    "mc_delta_dictionary", "mc_delta_dictionary_scratch", "mc_merge_dictionaries",
    "mc_merge_dictionaries_scratch", "mc_reencode", "mc_merge_batched_bounds",
    "mc_merge_columns_batched", "mc_graph_launch", "mc_graph_destroy", "mc_ctx_set_timing",
    "mc_ctx_step_times", "mc_copy_bytes", "mc_gather_ref", "mc_merge_column_naive",
    "mc_ctx_set_tuning", "mc_ctx_get_tuning", "mc_autotune_batched", "mc_merge_bounds_ctx",
    "mc_delta_index_bytes", "mc_delta_index_reset", "mc_delta_index_append",
    "mc_merge_indexed_bounds", "mc_merge_column_indexed", "mc_merge_batched_bounds_ctx",
    "mc_merge_column_noalloc", "mc_ctx_set_validate", "mc_tune_class", "mc_ctx_set_class_tuning",
    "mc_ctx_get_class_tuning", "mc_autotune_batched_classes",
]

# Tuning classes of the batched merge (MC_TUNE_CLASSES in colmerge.h).
TUNE_CLASSES = 36

# Entries of mc_ctx_step_times (MC_STEP_TIMES in colmerge.h).
STEP_TIMES = 6

# Workspace of mc_merge_column_noalloc (MC_NOALLOC_SCRATCH_BYTES in colmerge.h).
NOALLOC_SCRATCH_BYTES = 64 << 20


class McResult(ctypes.Structure):
    _fields_ = [("new_dict_len", ctypes.c_uint64), ("new_codes_words", ctypes.c_uint64),
                ("delta_dict_len", ctypes.c_uint64), ("new_bitwidth", ctypes.c_uint32),
                ("error", ctypes.c_uint32)]


class McColumnIn(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int32), ("bitwidth", ctypes.c_uint32),
                ("main_dict", ctypes.c_void_p), ("main_dict_len", ctypes.c_uint64),
                ("main_codes", ctypes.c_void_p), ("main_rows", ctypes.c_uint64),
                ("delta_values", ctypes.c_void_p), ("delta_rows", ctypes.c_uint64)]


class McColumnOut(ctypes.Structure):
    _fields_ = [("new_dict", ctypes.c_void_p), ("new_dict_cap", ctypes.c_uint64),
                ("new_codes", ctypes.c_void_p), ("new_codes_cap_words", ctypes.c_uint64),
                ("x_main", ctypes.c_void_p), ("x_delta", ctypes.c_void_p),
                ("result", ctypes.c_void_p)]


MC_BATCHED_PHASES, MC_BATCHED_PERSISTENT = 0, 1


class McTuning(ctypes.Structure):
    _fields_ = [("repack_codes", ctypes.c_uint32), ("prefix_run", ctypes.c_uint32),
                ("hash_min_rows", ctypes.c_uint32), ("batched_launch", ctypes.c_uint32),
                ("persist_workers", ctypes.c_uint32), ("persist_repack", ctypes.c_uint32),
                ("persist_merge", ctypes.c_uint32), ("hash_dict_ratio", ctypes.c_uint32)]


class McDeltaIndex(ctypes.Structure):
    _fields_ = [("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_uint64),
                ("capacity", ctypes.c_uint64), ("type", ctypes.c_int32),
                ("reserved", ctypes.c_uint32)]


class ColmergeError(RuntimeError):
    def __init__(self, code, what, msg):
        super().__init__(f"{what}: {STATUS.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load():
    """Load libcolmerge.so and declare its signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                           "(the merge has no path other than the HIP library)")
    lib = ctypes.CDLL(LIB_PATH)
    p, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32
    pu64 = ctypes.POINTER(ctypes.c_uint64)
    pin, pout = ctypes.POINTER(McColumnIn), ctypes.POINTER(McColumnOut)
    sig = {
        "mc_ctx_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(p)]),
        "mc_ctx_destroy": (None, [p]),
        "mc_last_error": (ctypes.c_char_p, []),
        "mc_merge_bounds": (ctypes.c_int, [pin, pu64, pu64, pu64]),
        "mc_merge_bounds_ctx": (ctypes.c_int, [p, pin, pu64, pu64, pu64]),
        "mc_delta_index_bytes": (ctypes.c_int, [i32, u64, pu64]),
        "mc_delta_index_reset": (ctypes.c_int, [p, ctypes.POINTER(McDeltaIndex), p]),
        "mc_delta_index_append": (ctypes.c_int, [p, ctypes.POINTER(McDeltaIndex), p, u64, u64, p]),
        "mc_merge_indexed_bounds": (ctypes.c_int, [pin, pu64]),
        "mc_merge_column_indexed": (ctypes.c_int, [p, pin, ctypes.POINTER(McDeltaIndex), pout, p,
                                                   u64, p]),
        "mc_merge_column": (ctypes.c_int, [p, pin, pout, p, u64, p]),
        "mc_merge_column_naive": (ctypes.c_int, [p, pin, pout, p, u64, p]),
        "mc_merge_column_noalloc": (ctypes.c_int, [p, pin, pout, p]),
        "mc_delta_dictionary": (ctypes.c_int, [p, i32, p, u64, p, p, p, p, u64, p]),
        "mc_delta_dictionary_scratch": (ctypes.c_int, [i32, u64, pu64]),
        "mc_merge_dictionaries": (ctypes.c_int, [p, i32, p, u64, p, p, u64, p, p, p, u64, p, p,
                                                 u64, p]),
        "mc_merge_dictionaries_scratch": (ctypes.c_int, [u64, u64, pu64]),
        "mc_reencode": (ctypes.c_int, [p, p, u64, u32, p, u64, p, u64, p, p, p, u64, p]),
        "mc_merge_batched_bounds": (ctypes.c_int, [pin, u32, pu64]),
        "mc_merge_batched_bounds_ctx": (ctypes.c_int, [p, pin, u32, pu64]),
        "mc_merge_columns_batched": (ctypes.c_int, [p, pin, pout, u32, p, u64, p,
                                                    ctypes.POINTER(p)]),
        "mc_graph_launch": (ctypes.c_int, [p, p]),
        "mc_graph_destroy": (None, [p]),
        "mc_ctx_set_timing": (ctypes.c_int, [p, ctypes.c_int]),
        "mc_ctx_step_times": (ctypes.c_int, [p, ctypes.POINTER(ctypes.c_float), u32]),
        "mc_ctx_set_validate": (ctypes.c_int, [p, ctypes.c_int]),
        "mc_copy_bytes": (ctypes.c_int, [p, p, p, u64, p]),
        "mc_gather_ref": (ctypes.c_int, [p, p, u64, p, u32, u32, p, p]),
        "mc_ctx_set_tuning": (ctypes.c_int, [p, ctypes.POINTER(McTuning)]),
        "mc_ctx_get_tuning": (ctypes.c_int, [p, ctypes.POINTER(McTuning)]),
        "mc_autotune_batched": (ctypes.c_int, [p, pin, pout, u32, p, u64, p,
                                               ctypes.POINTER(McTuning),
                                               ctypes.POINTER(ctypes.c_float)]),
        "mc_tune_class": (ctypes.c_int, [pin, ctypes.POINTER(u32)]),
        "mc_ctx_set_class_tuning": (ctypes.c_int, [p, u32, ctypes.POINTER(McTuning)]),
        "mc_ctx_get_class_tuning": (ctypes.c_int, [p, u32, ctypes.POINTER(McTuning),
                                                   ctypes.POINTER(ctypes.c_int)]),
        "mc_autotune_batched_classes": (ctypes.c_int, [p, pin, pout, u32, p, u64, p,
                                                       ctypes.POINTER(u32)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def check(rc, what):
    if rc != 0:
        msg = load().mc_last_error()
        raise ColmergeError(rc, what, msg.decode() if msg else "")
