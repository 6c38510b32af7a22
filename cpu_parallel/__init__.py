"""Multi-threaded CPU merge of one column (Section 6.2's parallel scheme on
the host's cores): a measurement baseline beside the GPU library, in its own
shared library (``libcolmerge_cpu.so``, built from ``colmerge_cpu.cpp`` with
g++ and std::thread).  It shares no code with the GPU library or the oracle.

Values and packed codes use the numpy conventions of ``workloads.gen``:
``"u32"`` / ``"u64"`` 1-D arrays, ``"str16"`` (n, 16) uint8, codes as uint64
words.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "colmerge_cpu.cpp")
_LIB_PATH = os.path.join(_HERE, "libcolmerge_cpu.so")

TYPES = {"u32": 0, "u64": 1, "str16": 2}
DTYPES = {"u32": np.uint32, "u64": np.uint64}


class CpuMergeError(RuntimeError):
    pass


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["g++", "-O3", "-std=c++17", "-fPIC", "-shared", "-pthread", "-Wall", "-o", tmp,
               _SRC]
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise CpuMergeError(f"g++ failed:\n{res.stdout}{res.stderr}")
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        p, u64, u32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32
        lib.cmp_merge_column.restype = ctypes.c_int
        lib.cmp_merge_column.argtypes = [ctypes.c_int, p, u64, p, u64, u32, p, u64, ctypes.c_int,
                                         p, p, p, p, ctypes.POINTER(u64), ctypes.POINTER(u32),
                                         ctypes.POINTER(u64)]
        _lib = lib
    return _lib


def _arr(vtype, a, n):
    if vtype == "str16":
        return np.ascontiguousarray(a, dtype=np.uint8).reshape(n, 16)
    return np.ascontiguousarray(a, dtype=DTYPES[vtype]).reshape(n)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a.size else None


def alloc_outputs(vtype: str, n_um: int, n_main: int, nd: int) -> dict:
    """Output buffers for a merge of these sizes (reusable across calls, so a
    timed call does not pay for fresh pages)."""
    shape = (n_um + nd, 16) if vtype == "str16" else (n_um + nd,)
    rows = n_main + nd
    return {"u_new": np.zeros(shape, dtype=np.uint8 if vtype == "str16" else DTYPES[vtype]),
            "out": np.zeros(max(1, (rows * 32 + 63) // 64), dtype=np.uint64),
            "x_m": np.zeros(max(1, n_um), dtype=np.uint32),
            "x_d": np.zeros(max(1, nd), dtype=np.uint32),
            "sizes": (vtype, n_um, n_main, nd)}


def merge_column(vtype: str, u_m, main_packed, n_main: int, w: int, delta, threads: int,
                 outputs: dict | None = None) -> dict:
    """The merged column: dict with u_new, codes (uint64 words), w_new, n_new,
    n_words, x_m, x_d (|U_D| entries), views into `outputs` (from
    alloc_outputs with the same sizes) when given."""
    lib = _load()
    n_um = int(len(u_m))
    nd = int(len(delta))
    u_m = _arr(vtype, u_m, n_um)
    delta = _arr(vtype, delta, nd)
    codes = np.ascontiguousarray(main_packed, dtype=np.uint64)
    if outputs is None:
        outputs = alloc_outputs(vtype, n_um, n_main, nd)
    elif outputs["sizes"] != (vtype, n_um, n_main, nd):
        raise CpuMergeError(f"outputs sized for {outputs['sizes']}, not {(vtype, n_um, n_main, nd)}")
    u_new, out, x_m, x_d = outputs["u_new"], outputs["out"], outputs["x_m"], outputs["x_d"]
    rows = n_main + nd
    n_new, w_new, n_ud = ctypes.c_uint64(), ctypes.c_uint32(), ctypes.c_uint64()
    rc = lib.cmp_merge_column(TYPES[vtype], _ptr(u_m), n_um, _ptr(codes), n_main, w,
                              _ptr(delta), nd, threads, _ptr(u_new), _ptr(out), _ptr(x_m),
                              _ptr(x_d), ctypes.byref(n_new), ctypes.byref(w_new),
                              ctypes.byref(n_ud))
    if rc != 0:
        raise CpuMergeError(f"cmp_merge_column returned {rc}")
    nn, wn = int(n_new.value), int(w_new.value)
    nw = (rows * wn + 63) // 64
    return {"u_new": u_new[:nn], "codes": out[:nw], "w_new": wn, "n_new": nn, "n_words": nw,
            "x_m": x_m[:n_um], "x_d": x_d[:int(n_ud.value)]}
