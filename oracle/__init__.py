"""Serial CPU oracle for the online column merge (arXiv 1109.6885, Section 5).

TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the
benchmark's CPU-baseline leg are the only callers.  The GPU library never
imports this package and shares no code with it.

This module is a thin ctypes wrapper over ``libcolmerge_oracle.so`` (plain C,
``colmerge_oracle.c``).  Values are numpy arrays:

* ``"u32"``   -> 1-D ``uint32``
* ``"u64"``   -> 1-D ``uint64``
* ``"str16"`` -> 2-D ``uint8`` of shape (n, 16), compared as unsigned bytes

Packed codes are 1-D ``uint64`` word arrays (code i at stream bits
[i*w, (i+1)*w), least significant bit first).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "colmerge_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libcolmerge_oracle.so")

TYPES = {"u32": 0, "u64": 1, "str16": 2}
VALUE_LEN = {"u32": 4, "u64": 8, "str16": 16}


class OracleError(RuntimeError):
    pass


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (one C file, no dependencies)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra",
                               "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB_PATH)
        u64, u32, p = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p
        pu64 = ctypes.POINTER(ctypes.c_uint64)
        pu32 = ctypes.POINTER(ctypes.c_uint32)
        lib.cmo_width.argtypes = [u64]
        lib.cmo_width.restype = u32
        lib.cmo_words.argtypes = [u64, u32]
        lib.cmo_words.restype = u64
        lib.cmo_unpack.argtypes = [p, u64, u32]
        lib.cmo_unpack.restype = u32
        lib.cmo_pack.argtypes = [p, u64, u32, u32]
        lib.cmo_pack.restype = None
        lib.cmo_delta_dictionary.argtypes = [ctypes.c_int, p, u64, p, p, pu64]
        lib.cmo_merge_dictionaries.argtypes = [ctypes.c_int, p, u64, p, u64, p,
                                               p, p, pu64]
        lib.cmo_reencode.argtypes = [p, u64, u32, p, u64, p, u64, p, u64, u32, p]
        lib.cmo_reencode_naive.argtypes = [ctypes.c_int, p, u64, p, u64, u32, p,
                                           u64, p, u64, u32, p]
        lib.cmo_merge_column.argtypes = [ctypes.c_int, p, u64, p, u64, u32, p,
                                         u64, p, p, p, p, p, p, pu64, pu32, pu64,
                                         pu64]
        for f in ("cmo_delta_dictionary", "cmo_merge_dictionaries",
                  "cmo_reencode", "cmo_reencode_naive", "cmo_merge_column"):
            getattr(lib, f).restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    if a is None or a.size == 0:
        return None
    return ctypes.c_void_p(a.ctypes.data)


def _nvals(values, vtype):
    return 0 if values is None else (values.shape[0])


def _check(rc, what):
    if rc != 0:
        raise OracleError(f"{what} failed with code {rc}")


def _contig(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _vals(values, vtype):
    if vtype == "u32":
        return _contig(values, np.uint32).reshape(-1)
    if vtype == "u64":
        return _contig(values, np.uint64).reshape(-1)
    return _contig(values, np.uint8).reshape(-1, 16)


def _empty_vals(n, vtype):
    if vtype == "u32":
        return np.zeros(n, np.uint32)
    if vtype == "u64":
        return np.zeros(n, np.uint64)
    return np.zeros((n, 16), np.uint8)


def width(n: int) -> int:
    """Eq. 4 with the one-bit floor for n <= 1."""
    return int(_load().cmo_width(n))


def words(n: int, w: int) -> int:
    return int(_load().cmo_words(n, w))


def unpack(packed: np.ndarray, i: int, w: int) -> int:
    packed = _contig(packed, np.uint64)
    return int(_load().cmo_unpack(_ptr(packed), i, w))


def pack_codes(codes, w: int) -> np.ndarray:
    """Pack a code sequence bit by bit with the oracle's packer."""
    codes = np.asarray(codes, dtype=np.uint64).reshape(-1)
    out = np.zeros(max(words(len(codes), w), 0), np.uint64)
    lib = _load()
    for i, c in enumerate(codes):
        lib.cmo_pack(_ptr(out), i, w, int(c))
    return out


def unpack_codes(packed, n: int, w: int) -> np.ndarray:
    packed = _contig(packed, np.uint64)
    lib = _load()
    return np.array([lib.cmo_unpack(_ptr(packed), i, w) for i in range(n)],
                    dtype=np.uint32)


def delta_dictionary(vtype: str, delta):
    """Step 1(a): (U_D, drank)."""
    delta = _vals(delta, vtype)
    n = delta.shape[0]
    u_d = _empty_vals(n, vtype)
    drank = np.zeros(n, np.uint32)
    n_ud = ctypes.c_uint64(0)
    rc = _load().cmo_delta_dictionary(TYPES[vtype], _ptr(delta), n, _ptr(u_d),
                                      _ptr(drank), ctypes.byref(n_ud))
    _check(rc, "cmo_delta_dictionary")
    return u_d[: n_ud.value].copy(), drank


def merge_dictionaries(vtype: str, u_m, u_d):
    """Step 1(b): (U', X_M, X_D)."""
    u_m = _vals(u_m, vtype)
    u_d = _vals(u_d, vtype)
    a, b = u_m.shape[0], u_d.shape[0]
    u_new = _empty_vals(a + b, vtype)
    x_m = np.zeros(a, np.uint32)
    x_d = np.zeros(b, np.uint32)
    n = ctypes.c_uint64(0)
    rc = _load().cmo_merge_dictionaries(TYPES[vtype], _ptr(u_m), a, _ptr(u_d), b,
                                        _ptr(u_new), _ptr(x_m), _ptr(x_d),
                                        ctypes.byref(n))
    _check(rc, "cmo_merge_dictionaries")
    return u_new[: n.value].copy(), x_m, x_d


def reencode(main_codes, n_main, w, x_m, drank, x_d, w_new):
    """Step 2(b) through the translation tables (Eq. 11)."""
    main_codes = _contig(main_codes, np.uint64)
    x_m = _contig(x_m, np.uint32)
    x_d = _contig(x_d, np.uint32)
    drank = _contig(drank, np.uint32)
    n_delta = drank.shape[0]
    out = np.zeros(max(words(n_main + n_delta, w_new), 1), np.uint64)
    rc = _load().cmo_reencode(_ptr(main_codes), n_main, w, _ptr(x_m),
                              x_m.shape[0], _ptr(drank), n_delta, _ptr(x_d),
                              x_d.shape[0], w_new, _ptr(out))
    _check(rc, "cmo_reencode")
    return out[: words(n_main + n_delta, w_new)]


def reencode_naive(vtype, u_m, main_codes, n_main, w, delta, u_new, w_new):
    """Step 2(b) the naive way (Section 5.2): decode, then binary search."""
    u_m = _vals(u_m, vtype)
    delta = _vals(delta, vtype)
    u_new = _vals(u_new, vtype)
    main_codes = _contig(main_codes, np.uint64)
    n_delta = delta.shape[0]
    out = np.zeros(max(words(n_main + n_delta, w_new), 1), np.uint64)
    rc = _load().cmo_reencode_naive(TYPES[vtype], _ptr(u_m), u_m.shape[0],
                                    _ptr(main_codes), n_main, w, _ptr(delta),
                                    n_delta, _ptr(u_new), u_new.shape[0], w_new,
                                    _ptr(out))
    _check(rc, "cmo_reencode_naive")
    return out[: words(n_main + n_delta, w_new)]


def merge_column(vtype: str, u_m, main_codes, n_main: int, w: int, delta):
    """The whole merge of one column.  Returns a dict with keys
    u_new, codes (W' words), w_new, n_new, n_words, x_m, x_d, u_d, drank."""
    u_m = _vals(u_m, vtype)
    delta = _vals(delta, vtype)
    main_codes = _contig(main_codes, np.uint64)
    a, nd = u_m.shape[0], delta.shape[0]
    u_new = _empty_vals(a + nd, vtype)
    codes = np.zeros(max(words(n_main + nd, 32), 1), np.uint64)
    x_m = np.zeros(a, np.uint32)
    x_d = np.zeros(nd, np.uint32)
    u_d = _empty_vals(nd, vtype)
    drank = np.zeros(nd, np.uint32)
    n_new = ctypes.c_uint64(0)
    w_new = ctypes.c_uint32(0)
    n_ud = ctypes.c_uint64(0)
    n_words = ctypes.c_uint64(0)
    rc = _load().cmo_merge_column(
        TYPES[vtype], _ptr(u_m), a, _ptr(main_codes), n_main, w, _ptr(delta), nd,
        _ptr(u_new), _ptr(codes), _ptr(x_m), _ptr(x_d), _ptr(u_d), _ptr(drank),
        ctypes.byref(n_new), ctypes.byref(w_new), ctypes.byref(n_ud),
        ctypes.byref(n_words))
    _check(rc, "cmo_merge_column")
    return {
        "u_new": u_new[: n_new.value].copy(),
        "codes": codes[: n_words.value].copy(),
        "w_new": int(w_new.value),
        "n_new": int(n_new.value),
        "n_words": int(n_words.value),
        "x_m": x_m,
        "x_d": x_d[: n_ud.value].copy(),
        "u_d": u_d[: n_ud.value].copy(),
        "drank": drank,
    }
