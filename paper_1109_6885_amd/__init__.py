"""MI355X column merge: Python binding over libcolmerge.so.

The library implements the online merge of a dictionary-encoded column
(Krueger et al., arXiv 1109.6885, Sections 5 and 6) as HIP kernels for
gfx950 behind the C ABI of include/colmerge.h.  This module only marshals
torch tensors into that ABI; PyTorch provides device memory and streams.

Tensor conventions (all on the GPU):
  values  u32 -> int32 (raw bits), u64 -> int64 (raw bits), str16 -> uint8 (n, 16)
  codes   packed 64-bit words as int64, code i at bits [i*w, (i+1)*w), LSB first
  tables  X_M / X_D as int32 (raw uint32 bits)
"""
from __future__ import annotations

import ctypes
import json
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import (ColmergeError, McColumnIn, McColumnOut, McDeltaIndex, McResult, McTuning,
                   TYPE_CODES, VALUE_LEN, check, load)

__all__ = [
    "Context", "context", "to_device", "value_tensor_empty", "merge_bounds", "merge_column",
    "delta_dictionary", "merge_dictionaries", "reencode", "merge_columns_batched",
    "MergeOutput", "ColumnInput", "ColmergeError", "RESULT_BYTES",
]

RESULT_BYTES = ctypes.sizeof(McResult)  # 32


class Context:
    """An mc_ctx bound to one device."""

    def __init__(self, device: int = 0):
        lib = load()
        h = ctypes.c_void_p()
        check(lib.mc_ctx_create(device, ctypes.byref(h)), "mc_ctx_create")
        self.handle = h
        self.device = device

    def set_timing(self, on: bool):
        check(load().mc_ctx_set_timing(self.handle, int(bool(on))), "mc_ctx_set_timing")

    def step_times(self):
        """Average ms over the timed merges for [delta sort, delta dictionary
        emit, dictionary merge, re-encode, whole, re-encode kernel alone]."""
        arr = (ctypes.c_float * _lib.STEP_TIMES)()
        check(load().mc_ctx_step_times(self.handle, arr, _lib.STEP_TIMES), "mc_ctx_step_times")
        return list(arr)

    def set_validate(self, on: bool):
        """mc_ctx_set_validate: synchronous merges that check U_M's order and
        the main codes' range on the device and raise MC_E_DATA."""
        check(load().mc_ctx_set_validate(self.handle, int(bool(on))), "mc_ctx_set_validate")

    TUNING_FIELDS = ("repack_codes", "prefix_run", "hash_min_rows", "batched_launch",
                     "persist_workers", "persist_repack", "persist_merge", "hash_dict_ratio")

    def set_tuning(self, repack_codes: int = 2048, prefix_run: int = 32, hash_min_rows: int = 0,
                   batched_launch: int = 0, persist_workers: int = 0, persist_repack: int = 0,
                   persist_merge: int = 0, hash_dict_ratio: int = 0):
        """mc_ctx_set_tuning: launch shapes for every later merge on this context
        (batched_launch: 0 one launch per phase, 1 one persistent launch;
        hash_dict_ratio: 0 default 64, 0xFFFFFFFF never)."""
        t = McTuning(repack_codes, prefix_run, hash_min_rows, batched_launch, persist_workers,
                     persist_repack, persist_merge, hash_dict_ratio)
        check(load().mc_ctx_set_tuning(self.handle, ctypes.byref(t)), "mc_ctx_set_tuning")

    def get_tuning(self) -> dict:
        t = McTuning()
        check(load().mc_ctx_get_tuning(self.handle, ctypes.byref(t)), "mc_ctx_get_tuning")
        return {f: getattr(t, f) for f in self.TUNING_FIELDS}

    # ---- per-class shapes of the batched merge (a cache in the context) ----

    CLASS_FIELDS = ("repack_codes", "prefix_run")

    def set_class_tuning(self, cls: int, repack_codes: int | None = None,
                         prefix_run: int | None = None):
        """mc_ctx_set_class_tuning: cache shapes for class `cls`; with both
        shapes None the class's entry is removed."""
        if repack_codes is None and prefix_run is None:
            check(load().mc_ctx_set_class_tuning(self.handle, cls, None),
                  "mc_ctx_set_class_tuning")
            return
        cur = self.get_class_tuning(cls)[0]
        t = McTuning(repack_codes or cur["repack_codes"], prefix_run or cur["prefix_run"])
        check(load().mc_ctx_set_class_tuning(self.handle, cls, ctypes.byref(t)),
              "mc_ctx_set_class_tuning")

    def get_class_tuning(self, cls: int):
        """mc_ctx_get_class_tuning: (shapes a column of class `cls` gets, cached?)."""
        t, is_set = McTuning(), ctypes.c_int()
        check(load().mc_ctx_get_class_tuning(self.handle, cls, ctypes.byref(t),
                                             ctypes.byref(is_set)), "mc_ctx_get_class_tuning")
        return {f: getattr(t, f) for f in self.CLASS_FIELDS}, bool(is_set.value)

    def class_tuning_cache(self) -> dict:
        """The cached classes: {class: {"repack_codes": ..., "prefix_run": ...}}."""
        out = {}
        for c in range(_lib.TUNE_CLASSES):
            shapes, is_set = self.get_class_tuning(c)
            if is_set:
                out[c] = shapes
        return out

    def save_class_tuning(self, path: str):
        """Write the cache as JSON (keys: class numbers)."""
        with open(path, "w") as f:
            json.dump({str(c): v for c, v in self.class_tuning_cache().items()}, f, indent=1)

    def load_class_tuning(self, path: str):
        """Load a cache written by save_class_tuning into this context."""
        with open(path) as f:
            data = json.load(f)
        for c, v in data.items():
            self.set_class_tuning(int(c), int(v["repack_codes"]), int(v["prefix_run"]))

    def __del__(self):
        try:
            if self.handle:
                load().mc_ctx_destroy(self.handle)
        except Exception:
            pass


_ctx = {}


def context(device: int | None = None) -> Context:
    if device is None:
        device = torch.cuda.current_device()
    if device not in _ctx:
        _ctx[device] = Context(device)
    return _ctx[device]


# ---------------------------------------------------------------------------
# Tensor helpers
# ---------------------------------------------------------------------------

_NP_VIEW = {"u32": np.int32, "u64": np.int64}


def to_device(arr: np.ndarray, vtype: str | None = None, device="cuda") -> torch.Tensor:
    """Copy a numpy value/code array to the GPU keeping its bits."""
    a = np.ascontiguousarray(arr)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    elif a.dtype == np.uint64:
        a = a.view(np.int64)
    return torch.from_numpy(a).to(device)


def value_tensor_empty(vtype: str, n: int, device="cuda") -> torch.Tensor:
    if vtype == "u32":
        return torch.empty(n, dtype=torch.int32, device=device)
    if vtype == "u64":
        return torch.empty(n, dtype=torch.int64, device=device)
    return torch.empty((n, 16), dtype=torch.uint8, device=device)


def _ptr(t):
    if t is None:
        return None
    if t.numel() == 0:
        return None
    if not t.is_cuda:
        raise ValueError("tensors passed to the merge library must be on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensors passed to the merge library must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _nvals(t, vtype):
    if t is None:
        return 0
    return int(t.shape[0])


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


# ---------------------------------------------------------------------------
# Whole-column merge
# ---------------------------------------------------------------------------

@dataclass
class ColumnInput:
    """Device inputs of one column merge."""
    vtype: str
    u_m: torch.Tensor
    main_codes: torch.Tensor
    n_main: int
    w: int
    delta: torch.Tensor

    def descriptor(self) -> McColumnIn:
        d = McColumnIn()
        d.type = TYPE_CODES[self.vtype]
        d.bitwidth = self.w
        d.main_dict = _ptr(self.u_m)
        d.main_dict_len = _nvals(self.u_m, self.vtype)
        d.main_codes = _ptr(self.main_codes)
        d.main_rows = self.n_main
        d.delta_values = _ptr(self.delta)
        d.delta_rows = _nvals(self.delta, self.vtype)
        return d

    @classmethod
    def from_numpy(cls, col, device="cuda"):
        """From a workloads.Column (host arrays)."""
        return cls(col.vtype, to_device(col.u_m, device=device),
                   to_device(col.main_packed, device=device), col.n_main, col.w,
                   to_device(col.delta, device=device))


@dataclass
class MergeOutput:
    vtype: str
    new_dict: torch.Tensor     # capacity |U_M| + N_D
    new_codes: torch.Tensor    # capacity from mc_merge_bounds
    x_main: torch.Tensor | None
    x_delta: torch.Tensor | None
    result: torch.Tensor       # 32 bytes of device scalars
    rows: int

    def descriptor(self) -> McColumnOut:
        d = McColumnOut()
        d.new_dict = _ptr(self.new_dict)
        d.new_dict_cap = int(self.new_dict.shape[0])
        d.new_codes = _ptr(self.new_codes)
        d.new_codes_cap_words = int(self.new_codes.shape[0])
        d.x_main = _ptr(self.x_main)
        d.x_delta = _ptr(self.x_delta)
        d.result = _ptr(self.result)
        return d

    def scalars(self) -> dict:
        """Copy the device scalars to the host (synchronizes on them)."""
        r = self.result.cpu().numpy().view(np.uint8)
        res = McResult.from_buffer_copy(r.tobytes())
        return {"n_new": int(res.new_dict_len), "words": int(res.new_codes_words),
                "n_ud": int(res.delta_dict_len), "w_new": int(res.new_bitwidth),
                "error": int(res.error)}

    def fetch(self) -> dict:
        """Host copies of the exact results: U', packed codes, w', tables."""
        s = self.scalars()
        out = dict(s)
        nd = s["n_new"]
        nv = self.new_dict[:nd].cpu().numpy()
        if self.vtype == "u32":
            nv = nv.view(np.uint32)
        elif self.vtype == "u64":
            nv = nv.view(np.uint64)
        out["u_new"] = nv
        out["codes"] = self.new_codes[: s["words"]].cpu().numpy().view(np.uint64)
        if self.x_main is not None:
            out["x_m"] = self.x_main.cpu().numpy().view(np.uint32)
        if self.x_delta is not None:
            out["x_d"] = self.x_delta[: s["n_ud"]].cpu().numpy().view(np.uint32)
        return out


def bounds_of(desc: McColumnIn):
    """mc_merge_bounds on a raw descriptor: (dict_cap, codes_words, scratch_bytes)."""
    a, b, c = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    check(load().mc_merge_bounds(ctypes.byref(desc), ctypes.byref(a), ctypes.byref(b),
                                 ctypes.byref(c)), "mc_merge_bounds")
    return int(a.value), int(b.value), int(c.value)


def batched_bounds_of(descs, ctx: "Context | None" = None) -> int:
    """mc_merge_batched_bounds_ctx on raw descriptors (ctx None: default tuning)."""
    arr = (McColumnIn * len(descs))(*descs)
    sb = ctypes.c_uint64()
    check(load().mc_merge_batched_bounds_ctx(ctx.handle if ctx is not None else None, arr,
                                             len(descs), ctypes.byref(sb)),
          "mc_merge_batched_bounds_ctx")
    return int(sb.value)


def merge_bounds(col: ColumnInput, ctx: Context | None = None):
    """(dict_cap, codes_words, scratch_bytes) for one column (host only);
    with ctx, for merges on that context (mc_merge_bounds_ctx)."""
    d = col.descriptor()
    a, b, c = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    check(load().mc_merge_bounds_ctx(ctx.handle if ctx is not None else None, ctypes.byref(d),
                                     ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
          "mc_merge_bounds_ctx")
    return int(a.value), int(b.value), int(c.value)


def alloc_output(col: ColumnInput, tables: bool = False, device="cuda") -> MergeOutput:
    dict_cap, words, _ = merge_bounds(col)
    n_delta = _nvals(col.delta, col.vtype)
    return MergeOutput(
        col.vtype,
        value_tensor_empty(col.vtype, dict_cap, device),
        torch.empty(max(words, 2), dtype=torch.int64, device=device),
        torch.empty(_nvals(col.u_m, col.vtype), dtype=torch.int32, device=device) if tables else None,
        torch.empty(n_delta, dtype=torch.int32, device=device) if tables else None,
        torch.zeros(RESULT_BYTES, dtype=torch.uint8, device=device),
        col.n_main + n_delta,
    )


def alloc_scratch(nbytes: int, device="cuda") -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def merge_column(col: ColumnInput, out: MergeOutput | None = None,
                 scratch: torch.Tensor | None = None, tables: bool = False,
                 stream=None, ctx: Context | None = None) -> MergeOutput:
    """mc_merge_column: enqueue the whole merge of one column."""
    ctx = ctx or context()
    if out is None:
        out = alloc_output(col, tables)
    if scratch is None:
        scratch = alloc_scratch(merge_bounds(col, ctx)[2])
    din, dout = col.descriptor(), out.descriptor()
    check(load().mc_merge_column(ctx.handle, ctypes.byref(din), ctypes.byref(dout),
                                 _ptr(scratch), scratch.numel(), _stream(stream)),
          "mc_merge_column")
    return out


def merge_column_noalloc(col: ColumnInput, out: MergeOutput, stream=None,
                         ctx: Context | None = None) -> MergeOutput:
    """mc_merge_column_noalloc: the merge of one column with the library's
    own per-device workspace (no allocation in the call; `out` must be
    allocated beforehand)."""
    ctx = ctx or context()
    din, dout = col.descriptor(), out.descriptor()
    check(load().mc_merge_column_noalloc(ctx.handle, ctypes.byref(din), ctypes.byref(dout),
                                         _stream(stream)), "mc_merge_column_noalloc")
    return out


def merge_column_naive(col: ColumnInput, out: MergeOutput | None = None,
                       scratch: torch.Tensor | None = None, tables: bool = False,
                       stream=None, ctx: Context | None = None) -> MergeOutput:
    """mc_merge_column_naive: the merge with the unoptimized Step 2(b)."""
    ctx = ctx or context()
    if out is None:
        out = alloc_output(col, tables)
    if scratch is None:
        scratch = alloc_scratch(merge_bounds(col, ctx)[2])
    din, dout = col.descriptor(), out.descriptor()
    check(load().mc_merge_column_naive(ctx.handle, ctypes.byref(din), ctypes.byref(dout),
                                       _ptr(scratch), scratch.numel(), _stream(stream)),
          "mc_merge_column_naive")
    return out


# ---------------------------------------------------------------------------
# Delta index (Step 1(a)'s hashing done as rows are appended)
# ---------------------------------------------------------------------------

class DeltaIndex:
    """An mc_delta_index for a delta buffer of up to `capacity` rows.  The
    caller appends rows to its delta buffer and then calls append(delta, n)
    for them; merge_column_indexed merges the indexed rows."""

    def __init__(self, vtype: str, capacity: int, stream=None, ctx: Context | None = None):
        self.ctx = ctx or context()
        nb = ctypes.c_uint64()
        check(load().mc_delta_index_bytes(TYPE_CODES[vtype], capacity, ctypes.byref(nb)),
              "mc_delta_index_bytes")
        self.workspace = alloc_scratch(nb.value)
        self.desc = McDeltaIndex(_ptr(self.workspace), nb.value, capacity, TYPE_CODES[vtype], 0)
        self.vtype = vtype
        self.capacity = capacity
        self.rows = 0
        self.reset(stream)

    def reset(self, stream=None):
        check(load().mc_delta_index_reset(self.ctx.handle, ctypes.byref(self.desc),
                                          _stream(stream)), "mc_delta_index_reset")
        self.rows = 0

    def append(self, delta: torch.Tensor, rows: int, stream=None):
        """Index the next `rows` rows of `delta` (rows [self.rows, self.rows + rows))."""
        check(load().mc_delta_index_append(self.ctx.handle, ctypes.byref(self.desc), _ptr(delta),
                                           self.rows, rows, _stream(stream)),
              "mc_delta_index_append")
        self.rows += rows


def merge_indexed_bounds(col: ColumnInput) -> int:
    d = col.descriptor()
    sb = ctypes.c_uint64()
    check(load().mc_merge_indexed_bounds(ctypes.byref(d), ctypes.byref(sb)),
          "mc_merge_indexed_bounds")
    return int(sb.value)


def merge_column_indexed(col: ColumnInput, index: DeltaIndex, out: MergeOutput | None = None,
                         scratch: torch.Tensor | None = None, tables: bool = False,
                         stream=None, ctx: Context | None = None) -> MergeOutput:
    """mc_merge_column_indexed: the merge with Step 1(a) starting from the index
    (col.delta holds the indexed rows)."""
    ctx = ctx or context()
    if out is None:
        out = alloc_output(col, tables)
    if scratch is None:
        scratch = alloc_scratch(merge_indexed_bounds(col))
    din, dout = col.descriptor(), out.descriptor()
    check(load().mc_merge_column_indexed(ctx.handle, ctypes.byref(din), ctypes.byref(index.desc),
                                         ctypes.byref(dout), _ptr(scratch), scratch.numel(),
                                         _stream(stream)), "mc_merge_column_indexed")
    return out


# ---------------------------------------------------------------------------
# Single steps
# ---------------------------------------------------------------------------

def delta_dictionary(vtype: str, delta: torch.Tensor, stream=None, ctx=None):
    """mc_delta_dictionary: (u_d capacity tensor, drank int32, count int64[1] device)."""
    ctx = ctx or context()
    n = _nvals(delta, vtype)
    sb = ctypes.c_uint64()
    check(load().mc_delta_dictionary_scratch(TYPE_CODES[vtype], n, ctypes.byref(sb)),
          "mc_delta_dictionary_scratch")
    scratch = alloc_scratch(sb.value)
    u_d = value_tensor_empty(vtype, max(n, 1))
    drank = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    count = torch.zeros(2, dtype=torch.int64, device="cuda")
    check(load().mc_delta_dictionary(ctx.handle, TYPE_CODES[vtype], _ptr(delta), n, _ptr(u_d),
                                     _ptr(drank), _ptr(count), _ptr(scratch), scratch.numel(),
                                     _stream(stream)), "mc_delta_dictionary")
    return u_d, drank[:n], count


def merge_dictionaries(vtype: str, u_m: torch.Tensor, u_d: torch.Tensor, d_count: torch.Tensor,
                       n_ud_max: int, rows_total: int, stream=None, ctx=None):
    """mc_merge_dictionaries: (u_new, x_m, x_d, result)."""
    ctx = ctx or context()
    n_um = _nvals(u_m, vtype)
    sb = ctypes.c_uint64()
    check(load().mc_merge_dictionaries_scratch(n_um, n_ud_max, ctypes.byref(sb)),
          "mc_merge_dictionaries_scratch")
    scratch = alloc_scratch(sb.value)
    u_new = value_tensor_empty(vtype, max(n_um + n_ud_max, 1))
    x_m = torch.empty(max(n_um, 1), dtype=torch.int32, device="cuda")
    x_d = torch.empty(max(n_ud_max, 1), dtype=torch.int32, device="cuda")
    result = torch.zeros(RESULT_BYTES, dtype=torch.uint8, device="cuda")
    check(load().mc_merge_dictionaries(ctx.handle, TYPE_CODES[vtype], _ptr(u_m), n_um, _ptr(u_d),
                                       _ptr(d_count), n_ud_max, _ptr(u_new), _ptr(x_m),
                                       _ptr(x_d), rows_total, _ptr(result), _ptr(scratch),
                                       scratch.numel(), _stream(stream)),
          "mc_merge_dictionaries")
    return u_new, x_m, x_d, result


def reencode(main_codes: torch.Tensor, n_main: int, w: int, x_m: torch.Tensor, n_um: int,
             drank: torch.Tensor, x_d: torch.Tensor, result: torch.Tensor, out: torch.Tensor,
             stream=None, ctx=None):
    """mc_reencode: Step 2(b) into `out` (w' and |U_D| read from `result`)."""
    ctx = ctx or context()
    n_delta = 0 if drank is None else int(drank.shape[0])
    check(load().mc_reencode(ctx.handle, _ptr(main_codes), n_main, w, _ptr(x_m), n_um,
                             _ptr(drank), n_delta, _ptr(x_d), _ptr(result), _ptr(out),
                             int(out.shape[0]), _stream(stream)), "mc_reencode")
    return out


def copy_bytes(src: torch.Tensor, dst: torch.Tensor, nbytes: int | None = None, stream=None,
               ctx=None):
    """mc_copy_bytes: plain 128-bit device copy (bandwidth reference)."""
    ctx = ctx or context()
    n = src.numel() * src.element_size() if nbytes is None else nbytes
    check(load().mc_copy_bytes(ctx.handle, _ptr(src), _ptr(dst), n, _stream(stream)),
          "mc_copy_bytes")


def gather_ref(idx: torch.Tensor, table: torch.Tensor, out: torch.Tensor, stream=None, ctx=None):
    """mc_gather_ref: out[i] = table[idx[i] % len(table)] (random-gather reference)."""
    ctx = ctx or context()
    check(load().mc_gather_ref(ctx.handle, _ptr(idx), idx.numel(), _ptr(table),
                               table.element_size(), table.numel(), _ptr(out), _stream(stream)),
          "mc_gather_ref")


# ---------------------------------------------------------------------------
# Batched
# ---------------------------------------------------------------------------

class Graph:
    def __init__(self, handle, keep):
        self.handle = handle
        self._keep = keep  # descriptors and buffers the graph refers to

    def launch(self, stream=None):
        check(load().mc_graph_launch(self.handle, _stream(stream)), "mc_graph_launch")

    def __del__(self):
        try:
            if self.handle:
                load().mc_graph_destroy(self.handle)
        except Exception:
            pass


def batched_bounds(cols, ctx: "Context | None" = None) -> int:
    """Scratch bytes for one batched merge of these columns on ctx (None:
    default tuning)."""
    return batched_bounds_of([c.descriptor() for c in cols], ctx)


# candidates of mc_autotune_batched, in the order of its times
AUTOTUNE_CANDIDATES = ([{"repack_codes": c, "prefix_run": 32} for c in (1024, 2048, 4096)]
                       + [{"repack_codes": None, "prefix_run": r} for r in (16, 32, 64)])


def autotune_batched(cols, outs=None, scratch=None, stream=None, ctx=None):
    """mc_autotune_batched: time the candidate launch shapes on this batch,
    keep the fastest in the context.  Returns (chosen dict, candidate ms list,
    outs); the outputs hold the batch's merge result."""
    ctx = ctx or context()
    if outs is None:
        outs = [alloc_output(c) for c in cols]
    if scratch is None:
        scratch = alloc_scratch(batched_bounds(cols, ctx))
    ins = (McColumnIn * len(cols))(*[c.descriptor() for c in cols])
    os_ = (McColumnOut * len(cols))(*[o.descriptor() for o in outs])
    t = McTuning()
    times = (ctypes.c_float * 6)()
    check(load().mc_autotune_batched(ctx.handle, ins, os_, len(cols), _ptr(scratch),
                                     scratch.numel(), _stream(stream), ctypes.byref(t), times),
          "mc_autotune_batched")
    return ({f: getattr(t, f) for f in Context.TUNING_FIELDS}, list(times), outs)


def tune_class(col) -> int:
    """mc_tune_class: the tuning class of a column (ColumnInput)."""
    c = ctypes.c_uint32()
    d = col.descriptor()
    check(load().mc_tune_class(ctypes.byref(d), ctypes.byref(c)), "mc_tune_class")
    return c.value


def autotune_batched_classes(cols, outs=None, scratch=None, stream=None, ctx=None):
    """mc_autotune_batched_classes: time the candidate shapes per class of
    this batch and cache the fastest per class in the context.  Returns
    (classes tuned, outs); the outputs hold the batch's merge result."""
    ctx = ctx or context()
    if outs is None:
        outs = [alloc_output(c) for c in cols]
    if scratch is None:
        scratch = alloc_scratch(batched_bounds(cols, ctx))
    ins = (McColumnIn * len(cols))(*[c.descriptor() for c in cols])
    os_ = (McColumnOut * len(cols))(*[o.descriptor() for o in outs])
    n = ctypes.c_uint32()
    check(load().mc_autotune_batched_classes(ctx.handle, ins, os_, len(cols), _ptr(scratch),
                                             scratch.numel(), _stream(stream), ctypes.byref(n)),
          "mc_autotune_batched_classes")
    return n.value, outs


def merge_columns_batched(cols, outs=None, scratch=None, graph: bool = False, stream=None,
                          ctx=None, descs=None):
    """mc_merge_columns_batched over a list of ColumnInput (descs: their
    descriptors, if already built).  Returns (outs, Graph|None)."""
    ctx = ctx or context()
    if descs is None:
        descs = [c.descriptor() for c in cols]
    if outs is None:
        outs = [alloc_output(c) for c in cols]
    if scratch is None:
        scratch = alloc_scratch(batched_bounds_of(descs, ctx))
    ins = (McColumnIn * len(cols))(*descs)
    os_ = (McColumnOut * len(cols))(*[o.descriptor() for o in outs])
    g = ctypes.c_void_p() if graph else None
    check(load().mc_merge_columns_batched(ctx.handle, ins, os_, len(cols), _ptr(scratch),
                                          scratch.numel(), _stream(stream),
                                          ctypes.byref(g) if graph else None),
          "mc_merge_columns_batched")
    return outs, (Graph(g, (cols, outs, scratch, ins, os_)) if graph else None)
