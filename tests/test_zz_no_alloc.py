"""The allocation-free merge (mc_merge_column_noalloc) against the merge
with a caller-provided workspace (mc_merge_column), byte for byte, on two
calls in a row -- the second with a smaller column, so that it runs on the
workspace the first one left behind -- and against the oracle; a column
whose workspace exceeds the library's array is refused before any launch."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_1109_6885_amd as cm
from paper_1109_6885_amd import _lib
from workloads import gen

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


def _same(a, b):
    assert a["error"] == 0 and b["error"] == 0
    for k in ("n_new", "w_new", "words", "n_ud"):
        assert a[k] == b[k], k
    for k in ("u_new", "codes", "x_m", "x_d"):
        assert np.array_equal(a[k], b[k]), k


def _check_against_oracle(col, got):
    ref = oracle.merge_column(col.vtype, col.u_m, col.main_packed, col.n_main, col.w, col.delta)
    assert got["n_new"] == ref["n_new"] and got["w_new"] == ref["w_new"]
    assert got["words"] == ref["n_words"]
    assert np.array_equal(got["u_new"], ref["u_new"])
    assert np.array_equal(got["codes"], ref["codes"])
    assert np.array_equal(got["x_m"], ref["x_m"]) and np.array_equal(got["x_d"], ref["x_d"])


def test_noalloc_matches_merge_column_twice():
    rng = np.random.default_rng(4242)
    # the first column's workspace is large (full sort buffers, tables);
    # the second is smaller and runs on what the first left behind
    cols = [gen.random_column(rng, "u64", 200_000, 400_001, 150_000, 0.7),
            gen.random_column(rng, "str16", 3_000, 20_000, 5_001, 0.4)]
    ctx = cm.context()
    stream = torch.cuda.current_stream()
    for i, col in enumerate(cols):
        dcol = cm.ColumnInput.from_numpy(col)
        sb = cm.merge_bounds(dcol, ctx)[2]
        say(f"case noalloc call {i}: {col.vtype} n_um={col.u_m.shape[0]} n_main={col.n_main} "
            f"nd={col.n_delta} workspace={sb}")
        assert sb <= _lib.NOALLOC_SCRATCH_BYTES
        ref_out = cm.merge_column(dcol, tables=True, stream=stream, ctx=ctx)
        out = cm.alloc_output(dcol, tables=True)
        torch.cuda.synchronize()
        cm.merge_column_noalloc(dcol, out, stream=stream, ctx=ctx)
        torch.cuda.synchronize()
        got, ref = out.fetch(), ref_out.fetch()
        _same(got, ref)
        _check_against_oracle(col, got)


def test_noalloc_refuses_oversized_workspace():
    """A column whose workspace is above the array's size is refused on the
    host with MC_E_CAP; nothing is launched."""
    lib = _lib.load()
    ctx = cm.context()
    d = _lib.McColumnIn()
    d.type, d.bitwidth = 1, 24
    buf = torch.zeros(64, dtype=torch.int64, device="cuda")
    p = buf.data_ptr()
    d.main_dict, d.main_dict_len = p, 10_000_000
    d.main_codes, d.main_rows = p, 50_000_000
    d.delta_values, d.delta_rows = p, 8_000_000
    dc, words, sb = cm.bounds_of(d)
    assert sb > _lib.NOALLOC_SCRATCH_BYTES
    o = _lib.McColumnOut()
    o.new_dict, o.new_dict_cap = p, dc
    o.new_codes, o.new_codes_cap_words = p, words
    o.result = p
    rc = lib.mc_merge_column_noalloc(ctx.handle, ctypes.byref(d), ctypes.byref(o),
                                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == -2
    assert b"MC_NOALLOC_SCRATCH_BYTES" in lib.mc_last_error()
