"""Delta index (Step 1(a)'s hashing done as rows are appended, in batches):
the indexed merge gives the oracle's bytes, for ragged batches with values
repeated within and across batches, after a reset, and for an empty delta."""
import sys

import numpy as np
import pytest
import torch

from hypothesis import HealthCheck, Phase, given, settings
from hypothesis import strategies as st

import oracle
import paper_1109_6885_amd as cm
from test_oracle import tiny_columns
from workloads import gen

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def ora(col):
    return oracle.merge_column(col.vtype, col.u_m, col.main_packed, col.n_main, col.w, col.delta)


def same(got, ref):
    assert got["error"] == 0, f"device error word {got['error']}"
    assert got["n_new"] == ref["n_new"] and got["w_new"] == ref["w_new"]
    assert got["words"] == ref["n_words"]
    assert np.array_equal(got["u_new"], ref["u_new"])
    assert np.array_equal(got["codes"], ref["codes"])
    assert np.array_equal(got["x_m"], ref["x_m"])
    assert np.array_equal(got["x_d"], ref["x_d"])
    assert got["n_ud"] == ref["u_d"].shape[0]


BATCHES = [1, 4096, 12_345, 100_000, 2, 133_557]  # 250,001 rows


@pytest.mark.parametrize("vtype", ["u32", "u64", "str16"])
def test_indexed_merge_matches_oracle(vtype):
    rng = np.random.default_rng({"u32": 61, "u64": 62, "str16": 63}[vtype])
    col = gen.random_column(rng, vtype, 20_000, 100_003, sum(BATCHES), 0.4, zipf_s=1.1,
                            new_pool=20_000)
    dcol = cm.ColumnInput.from_numpy(col)
    ix = cm.DeltaIndex(vtype, 300_000)
    for b in BATCHES:
        say(f"case index append {vtype} rows {ix.rows}..{ix.rows + b}")
        ix.append(dcol.delta, b)
    say(f"case indexed merge {vtype} nd={col.n_delta}")
    out = cm.merge_column_indexed(dcol, ix, tables=True)
    torch.cuda.synchronize()
    same(out.fetch(), ora(col))

    # the same index, reset, over the first 70,001 rows of a new delta
    col2 = gen.random_column(rng, vtype, 20_000, 100_003, 70_001, 0.9)
    dcol2 = cm.ColumnInput.from_numpy(col2)
    ix.reset()
    for b in (35_000, 35_001):
        ix.append(dcol2.delta, b)
    say(f"case indexed merge after reset {vtype} nd={col2.n_delta}")
    out2 = cm.merge_column_indexed(dcol2, ix, tables=True)
    torch.cuda.synchronize()
    same(out2.fetch(), ora(col2))


def test_indexed_merge_empty_delta():
    rng = np.random.default_rng(64)
    col = gen.random_column(rng, "u64", 5000, 30_000, 0)
    dcol = cm.ColumnInput.from_numpy(col)
    ix = cm.DeltaIndex("u64", 1000)
    say("case indexed merge, empty delta")
    out = cm.merge_column_indexed(dcol, ix, tables=True)
    torch.cuda.synchronize()
    same(out.fetch(), ora(col))


def test_index_append_rejects_overflow():
    ix = cm.DeltaIndex("u32", 100)
    delta = torch.zeros(128, dtype=torch.int32, device="cuda")
    ix.append(delta, 60)
    with pytest.raises(cm.ColmergeError):
        ix.append(delta, 41)


@settings(max_examples=40, deadline=None, derandomize=True, database=None,
          phases=[Phase.explicit, Phase.generate], suppress_health_check=list(HealthCheck))
@given(tiny_columns(), st.lists(st.integers(1, 25), min_size=1, max_size=8))
def test_hypothesis_indexed(col, cuts):
    """Tiny columns from the oracle's hypothesis strategy with the delta
    appended to an index in batches of 1 to 25 rows (the last batch takes
    the rest), generated deterministically and never shrunk."""
    dcol = cm.ColumnInput.from_numpy(col)
    ix = cm.DeltaIndex(col.vtype, max(col.n_delta, 1))
    done = 0
    for b in cuts:
        b = min(b, col.n_delta - done)
        if b <= 0:
            break
        ix.append(dcol.delta, b)
        done += b
    if done < col.n_delta:
        ix.append(dcol.delta, col.n_delta - done)
    say(f"case hypothesis indexed {col.vtype} n_um={col.u_m.shape[0]} nd={col.n_delta} "
        f"batches={cuts}")
    out = cm.merge_column_indexed(dcol, ix, tables=True)
    torch.cuda.synchronize()
    same(out.fetch(), ora(col))
