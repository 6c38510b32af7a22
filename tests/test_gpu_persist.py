"""The batched merge as one persistent launch (MC_BATCHED_PERSISTENT):
every column against the oracle, byte for byte, with the GPU's own number of
workers and with 1, 3 and 7 workgroups (the queue completes with any number:
every item waits only for items already taken), several item sizes, graph
replays, columns that take the full-sort fallback, the hashing route and the
sparse X_M records, and equality with the one-launch-per-phase form."""
import numpy as np
import pytest
import torch

from hypothesis import HealthCheck, Phase, given, settings
from hypothesis import strategies as st

import oracle
import paper_1109_6885_amd as cm
from test_gpu_batched import few_prefix_values, small_batch
from test_oracle import tiny_columns
from workloads import gen

# The persistent launch stalled on the GPU in its first two runs (the second
# with one workgroup, where no workgroup waits for another); its cause is not
# found, so the library refuses MC_BATCHED_PERSISTENT and these cases do not
# run on the GPU.  The queue protocol itself is checked on the CPU
# (test_queue_model.py).
pytestmark = [pytest.mark.gpu,
              pytest.mark.skip(reason="MC_BATCHED_PERSISTENT is disabled: its launch stalled on "
                                      "the GPU (also with one workgroup); cause not found")]

PERSISTENT = 1


def say(msg):
    print(msg, flush=True)


def persist_ctx(**kw):
    ctx = cm.Context(torch.cuda.current_device())
    ctx.set_tuning(batched_launch=PERSISTENT, **kw)
    return ctx


def check_col(col, got):
    ref = oracle.merge_column(col.vtype, col.u_m, col.main_packed, col.n_main, col.w, col.delta)
    assert got["error"] == 0, got["error"]
    assert got["n_new"] == ref["n_new"] and got["w_new"] == ref["w_new"]
    assert got["words"] == ref["n_words"]
    assert np.array_equal(got["u_new"], ref["u_new"])
    assert np.array_equal(got["codes"], ref["codes"])


def run_and_check(cols, ctx, graph=False):
    dcols = [cm.ColumnInput.from_numpy(c) for c in cols]
    outs, g = cm.merge_columns_batched(dcols, ctx=ctx, graph=graph)
    torch.cuda.synchronize()
    for c, o in zip(cols, outs):
        check_col(c, o.fetch())
    return dcols, outs, g


# one worker first: it never waits for another workgroup, so it checks the
# items and their order apart from any waiting
@pytest.mark.parametrize("workers,repack,merge", [(1, 1, 1), (3, 5, 3), (7, 2, 1), (0, 0, 0),
                                                  (0, 1, 1), (0, 64, 16)])
def test_persistent_small_batch(workers, repack, merge):
    cols = small_batch(30, 0.002)
    say(f"case persistent small batch, {len(cols)} columns, workers={workers} "
        f"repack_per={repack} merge_per={merge}")
    run_and_check(cols, persist_ctx(persist_workers=workers, persist_repack=repack,
                                    persist_merge=merge))


@pytest.mark.parametrize("codes", [1024, 4096])
def test_persistent_tile_sizes(codes):
    cols = small_batch(20, 0.002)
    say(f"case persistent re-encode tile {codes}, {len(cols)} columns")
    run_and_check(cols, persist_ctx(repack_codes=codes))


def test_persistent_graph_replays():
    cols = small_batch(24, 0.001)
    say(f"case persistent graph, {len(cols)} columns")
    _, outs, graph = run_and_check(cols, persist_ctx(), graph=True)
    first = [o.fetch() for o in outs]
    for rep in range(3):
        for o in outs:
            o.new_codes.zero_()
            o.new_dict.zero_()
        x = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        graph.launch()
        torch.cuda.synchronize()
        for g0, o in zip(first, outs):
            g = o.fetch()
            assert g["error"] == 0
            assert np.array_equal(g["codes"], g0["codes"]), f"replay {rep}"
            assert np.array_equal(g["u_new"], g0["u_new"]), f"replay {rep}"
        del x


@pytest.mark.parametrize("workers", [0, 5])
def test_persistent_full_sort_fallback(workers):
    """Columns the prefix sort leaves unsorted (values sharing their leading
    bytes; ten of 600,000 delta rows each) between ordinary columns: the
    global fallback phases and the columns that wait for them."""
    rng = np.random.default_rng(17)
    cols = []
    for i, vt in enumerate(("u64", "u32", "str16") * 2 + ("u64",)):
        base = gen.random_column(rng, vt, 3000, 20_000, 0)
        n = 600_000 if workers == 0 else 40_000
        d = np.concatenate([few_prefix_values(rng, vt, n), base.u_m[rng.integers(0, 3000, 50)]])
        cols.append(gen.Column(vt, base.u_m, base.main_packed, base.n_main, base.w,
                               d[rng.permutation(d.shape[0])]))
        if i % 2 == 0:
            cols.append(gen.random_column(rng, vt, 4000, 30_000, 9_000, 0.5))
    say(f"case persistent full-sort fallback, {len(cols)} columns, workers={workers}")
    run_and_check(cols, persist_ctx(persist_workers=workers))


def test_persistent_hash_route():
    """Deltas of 2^21 rows or more hash first inside the persistent launch,
    beside radix-route and empty-delta columns; and every delta hashed
    (hash_min_rows = 1)."""
    rng = np.random.default_rng(11)
    n = (1 << 21) + 777
    cols = [gen.random_column(rng, "u64", 50_000, 200_000, n, 0.5),
            gen.random_column(rng, "u32", 300, 2000, 100, 0.5),
            gen.random_column(rng, "str16", 20_000, 100_000, n + 5, 0.3, zipf_s=1.1,
                              new_pool=5000),
            gen.random_column(rng, "u32", 1000, 10_000, 0)]
    say(f"case persistent hash route, delta rows {[c.n_delta for c in cols]}")
    run_and_check(cols, persist_ctx())
    small = small_batch(16, 0.002)
    say(f"case persistent forced hash route, {len(small)} columns")
    run_and_check(small, persist_ctx(hash_min_rows=1, persist_workers=4))


def test_persistent_sparse_records_and_partitioned_merge():
    rng = np.random.default_rng(96)
    cols = [gen.random_column(rng, "u64", 20_000, 150_000, 3_000, 0.3),
            gen.random_column(rng, "str16", 70_000, 100_000, 8_000, 0.4),
            gen.random_column(rng, "u64", 1_040_000, 60_000, 20_000, 0.5),
            gen.random_column(rng, "u32", 300_001, 120_000, 20_000, 0.5),
            gen.random_column(rng, "str16", 600_000, 30_000, 500_000, 0.9)]
    say(f"case persistent sparse records and partitioned merges, {len(cols)} columns")
    run_and_check(cols, persist_ctx())


def test_persistent_equals_phased():
    cols = small_batch(16, 0.003)
    say(f"case persistent vs phased, {len(cols)} columns")
    dcols = [cm.ColumnInput.from_numpy(c) for c in cols]
    a, _ = cm.merge_columns_batched(dcols, ctx=persist_ctx())
    b, _ = cm.merge_columns_batched(dcols, ctx=cm.Context(torch.cuda.current_device()))
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        gx, gy = x.fetch(), y.fetch()
        assert gx["error"] == 0 and gy["error"] == 0
        assert np.array_equal(gx["codes"], gy["codes"])
        assert np.array_equal(gx["u_new"], gy["u_new"])


@settings(max_examples=30, deadline=None, derandomize=True, database=None,
          phases=[Phase.explicit, Phase.generate], suppress_health_check=list(HealthCheck))
@given(st.lists(tiny_columns(), min_size=1, max_size=10), st.sampled_from([0, 1, 2, 9]))
def test_hypothesis_persistent_batches(cols, workers):
    """Batches of 1 to 10 columns from the oracle's hypothesis strategy
    (nothing to sort, merge or re-encode in some columns), 0 (the GPU's
    own count), 1, 2 or 9 workers."""
    say(f"case hypothesis persistent batch of {len(cols)}, workers={workers}: "
        + ", ".join(f"{c.vtype}/{c.u_m.shape[0]}/{c.n_main}/{c.n_delta}" for c in cols))
    run_and_check(cols, persist_ctx(persist_workers=workers))
