"""Batched merge (many uneven columns of mixed value types in one launch
sequence, optionally captured in a HIP graph) against the oracle, column by
column, byte for byte; graph replays checked one by one."""
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


def check_col(col, got):
    ref = oracle.merge_column(col.vtype, col.u_m, col.main_packed, col.n_main, col.w, col.delta)
    assert got["error"] == 0
    assert got["n_new"] == ref["n_new"] and got["w_new"] == ref["w_new"]
    assert got["words"] == ref["n_words"]
    assert np.array_equal(got["u_new"], ref["u_new"])
    assert np.array_equal(got["codes"], ref["codes"])


def small_batch(ncols=40, scale=0.002):
    cols = gen.batched_columns(ncols, scale)
    # add the edge cases: empty delta, empty main, one-entry dictionary
    rng = np.random.default_rng(5)
    cols.append(gen.random_column(rng, "u64", 100, 5000, 0))
    cols.append(gen.random_column(rng, "str16", 0, 0, 3000, 1.0))
    cols.append(gen.random_column(rng, "u32", 1, 777, 5, 0.0))
    return cols


def test_batched_direct():
    cols = small_batch()
    say(f"case batched direct, {len(cols)} columns")
    dcols = [cm.ColumnInput.from_numpy(c) for c in cols]
    outs, _ = cm.merge_columns_batched(dcols)
    torch.cuda.synchronize()
    for c, o in zip(cols, outs):
        check_col(c, o.fetch())


def test_batched_partitioned_merge():
    """Columns whose dictionaries merge over 2^20 positions (at least 128
    tiles) find the merge tile boundaries in a launch of their own; mixed
    with small columns."""
    rng = np.random.default_rng(6)
    cols = [gen.random_column(rng, "u64", 1_040_000, 60_000, 20_000, 0.5),
            gen.random_column(rng, "u32", 300, 2000, 100, 0.5),
            gen.random_column(rng, "str16", 600_000, 30_000, 500_000, 0.9),
            gen.random_column(rng, "u32", 1_100_000, 10_000, 0)]
    say(f"case batched partitioned merge, {len(cols)} columns")
    dcols = [cm.ColumnInput.from_numpy(c) for c in cols]
    outs, _ = cm.merge_columns_batched(dcols)
    torch.cuda.synchronize()
    for c, o in zip(cols, outs):
        check_col(c, o.fetch())


def test_batched_sparse_xm_records():
    """Columns whose re-encode reads the sparse X_M records (dictionaries of
    16K-300K entries with few new values; one with new values bunched into
    one gap so that a record overflows) between columns that keep the 16-bit
    table (dense insertions, small dictionaries), in one batched call and
    replayed from a graph."""
    rng = np.random.default_rng(96)
    cols = [gen.random_column(rng, "u64", 20_000, 150_000, 3_000, 0.3),
            gen.random_column(rng, "u32", 300, 2000, 100, 0.5),
            gen.random_column(rng, "str16", 70_000, 100_000, 8_000, 0.4),
            gen.random_column(rng, "u64", 16_384, 80_000, 60_000, 1.0),
            gen.random_column(rng, "u32", 300_001, 120_000, 20_000, 0.5)]
    c = gen.random_column(rng, "u64", 100_000, 90_000, 5_000, 0.2)
    lo = int(c.u_m[40_000])
    extra = np.arange(lo + 1, lo + 401, dtype=np.uint64)
    assert int(extra[-1]) < int(c.u_m[40_001])
    d = np.concatenate([c.delta, extra])
    cols.append(gen.Column("u64", c.u_m, c.main_packed, c.n_main, c.w,
                           d[rng.permutation(d.shape[0])]))
    say(f"case batched sparse X_M records, {len(cols)} columns")
    dcols = [cm.ColumnInput.from_numpy(c) for c in cols]
    outs, graph = cm.merge_columns_batched(dcols, graph=True)
    torch.cuda.synchronize()
    for c, o in zip(cols, outs):
        check_col(c, o.fetch())
    for _ in range(2):
        graph.launch()
        torch.cuda.synchronize()
        for c, o in zip(cols, outs):
            check_col(c, o.fetch())


def test_batched_prefix_sort_fallback():
    """Columns whose values share their leading bytes between ordinary
    columns, in one batch; twice, through a graph, so the sort's counters
    restart."""
    rng = np.random.default_rng(8)
    cols = []
    for vt in ("u64", "u32", "str16"):
        base = gen.random_column(rng, vt, 2000, 10_000, 0)
        if vt == "str16":
            d = rng.integers(0x20, 0x7F, size=(30_000, 16), dtype=np.uint8)
            d[:, 0], d[:, 1] = ord("q"), ord("r")
        elif vt == "u32":
            d = (np.uint32(0x4321) << np.uint32(16)) | rng.integers(0, 1 << 16, 30_000).astype(np.uint32)
        else:
            d = (np.uint64(0x4321) << np.uint64(48)) | rng.integers(0, 1 << 48, 30_000, dtype=np.uint64)
        d = np.concatenate([d, gen.random_values(rng, vt, 10)])
        cols.append(gen.Column(vt, base.u_m, base.main_packed, base.n_main, base.w,
                               d[rng.permutation(d.shape[0])]))
        cols.append(gen.random_column(rng, vt, 5000, 20_000, 7_000, 0.5))
    say(f"case batched prefix-sort fallback, {len(cols)} columns")
    dcols = [cm.ColumnInput.from_numpy(c) for c in cols]
    outs, graph = cm.merge_columns_batched(dcols, graph=True)
    torch.cuda.synchronize()
    for c, o in zip(cols, outs):
        check_col(c, o.fetch())
    for o in outs:
        o.new_codes.zero_()
        o.new_dict.zero_()
    graph.launch()
    torch.cuda.synchronize()
    for c, o in zip(cols, outs):
        check_col(c, o.fetch())


def few_prefix_values(rng, vtype, n):
    """n values whose three leading bytes each take one of two values and
    whose other bytes are random: every run of equal prefix holds about n / 8
    values in no order, so the prefix sort leaves them unsorted and the full
    sort has to run."""
    top = [rng.integers(0, 2, n) * 0x40 + 0x21 for _ in range(3)]
    if vtype == "str16":
        d = rng.integers(0x20, 0x7F, size=(n, 16), dtype=np.uint8)
        for i in range(3):
            d[:, i] = top[i]
        return d
    if vtype == "u32":
        v = rng.integers(0, 256, n).astype(np.uint32)
        for i in range(3):
            v |= top[i].astype(np.uint32) << np.uint32(24 - 8 * i)
        return v
    v = rng.integers(0, 1 << 40, n, dtype=np.uint64)
    for i in range(3):
        v |= top[i].astype(np.uint64) << np.uint64(56 - 8 * i)
    return v


def test_batched_full_sort_concurrent_streams():
    """Three batches enqueued on three streams at once, each with two columns
    that need the full sort between ordinary ones: every batch's one-launch
    full sort has at most one workgroup per two CUs and a grid-wide barrier
    that assumes they are all resident, and three of them fit together (a CU
    holds three of those workgroups).  Every column against the oracle."""
    rng = np.random.default_rng(23)
    batches = []
    for b in range(3):
        cols = []
        for vt in ("u64", "str16"):
            base = gen.random_column(rng, vt, 2000, 20_000, 0)
            d = np.concatenate([few_prefix_values(rng, vt, 200_000),
                                base.u_m[rng.integers(0, 2000, 40)]])
            cols.append(gen.Column(vt, base.u_m, base.main_packed, base.n_main, base.w,
                                   d[rng.permutation(d.shape[0])]))
        cols.append(gen.random_column(rng, "u32", 3000, 25_000, 6_000, 0.5))
        batches.append(cols)
    say("case batched full sort, three batches on three streams at once")
    streams = [torch.cuda.Stream() for _ in batches]
    ctxs = []
    for _ in batches:
        ctx = cm.Context(torch.cuda.current_device())
        ctx.set_tuning(hash_dict_ratio=0xFFFFFFFF)  # the radix route and its full sort
        ctxs.append(ctx)
    dcols = [[cm.ColumnInput.from_numpy(c) for c in cols] for cols in batches]
    outs = [[cm.alloc_output(d) for d in dc] for dc in dcols]
    scratch = [cm.alloc_scratch(cm.batched_bounds_of([d.descriptor() for d in dc], x))
               for dc, x in zip(dcols, ctxs)]
    torch.cuda.synchronize()
    for dc, o, sc, st, x in zip(dcols, outs, scratch, streams, ctxs):
        cm.merge_columns_batched(dc, outs=o, scratch=sc, stream=st, ctx=x)
    torch.cuda.synchronize()
    for cols, os_ in zip(batches, outs):
        for c, o in zip(cols, os_):
            check_col(c, o.fetch())


def test_batched_full_sort_many_columns():
    """Ten columns that all need the full sort, 600,000 delta rows each,
    between ordinary columns: the full sort's launch has fewer workgroups
    than those columns' tiles, digits and emit tiles, so each workgroup takes
    several, across column boundaries.  Through a graph, twice."""
    rng = np.random.default_rng(17)
    cols = []
    for i, vt in enumerate(("u64", "u32", "str16") * 3 + ("u64",)):
        base = gen.random_column(rng, vt, 3000, 20_000, 0)
        d = np.concatenate([few_prefix_values(rng, vt, 600_000),
                            base.u_m[rng.integers(0, 3000, 50)]])
        cols.append(gen.Column(vt, base.u_m, base.main_packed, base.n_main, base.w,
                               d[rng.permutation(d.shape[0])]))
        if i % 3 == 0:
            cols.append(gen.random_column(rng, vt, 4000, 30_000, 9_000, 0.5))
    say(f"case batched full sort, {len(cols)} columns")
    dcols = [cm.ColumnInput.from_numpy(c) for c in cols]
    # the radix route (600,000 rows over 3,000 entries would hash by default)
    ctx = cm.Context(torch.cuda.current_device())
    ctx.set_tuning(hash_dict_ratio=0xFFFFFFFF)
    outs, graph = cm.merge_columns_batched(dcols, graph=True, ctx=ctx)
    torch.cuda.synchronize()
    for c, o in zip(cols, outs):
        check_col(c, o.fetch())
    for o in outs:
        o.new_codes.zero_()
        o.new_dict.zero_()
    graph.launch()
    torch.cuda.synchronize()
    for c, o in zip(cols, outs):
        check_col(c, o.fetch())


def test_batched_few_main_values_repeated():
    """Columns whose deltas repeat a few main values (the shapes of the
    300-column batch that needed the full sort) beside ordinary ones: by
    default they hash first; with the rule off they take the radix route and
    the full sort; both agree with the oracle."""
    rng = np.random.default_rng(23)
    cols = []
    for vt, kd, nd in (("str16", 6, 63_400), ("u32", 119, 197_246), ("str16", 738, 168_887),
                       ("u64", 66, 155_927), ("str16", 50, 28_997)):
        cols.append(gen.random_column(rng, vt, kd, 30_000, nd, 0.5))
        cols.append(gen.random_column(rng, vt, 20_000, 30_000, 5_000, 0.5))
    dcols = [cm.ColumnInput.from_numpy(c) for c in cols]
    for ratio in (0, 0xFFFFFFFF):
        say(f"case batched few main values repeated, {len(cols)} columns, ratio {ratio:#x}")
        ctx = cm.Context(torch.cuda.current_device())
        ctx.set_tuning(hash_dict_ratio=ratio)
        outs, _ = cm.merge_columns_batched(dcols, ctx=ctx)
        torch.cuda.synchronize()
        for c, o in zip(cols, outs):
            check_col(c, o.fetch())


def test_class_shapes_mixed():
    """Per-class shapes: every class of the batch gets a different re-encode
    tile (1024, 2048, 4096 in turn) and prefix run, so one batch runs the
    three re-encode launches side by side; every column still matches the
    oracle, also from a graph, and clearing the cache restores the context's
    shapes."""
    cols = small_batch(30, 0.002)
    dcols = [cm.ColumnInput.from_numpy(c) for c in cols]
    ctx = cm.Context(torch.cuda.current_device())
    classes = sorted({cm.tune_class(d) for d in dcols})
    say(f"case mixed class shapes, {len(cols)} columns, classes {classes}")
    codes, runs = (1024, 2048, 4096), (16, 32, 64)
    for i, c in enumerate(classes):
        ctx.set_class_tuning(c, codes[i % 3], runs[(i // 3) % 3])
    assert set(ctx.class_tuning_cache()) == set(classes)
    assert len({ctx.get_class_tuning(c)[0]["repack_codes"] for c in classes}) == min(3, len(classes))
    for graph in (False, True):
        outs, g = cm.merge_columns_batched(dcols, ctx=ctx, graph=graph)
        torch.cuda.synchronize()
        for c, o in zip(cols, outs):
            check_col(c, o.fetch())
    for c in classes:
        ctx.set_class_tuning(c)
    assert ctx.class_tuning_cache() == {}
    assert ctx.get_class_tuning(classes[0]) == ({"repack_codes": 2048, "prefix_run": 32}, False)


def test_autotune_batched_classes(tmp_path):
    """The per-class autotuner caches one of its candidates for every class of
    the batch, leaves the batch's result in the outputs, and the cache
    survives a JSON round trip into a fresh context whose merges agree with
    the oracle."""
    cols = small_batch(24, 0.002)
    dcols = [cm.ColumnInput.from_numpy(c) for c in cols]
    ctx = cm.Context(torch.cuda.current_device())
    classes = {cm.tune_class(d) for d in dcols}
    say(f"case class autotune, {len(cols)} columns, {len(classes)} classes")
    n, outs = cm.autotune_batched_classes(dcols, ctx=ctx)
    torch.cuda.synchronize()
    assert n == len(classes)
    cache = ctx.class_tuning_cache()
    assert set(cache) == classes
    for v in cache.values():
        assert v["repack_codes"] in (1024, 2048, 4096) and v["prefix_run"] in (16, 32, 64)
    for c, o in zip(cols, outs):
        check_col(c, o.fetch())
    path = str(tmp_path / "classes.json")
    ctx.save_class_tuning(path)
    ctx2 = cm.Context(torch.cuda.current_device())
    ctx2.load_class_tuning(path)
    assert ctx2.class_tuning_cache() == cache
    outs2, _ = cm.merge_columns_batched(dcols, ctx=ctx2)
    torch.cuda.synchronize()
    for c, o in zip(cols, outs2):
        check_col(c, o.fetch())


def test_autotune_batched():
    """The autotuner picks one of its candidates, leaves the batch's result
    in the outputs, and later batched merges with the chosen shapes agree
    with the oracle."""
    cols = small_batch(20, 0.002)
    say(f"case autotune, {len(cols)} columns")
    ctx = cm.Context(torch.cuda.current_device())
    dcols = [cm.ColumnInput.from_numpy(c) for c in cols]
    chosen, times, outs = cm.autotune_batched(dcols, ctx=ctx)
    assert chosen["repack_codes"] in (1024, 2048, 4096)
    assert chosen["prefix_run"] in (16, 32, 64)
    assert len(times) == 6 and all(t > 0 for t in times)
    assert ctx.get_tuning() == chosen
    for c, o in zip(cols, outs):
        check_col(c, o.fetch())
    outs2, _ = cm.merge_columns_batched(dcols, ctx=ctx)
    torch.cuda.synchronize()
    for c, o in zip(cols, outs2):
        check_col(c, o.fetch())


def test_batched_graph_replays():
    cols = small_batch(24, 0.001)
    say(f"case batched graph, {len(cols)} columns")
    dcols = [cm.ColumnInput.from_numpy(c) for c in cols]
    outs, graph = cm.merge_columns_batched(dcols, graph=True)
    torch.cuda.synchronize()
    first = [o.fetch() for o in outs]
    for c, g in zip(cols, first):
        check_col(c, g)
    for rep in range(3):
        # eager work between replays, then clear the outputs and replay
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


def test_batched_equals_plain():
    cols = small_batch(16, 0.003)
    say(f"case batched vs plain, {len(cols)} columns")
    dcols = [cm.ColumnInput.from_numpy(c) for c in cols]
    outs, _ = cm.merge_columns_batched(dcols)
    plain = [cm.merge_column(d) for d in dcols]
    torch.cuda.synchronize()
    for a, b in zip(outs, plain):
        ga, gb = a.fetch(), b.fetch()
        assert np.array_equal(ga["codes"], gb["codes"])
        assert np.array_equal(ga["u_new"], gb["u_new"])
        assert ga["w_new"] == gb["w_new"]


def _replay_and_check(outs, graph, first, reps=3):
    for rep in range(reps):
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


def test_batched_hash_route():
    """Columns whose deltas reach 2^21 rows hash first inside the batch, as
    they do alone (all distinct, heavy duplicates), beside radix-route and
    empty-delta columns; directly, then from a graph replayed three times
    with eager work between the replays."""
    rng = np.random.default_rng(11)
    n = (1 << 21) + 777
    cols = [gen.random_column(rng, "u64", 50_000, 200_000, n, 0.5),
            gen.random_column(rng, "u32", 300, 2000, 100, 0.5),
            gen.random_column(rng, "str16", 20_000, 100_000, n + 5, 0.3, zipf_s=1.1,
                              new_pool=5000),
            gen.random_column(rng, "u32", 1000, 10_000, 0)]
    say(f"case batched hash route, {len(cols)} columns, delta rows {[c.n_delta for c in cols]}")
    dcols = [cm.ColumnInput.from_numpy(c) for c in cols]
    outs, _ = cm.merge_columns_batched(dcols)
    torch.cuda.synchronize()
    for c, o in zip(cols, outs):
        check_col(c, o.fetch())
    say("case batched hash route, graph")
    gouts, graph = cm.merge_columns_batched(dcols, graph=True)
    torch.cuda.synchronize()
    first = [o.fetch() for o in gouts]
    for c, g in zip(cols, first):
        check_col(c, g)
    _replay_and_check(gouts, graph, first)


def test_batched_forced_hash_route():
    """Every column with a delta through the hashing route (hash_min_rows = 1
    on the context, scratch from the context's bound): the whole small batch
    against the oracle, and the same as the plain calls on that context."""
    cols = small_batch(24, 0.002)
    say(f"case batched forced hash route, {len(cols)} columns")
    ctx = cm.Context(torch.cuda.current_device())
    ctx.set_tuning(hash_min_rows=1)
    dcols = [cm.ColumnInput.from_numpy(c) for c in cols]
    assert cm.batched_bounds(dcols, ctx) > cm.batched_bounds(dcols)
    outs, _ = cm.merge_columns_batched(dcols, ctx=ctx)
    torch.cuda.synchronize()
    for c, o in zip(cols, outs):
        check_col(c, o.fetch())
    plain = [cm.merge_column(d, ctx=ctx) for d in dcols]
    torch.cuda.synchronize()
    for a, b in zip(outs, plain):
        assert np.array_equal(a.fetch()["codes"], b.fetch()["codes"])


@settings(max_examples=40, deadline=None, derandomize=True, database=None,
          phases=[Phase.explicit, Phase.generate], suppress_health_check=list(HealthCheck))
@given(st.lists(tiny_columns(), min_size=1, max_size=10))
def test_hypothesis_batches(cols):
    """Batches of 1 to 10 columns from the oracle's hypothesis strategy
    (columns with nothing to sort, merge or re-encode give zero tiles in
    some phases), generated deterministically and never shrunk."""
    say(f"case hypothesis batch of {len(cols)}: "
        + ", ".join(f"{c.vtype}/{c.u_m.shape[0]}/{c.n_main}/{c.n_delta}" for c in cols))
    dcols = [cm.ColumnInput.from_numpy(c) for c in cols]
    outs, _ = cm.merge_columns_batched(dcols)
    torch.cuda.synchronize()
    for c, o in zip(cols, outs):
        check_col(c, o.fetch())


@pytest.mark.slow
def test_batched_full_c4_against_oracle():
    """The whole 300-column batched workload (1.96e9 rows, u32/u64/str16,
    rows log-uniform in [1M, 20M], distinct counts log-uniform in [2, 10M],
    delta 1% of rows, half new values), replayed from a HIP graph as the
    benchmark runs it: every column's |U'|, w', W', U' and all of its result
    words against the oracle's merge of the same column.  The oracle runs in
    worker processes that return SHA-256 digests of U' and of the result
    words (equal digests: equal bytes); a column whose digests differ is
    merged again by the oracle here and compared element by element."""
    import concurrent.futures as cf
    import multiprocessing as mp
    import os

    import oracle_pool

    workers = min(16, os.cpu_count() or 1)
    shapes = gen.batched_shapes(300)
    ctx = mp.get_context("spawn")
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=ctx) as pool:
        # largest columns first, so the pool's tail is short
        order = sorted(range(len(shapes)), key=lambda i: -shapes[i][1])
        futs = {i: pool.submit(oracle_pool.oracle_digest, shapes[i]) for i in order}
        cols = gen.batched_columns(300, workers=workers)
        say(f"case full batched workload, {len(cols)} columns, "
            f"{sum(c.n_main + c.n_delta for c in cols)} rows")
        dcols = [cm.ColumnInput.from_numpy(c) for c in cols]
        outs, graph = cm.merge_columns_batched(dcols, graph=True)
        torch.cuda.synchronize()
        for o in outs:                    # the replay must write everything again
            o.new_codes.zero_()
            o.new_dict.zero_()
        graph.launch()
        torch.cuda.synchronize()
        for j, (c, o) in enumerate(zip(cols, outs)):
            got, ref = o.fetch(), futs[j].result()
            assert got["error"] == 0, (j, got["error"])
            same = ((got["n_new"], got["w_new"], got["words"]) ==
                    (ref["n_new"], ref["w_new"], ref["n_words"])
                    and oracle_pool.digest(got["u_new"]) == ref["u_new"]
                    and oracle_pool.digest(got["codes"]) == ref["codes"])
            if not same:
                check_col(c, got)         # element-wise, to name what differs
                raise AssertionError(f"column {j}: digests differ")
    del graph, outs, dcols
    torch.cuda.empty_cache()
