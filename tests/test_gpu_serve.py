"""Served merges on the GPU: resident tables, appends overlapping merges on
a pool of streams, admission under a budget (continuous batching, the
online merge of Section 3).  Merges are launched exactly as the server
launches them (no synchronization added), and at least two run at once.
Every committed column is compared byte for byte with the oracle: each
table's merges are replayed on the host in commit order, the first from the
table's generated columns and each later one from the oracle's own previous
result, with the rows that the test appended into that merge's snapshot --
no oracle input comes from the GPU.  The same snapshot re-merged alone with
mc_merge_column gives the same bytes as in the mix."""
import collections

import numpy as np
import pytest
import torch

import oracle
import paper_1109_6885_amd as cm
from paper_1109_6885_amd import serve
from workloads import gen

pytestmark = pytest.mark.gpu


class RecordingExecutor(serve.GpuExecutor):
    """Records, per delta buffer, the host rows appended to it, and per
    merge the host rows of its snapshot, the table and the result columns.
    It adds no synchronization: merges overlap as in the server."""

    def __init__(self):
        super().__init__(n_streams=4)
        self.table_of = {}          # id(main) -> table
        self.host_rows = {}         # id(delta) -> list of per-column host arrays
        self.log = []               # (table, snapshot host rows, result main)

    def append(self, d, rows):
        self.host_rows.setdefault(id(d), []).append(rows["host"])
        return super().append(d, rows)

    def clear_delta(self, d):
        self.host_rows[id(d)] = []
        return super().clear_delta(d)

    def launch(self, m, d):
        job = super().launch(m, d)
        job["table"] = self.table_of[id(m)]
        job["snap_rows"] = list(self.host_rows.get(id(d), []))
        return job

    def result(self, job):
        new = super().result(job)
        self.table_of[id(new)] = job["table"]
        # a copy of the column list: committing the table's next merge
        # empties this main's list
        self.log.append((job["table"], job["snap_rows"], list(new.cols)))
        return new


def _host(t, vtype):
    a = t.cpu().numpy()
    return a.view(np.uint32) if vtype == "u32" else (a.view(np.uint64) if vtype == "u64" else a)


def test_served_alone_equals_in_the_mix():
    rng = np.random.default_rng(2024)
    ex = RecordingExecutor()
    ntab, ncol = 4, 6
    shapes = gen.batched_shapes(ntab * ncol, scale=0.01)
    tables = {}
    host_cols = {}
    for t in range(ntab):
        cols = []
        for vt, rows, kd, sub in shapes[t * ncol:(t + 1) * ncol]:
            r2 = np.random.default_rng(sub)
            cols.append(gen.random_column(r2, vt, kd, rows, 0))
        host_cols[t] = cols
        tables[t] = serve.gpu_main_from_columns(ex, cols)
        ex.table_of[id(tables[t])] = t
    s = serve.Server(ex, budget_bytes=64 << 30, max_inflight=3)
    for t, m in tables.items():
        s.add_table(t, m, delta_capacity=50_000)
    max_running = 0
    reqs = []
    for step in range(60):
        t = int(rng.integers(0, ntab))
        n = int(rng.integers(100, 2000))
        by_type = collections.defaultdict(list)
        per_col = []
        for c in host_cols[t]:
            half = n // 2
            new = gen.random_values(rng, c.vtype, n - half)
            old = c.u_m[rng.integers(0, c.u_m.shape[0], half)] if c.u_m.shape[0] else \
                gen.random_values(rng, c.vtype, half)
            v = np.concatenate([old, new], axis=0)
            by_type[c.vtype].append(v)
            per_col.append(v)
        batch = serve.append_batch(ex, s.tables[t].main,
                                   {vt: np.stack(vs) for vt, vs in by_type.items()}, n)
        batch["host"] = per_col
        s.append(t, batch)
        if step % 4 == 0:
            # a burst of requests for different tables: admitted together,
            # they run on different streams at once
            for tt in rng.permutation(ntab)[:3].tolist():
                reqs.append(s.submit_merge(int(tt)))
        s.poll()
        max_running = max(max_running, len(s.running))
    # a last merge per table folds every remaining appended row in
    for t in range(ntab):
        reqs.append(s.submit_merge(t))
    s.poll()
    max_running = max(max_running, len(s.running))
    s.drain()
    torch.cuda.synchronize()
    assert all(r.status == "committed" for r in reqs)
    assert len(ex.log) == len(reqs)
    assert max_running >= 2, "no two merges were ever in flight together"

    # the oracle, chained per table in commit order
    state = {t: [(c.u_m, c.main_packed, c.n_main, c.w) for c in host_cols[t]]
             for t in range(ntab)}
    for table, snap_rows, got_cols in ex.log:
        assert len(got_cols) == ncol
        for j, (c, got_col) in enumerate(zip(host_cols[table], got_cols)):
            u_m, packed, n_main, w = state[table][j]
            parts = [b[j] for b in snap_rows]
            delta = (np.concatenate(parts, axis=0) if parts else
                     gen.random_values(rng, c.vtype, 0))
            ref = oracle.merge_column(c.vtype, u_m, packed, n_main, w, delta)
            assert got_col.w == ref["w_new"]
            assert got_col.n_main == n_main + delta.shape[0]
            assert np.array_equal(_host(got_col.u_m, c.vtype), ref["u_new"])
            got_words = got_col.main_codes[: ref["n_words"]].cpu().numpy().view(np.uint64)
            assert np.array_equal(got_words, ref["codes"]), (table, j)
            state[table][j] = (ref["u_new"], ref["codes"], n_main + delta.shape[0],
                               ref["w_new"])
            # the same inputs merged alone, on an otherwise idle GPU (the
            # snapshot's delta buffer has been reused since, so its host rows
            # and the main the oracle chain reached -- byte-identical to the
            # GPU's, as asserted above -- are copied in again)
            alone = cm.merge_column(cm.ColumnInput.from_numpy(
                gen.Column(c.vtype, u_m, packed, n_main, w, delta)))
            torch.cuda.synchronize()
            a = alone.fetch()
            assert a["error"] == 0 and a["w_new"] == got_col.w
            assert np.array_equal(a["u_new"], ref["u_new"])
            assert np.array_equal(a["codes"], ref["codes"])
    st = s.stats()
    assert st["merges"] == len(reqs) and st["p99_ms"] is not None
    assert st["peak_in_use_bytes"] <= st["budget_bytes"]


def test_gpu_generator_layout():
    """The device-side generator packs like the host generator and makes
    sorted unique dictionaries."""
    from workloads import gpu_gen
    g = torch.Generator(device="cuda")
    g.manual_seed(1)
    for w in (1, 7, 13, 20, 32):
        codes = torch.randint(0, 2 ** w, (10_007,), generator=g, device="cuda", dtype=torch.int64)
        ref = gen.pack_codes(codes.cpu().numpy().astype(np.uint64), w)
        got = gpu_gen.pack_codes_gpu(codes, w).cpu().numpy().view(np.uint64)
        assert np.array_equal(got[: ref.shape[0]], ref)
    for vt in ("u32", "u64", "str16"):
        _, u, packed, n, w = gpu_gen.served_column(g, vt, 20_000, 3000)
        a = u.cpu().numpy()
        if vt == "u32":
            a = a.view(np.uint32)
        assert a.shape[0] == 3000
        assert np.array_equal(gen.sort_unique_values(a, vt), a)
