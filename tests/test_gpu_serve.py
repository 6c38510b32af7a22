"""Served merges on the GPU: resident tables, appends overlapping merges on
a pool of streams, admission under a budget.  Each committed result must be
byte-identical to the same merge run alone (its recorded snapshot re-merged
with mc_merge_column on an idle GPU), and the final tables must decode to
every row in order (checked against the oracle for one table)."""
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
    """Keeps a copy of every merge's inputs and its outputs."""

    def __init__(self):
        super().__init__(n_streams=4)
        self.log = []

    def launch(self, m, d):
        torch.cuda.synchronize()
        snap = [cm.ColumnInput(c.vtype, c.u_m.clone(), c.main_codes.clone(), c.n_main, c.w,
                               c.delta.clone()) for c in self._inputs(m, d)]
        job = super().launch(m, d)
        job["snap"] = snap
        return job

    def result(self, job):
        new = super().result(job)
        self.log.append((job["snap"], [(c.u_m, c.main_codes, c.w) for c in new.cols]))
        return new


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
    s = serve.Server(ex, budget_bytes=64 << 30, max_inflight=3)
    for t, m in tables.items():
        s.add_table(t, m, delta_capacity=50_000)
    appended = collections.defaultdict(list)
    reqs = []
    for step in range(40):
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
        if s.append(t, batch):
            appended[t].append(per_col)
        if step % 3 == 0:
            reqs.append(s.submit_merge(int(rng.integers(0, ntab))))
        s.poll()
    # a last merge per table folds every remaining appended row in
    for t in range(ntab):
        reqs.append(s.submit_merge(t))
    s.drain()
    torch.cuda.synchronize()
    assert all(r.status == "committed" for r in reqs)
    assert len(ex.log) == len(reqs)
    # every result equals the same merge run alone
    for snap, got in ex.log:
        for col, (u_new, codes, w_new) in zip(snap, got):
            alone = cm.merge_column(col)
            torch.cuda.synchronize()
            a = alone.fetch()
            assert a["error"] == 0 and a["w_new"] == w_new
            assert torch.equal(alone.new_dict[: a["n_new"]], u_new)
            assert np.array_equal(a["codes"], codes[: a["words"]].cpu().numpy().view(np.uint64))
    # table 0 end to end: its final main decodes to the original rows
    # followed by every appended row, in order
    for j, c in enumerate(host_cols[0]):
        fin = s.tables[0].main.cols[j]
        u = fin.u_m.cpu().numpy()
        if c.vtype == "u32":
            u = u.view(np.uint32)
        elif c.vtype == "u64":
            u = u.view(np.uint64)
        words = fin.main_codes.cpu().numpy().view(np.uint64)
        sample = np.random.default_rng(j).integers(0, fin.n_main, 300)
        orig = c.u_m[[oracle.unpack(c.main_packed, i, c.w) for i in range(c.n_main)]]
        added = [v[j] for v in appended[0]]
        expect = np.concatenate([orig] + added, axis=0) if added else orig
        assert expect.shape[0] == fin.n_main
        for i in sample.tolist():
            assert np.array_equal(u[oracle.unpack(words, i, fin.w)], expect[i])
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
