"""Serving logic without a GPU: the Server's admission, snapshot (second
delta), commit and statistics rules, driven through a CPU executor whose
merges are the oracle's and which finishes a merge only after a set number
of polls (so merges are in flight while appends and requests arrive)."""
import numpy as np
import pytest

import oracle
from paper_1109_6885_amd.serve import Server
from workloads import gen


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 0.001
        return self.t


class CpuMain:
    def __init__(self, cols):
        self.cols = cols  # list of dict(vtype, u_m, codes, n_main, w)


class CpuDelta:
    def __init__(self, ncols, cap):
        self.vals = [[] for _ in range(ncols)]
        self.cap = cap
        self.rows = 0


class CpuExecutor:
    def __init__(self, polls_to_finish=3):
        self.k = polls_to_finish
        self.launched = []

    def main_bytes(self, m):
        return sum(c["u_m"].nbytes + c["codes"].nbytes for c in m.cols)

    def main_rows(self, m):
        return sum(c["n_main"] for c in m.cols)

    def columns(self, m):
        return len(m.cols)

    def free_main(self, m):
        m.cols = []

    def new_delta(self, m, cap):
        return CpuDelta(len(m.cols), cap)

    def delta_rows(self, d):
        return d.rows

    def delta_capacity(self, d):
        return d.cap

    def delta_bytes(self, d):
        return d.cap * 16 * len(d.vals)

    def batch_rows(self, rows):
        return rows["n"]

    def grow_plan(self, d, n):
        # fixed capacity here: a full delta cannot grow (back-pressure)
        if d.rows + n <= d.cap:
            return 0, d.cap
        return 1, None

    def append(self, d, rows):
        for j, v in enumerate(rows["cols"]):
            d.vals[j].extend(list(v))
        d.rows += rows["n"]
        return True

    def clear_delta(self, d):
        d.vals = [[] for _ in d.vals]
        d.rows = 0

    def merge_bytes_at(self, m, rows):
        return sum((c["u_m"].shape[0] + rows) * 16 + (c["n_main"] + rows) * 4 + 4096
                   for c in m.cols)

    def merge_bytes(self, m, d):
        return self.merge_bytes_at(m, d.rows)

    def launch(self, m, d):
        job = {"m": m, "snap": [list(v) for v in d.vals], "polls": 0}
        self.launched.append(job)
        return job

    def finished(self, job):
        job["polls"] += 1
        return job["polls"] >= self.k

    def result(self, job):
        cols = []
        for c, vals in zip(job["m"].cols, job["snap"]):
            vt = c["vtype"]
            delta = (np.array(vals, np.uint8).reshape(-1, 16) if vt == "str16"
                     else np.array(vals, dtype=np.uint32 if vt == "u32" else np.uint64))
            r = oracle.merge_column(vt, c["u_m"], c["codes"], c["n_main"], c["w"], delta)
            cols.append({"vtype": vt, "u_m": r["u_new"], "codes": r["codes"],
                         "n_main": c["n_main"] + len(vals), "w": r["w_new"]})
        return CpuMain(cols)

    def idle(self):
        pass


def decode(c):
    codes = [oracle.unpack(c["codes"], i, c["w"]) for i in range(c["n_main"])]
    return [c["u_m"][k].tobytes() if c["vtype"] == "str16" else int(c["u_m"][k]) for k in codes]


def make_table(rng, ncols=3, rows=200):
    cols = []
    for j in range(ncols):
        vt = ("u32", "u64", "str16")[j % 3]
        col = gen.random_column(rng, vt, 20, rows, 0)
        cols.append({"vtype": vt, "u_m": col.u_m, "codes": col.main_packed, "n_main": rows,
                     "w": col.w})
    return CpuMain(cols)


def batch(rng, m, n):
    vals = []
    for c in m.cols:
        vals.append(list(gen.random_values(rng, c["vtype"], n)))
    return {"n": n, "cols": vals}


def test_snapshot_second_delta_and_commit():
    rng = np.random.default_rng(0)
    ex = CpuExecutor(polls_to_finish=4)
    s = Server(ex, budget_bytes=10 ** 9, clock=FakeClock())
    m = make_table(rng)
    expected = [decode(c) for c in m.cols]
    s.add_table(0, m, delta_capacity=1000)
    b1 = batch(rng, m, 50)
    assert s.append(0, b1)
    r1 = s.submit_merge(0)
    s.poll()
    assert r1.status == "running"
    # appends during the merge go to the second delta, not the snapshot
    b2 = batch(rng, m, 30)
    assert s.append(0, b2)
    assert len(ex.launched[0]["snap"][0]) == 50
    r2 = s.submit_merge(0)          # waits: one merge per table
    s.poll()
    assert r2.status == "queued"
    s.drain()
    assert r1.status == r2.status == "committed"
    assert r1.committed <= r2.admitted
    final = s.tables[0].main
    for j, c in enumerate(final.cols):
        vt = c["vtype"]
        add = [(bytes(np.asarray(v, np.uint8)) if vt == "str16" else int(v))
               for v in b1["cols"][j] + b2["cols"][j]]
        assert decode(c) == expected[j] + add
    st = s.stats()
    assert st["merges"] == 2 and st["p50_ms"] is not None and st["merged_rows"] == 3 * (250 + 280)


def test_budget_never_exceeded_and_fifo():
    rng = np.random.default_rng(1)
    ex = CpuExecutor(polls_to_finish=5)
    s = Server(ex, budget_bytes=10 ** 12, max_inflight=8, clock=FakeClock())
    for t in range(4):
        m = make_table(rng, 2, 100)
        s.add_table(t, m, delta_capacity=1000)
        s.append(t, batch(rng, m, 200))
    needs = [ex.merge_bytes(s.tables[t].main, s.tables[t].active) for t in range(4)]
    # room for the first two merges and half of the third
    s.budget = s.in_use() + needs[0] + needs[1] + needs[2] // 2
    reqs = [s.submit_merge(t) for t in range(4)]
    s.poll()
    assert [r.status for r in reqs] == ["running", "running", "queued", "queued"]
    assert s.admission_waits == 1
    peak = 0
    while s.queue or s.running:
        s.poll()
        peak = max(peak, s.in_use())
        assert s.in_use() <= s.budget
        # nothing overtakes the head of the queue
        if reqs[2].status == "queued":
            assert reqs[3].status == "queued"
    assert all(r.status == "committed" for r in reqs)
    assert reqs[2].admitted >= min(reqs[0].committed, reqs[1].committed)
    assert s.peak_in_use <= s.budget


def test_many_tables_random_traffic_stays_in_budget():
    rng = np.random.default_rng(11)
    ex = CpuExecutor(polls_to_finish=4)
    s = Server(ex, budget_bytes=10 ** 12, max_inflight=3, clock=FakeClock())
    for t in range(5):
        s.add_table(t, make_table(rng, 2, 60), delta_capacity=400)
    s.budget = s.in_use() + 150_000
    reqs = []
    for step in range(80):
        t = int(rng.integers(0, 5))
        s.append(t, batch(rng, s.tables[t].main, 5))
        if step % 4 == 0:
            reqs.append(s.submit_merge(int(rng.integers(0, 5))))
        s.poll()
        assert s.in_use() <= s.budget
    s.drain()
    assert all(r.status == "committed" for r in reqs)
    assert s.peak_in_use <= s.budget
    st = s.stats()
    assert st["merges"] == len(reqs) and st["p99_ms"] >= st["p50_ms"]


def test_cancel_queued_request_changes_nothing():
    rng = np.random.default_rng(2)
    ex = CpuExecutor()
    s = Server(ex, budget_bytes=10 ** 9, clock=FakeClock())
    m = make_table(rng)
    before = [decode(c) for c in m.cols]
    s.add_table(0, m, 100)
    s.append(0, batch(rng, m, 10))
    r = s.submit_merge(0)
    assert s.cancel(r) and r.status == "cancelled"
    s.drain()
    assert [decode(c) for c in s.tables[0].main.cols] == before
    assert s.tables[0].active.rows == 10    # the delta keeps its rows


def test_backpressure_when_delta_full():
    rng = np.random.default_rng(3)
    ex = CpuExecutor()
    s = Server(ex, budget_bytes=10 ** 9, clock=FakeClock())
    m = make_table(rng)
    s.add_table(0, m, 40)
    assert s.append(0, batch(rng, m, 30))
    assert not s.append(0, batch(rng, m, 30))
    assert s.stats()["backpressure"] == 1


def test_request_that_can_never_fit_is_rejected():
    rng = np.random.default_rng(4)
    ex = CpuExecutor()
    s = Server(ex, budget_bytes=1, clock=FakeClock())    # nothing fits
    m = make_table(rng)
    s.add_table(0, m, 10)
    r = s.submit_merge(0)
    s.poll()
    assert r.status == "rejected" and s.stats()["rejected"] == 1


def test_appends_cannot_starve_waiting_merges():
    """While a request waits for memory, deltas may not grow; and growth
    always leaves room for the largest merge seen."""
    rng = np.random.default_rng(6)

    class Growing(CpuExecutor):
        def grow_plan(self, d, n):
            if d.rows + n <= d.cap:
                return 0, d.cap
            return (d.rows + n - d.cap) * 64, d.rows + n

        def append(self, d, rows):
            d.cap = max(d.cap, d.rows + rows["n"])
            return super().append(d, rows)

    ex = Growing(polls_to_finish=6)
    s = Server(ex, budget_bytes=10 ** 12, max_inflight=4, clock=FakeClock())
    for t in range(3):
        s.add_table(t, make_table(rng, 2, 50), delta_capacity=10)
        s.append(t, batch(rng, s.tables[t].main, 10))
    needs = [ex.merge_bytes(s.tables[t].main, s.tables[t].active) for t in range(3)]
    s.budget = s.in_use() + needs[0] + needs[1] // 2
    assert s.reserve == max(s.tables[t].need_cap for t in range(3))
    r0, r1 = s.submit_merge(0), s.submit_merge(1)
    s.poll()
    assert r0.status == "running" and r1.status == "queued" and s.waiting_for_memory
    bp = s.backpressure
    assert not s.append(2, batch(rng, s.tables[2].main, 50))    # growth refused
    assert s.backpressure == bp + 1
    s.drain()
    assert r1.status == "committed"
    assert s.peak_in_use <= s.budget


def test_growth_keeps_room_for_the_largest_merge():
    rng = np.random.default_rng(8)

    class Growing(CpuExecutor):
        def grow_plan(self, d, n):
            if d.rows + n <= d.cap:
                return 0, d.cap
            return (2 * d.cap - d.cap) * 64, 2 * d.cap

        def append(self, d, rows):
            if d.rows + rows["n"] > d.cap:
                d.cap *= 2
            return super().append(d, rows)

        def delta_bytes(self, d):
            return d.cap * 64

    ex = Growing(polls_to_finish=3)
    s = Server(ex, budget_bytes=10 ** 12, clock=FakeClock())
    for t in range(3):
        s.add_table(t, make_table(rng, 2, 40), delta_capacity=8)
    s.budget = s.in_use() + 3 * s.reserve
    refused = 0
    for step in range(300):
        t = step % 3
        if not s.append(t, batch(rng, s.tables[t].main, 4)):
            refused += 1
        # the rule: whatever is in use, the largest possible merge still fits
        assert s.in_use() + s.reserve <= s.budget
    assert refused > 0
    reqs = [s.submit_merge(t) for t in range(3)]
    s.drain()
    assert all(r.status == "committed" for r in reqs) and s.rejected == 0


def test_merge_trigger_fraction_of_main():
    """Section 4's trigger: a merge is requested once the delta holds more
    than f * N_M rows, once per table at a time, and the merged table holds
    every appended row in order."""
    rng = np.random.default_rng(21)
    ex = CpuExecutor(polls_to_finish=2)
    s = Server(ex, budget_bytes=10 ** 12, clock=FakeClock(), merge_trigger=0.1)
    m = make_table(rng, 2, 200)       # N_M = 200 rows: trigger above 20 delta rows
    expected = [decode(c) for c in m.cols]
    shape = CpuMain([dict(c) for c in m.cols])  # batches keep the column types after commits
    s.add_table(0, m, delta_capacity=1000)
    batches = []
    for n in (10, 10):                 # 20 rows: not above 20
        batches.append(batch(rng, shape, n))
        assert s.append(0, batches[-1])
    assert not s.queue and s.auto_requests == 0
    batches.append(batch(rng, shape, 1))   # 21 rows: requested
    assert s.append(0, batches[-1])
    assert len(s.queue) == 1 and s.auto_requests == 1
    batches.append(batch(rng, shape, 5))   # still queued: no second request
    assert s.append(0, batches[-1])
    assert len(s.queue) == 1 and s.auto_requests == 1
    s.poll()                           # admitted: the active delta is the empty second one
    assert s.running and s.tables[0].merging is not None
    batches.append(batch(rng, shape, 30))  # above 0.1 * 200, but the table is merging
    assert s.append(0, batches[-1])
    assert s.auto_requests == 1
    s.drain()
    batches.append(batch(rng, shape, 1))   # N_M is now 226: 31 rows > 22.6 -> requested again
    assert s.append(0, batches[-1])
    assert s.auto_requests == 2
    s.drain()
    final = s.tables[0].main
    for j, c in enumerate(final.cols):
        vt = c["vtype"]
        add = [(bytes(np.asarray(v, np.uint8)) if vt == "str16" else int(v))
               for b in batches for v in b["cols"][j]]
        assert decode(c) == expected[j] + add
    assert s.stats()["auto_requests"] == 2


def test_appends_from_another_thread():
    """Appends from a host thread of their own while the merge loop polls
    (the served benchmark's arrangement): every public call holds the
    server's lock, so the two threads never see a table half-updated; every
    row that was accepted is in the final tables, in order, and the budget
    holds throughout."""
    import threading
    import time

    rng = np.random.default_rng(23)
    ex = CpuExecutor(polls_to_finish=3)
    s = Server(ex, budget_bytes=10 ** 12, max_inflight=3)
    tables = {t: make_table(rng, 2, 40) for t in range(3)}
    expected = {t: [decode(c) for c in m.cols] for t, m in tables.items()}
    for t, m in tables.items():
        s.add_table(t, m, delta_capacity=500)
    batches = {t: [batch(rng, tables[t], 5) for _ in range(40)] for t in tables}
    accepted = {t: [] for t in tables}
    errors = []

    def appender():
        try:
            for k in range(40):
                for t in tables:
                    if s.append(t, batches[t][k]):
                        accepted[t].append(batches[t][k])
                time.sleep(0.0005)
        except Exception as e:  # reported by the main thread
            errors.append(e)

    th = threading.Thread(target=appender)
    th.start()
    reqs = []
    while th.is_alive():
        reqs.append(s.submit_merge(int(rng.integers(0, 3))))
        s.poll()
        with s.lock:
            assert s.in_use() <= s.budget
        time.sleep(0.0003)
    th.join()
    assert not errors, errors
    for t in tables:
        reqs.append(s.submit_merge(t))
    s.drain()
    assert all(r.status == "committed" for r in reqs)
    for t, m in tables.items():
        for j, c in enumerate(s.tables[t].main.cols):
            vt = c["vtype"]
            add = [(bytes(np.asarray(v, np.uint8)) if vt == "str16" else int(v))
                   for b in accepted[t] for v in b["cols"][j]]
            assert decode(c) == expected[t][j] + add
