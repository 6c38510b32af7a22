"""Served merge stream: resident tables, delta appends, admitted merges.

The merge of Section 3 runs online: it works on a copy, incoming updates go
to a second delta during the merge, and the merged main is committed
atomically, the second delta then becoming the primary one.  This module
keeps that protocol for many tables at once on one GPU:

* every table keeps its main partition (per column: dictionary and packed
  codes) resident in HBM, plus two delta buffers (active and second);
* appends go to the active delta (host-to-device copies on an append stream);
* a merge request is admitted when the worst-case bytes of its outputs and
  workspace (mc_merge_bounds; the old main stays alive until commit, so the
  outputs are double-buffered) fit under the memory budget; requests that do
  not fit wait in arrival order, and so do requests for a table that is
  already merging;
* at admission the active delta is frozen as the merge's snapshot and the
  second delta becomes active, so appends continue during the merge;
* admitted merges run on a pool of streams and overlap each other and the
  appends (continuous batching: a request arriving while others run is
  admitted as soon as memory and a stream are free);
* commit swaps the table's main for the merge result, frees the old main and
  clears the snapshot buffer, which becomes the next second delta;
* latency = commit time - arrival time; p50/p99 and merged tuples/s are
  reported;
* optionally the paper's merge trigger (Section 4) submits the requests
  itself: a table is merged once its delta holds more than a given fraction
  of the main's rows.

The Server logic talks to an executor (GpuExecutor here; the tests also use
a CPU executor), so admission, snapshot and commit rules are checked without
a GPU.
"""
from __future__ import annotations

import collections
import threading
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class MergeRequest:
    table: int
    arrival: float
    admitted: float | None = None
    committed: float | None = None
    rows: int = 0               # merged tuples (all columns)
    reserved: int = 0           # bytes held from admission to commit
    status: str = "queued"      # queued | running | committed | cancelled | rejected
    job: object = None
    snapshot: object = None     # the frozen delta (executor object)
    completed: float | None = None  # when the merge's last kernel ended (device clock, if known)

    @property
    def latency(self):
        return None if self.committed is None else self.committed - self.arrival

    @property
    def device_latency(self):
        """Arrival to the merge's results in HBM, on the device's clock (the
        commit itself waits for the host's next poll)."""
        return None if self.completed is None else self.completed - self.arrival


@dataclass
class TableState:
    main: object                # executor's resident main (all columns)
    active: object              # delta receiving appends
    second: object              # empty delta, becomes active at admission
    merging: MergeRequest | None = None
    merges: int = 0
    need_cap: int = 0           # worst-case merge bytes with the active delta full


class Server:
    """Admission, snapshot and commit for merges of resident tables."""

    def __init__(self, executor, budget_bytes: int, max_inflight: int = 4, clock=None,
                 merge_trigger: float | None = None):
        self.ex = executor
        self.merge_trigger = merge_trigger  # f: merge once N_D > f * N_M (None: requests only)
        self.auto_requests = 0
        self.budget = int(budget_bytes)
        self.max_inflight = max_inflight
        self.clock = clock or time.perf_counter
        self.tables: dict[int, TableState] = {}
        self.queue: collections.deque[MergeRequest] = collections.deque()
        self.running: list[MergeRequest] = []
        self.done: list[MergeRequest] = []
        self.reserved = 0
        self.peak_in_use = 0
        self.admission_waits = 0    # polls in which the head request could not be admitted
        self.backpressure = 0       # appends refused because a delta was full
        self.appended_rows = 0
        self.rejected = 0           # requests that cannot fit even with nothing running
        self.reserve = 0            # headroom kept for merges: largest merge need seen
        self.waiting_for_memory = False
        self.t0 = self.clock()
        # appends may come from another host thread than the one that polls:
        # every public call holds this lock
        self.lock = threading.RLock()

    # ---- tables and appends -------------------------------------------------

    def add_table(self, tid: int, main, delta_capacity: int):
        t = TableState(main, self.ex.new_delta(main, delta_capacity),
                       self.ex.new_delta(main, delta_capacity))
        self.tables[tid] = t
        self._refresh_need(t)
        self._note_use()

    def _refresh_need(self, t: TableState):
        t.need_cap = self.ex.merge_bytes_at(t.main, self.ex.delta_capacity(t.active))
        self.reserve = max(x.need_cap for x in self.tables.values())

    def append(self, tid: int, rows) -> bool:
        """Append a batch (executor format) to the table's active delta,
        growing it if the budget allows.  Returns False (back-pressure) if
        the delta cannot take the rows.

        Memory rule: in_use + (largest worst-case merge of any table, with its
        active delta full) <= budget.  Merge bounds only grow with the delta,
        so a request can always be admitted once nothing else runs; appends
        cannot starve the merges that would free their memory.  While a
        request waits for memory no delta grows at all."""
        with self.lock:
            return self._append(tid, rows)

    def _append(self, tid: int, rows) -> bool:
        t = self.tables[tid]
        n = self.ex.batch_rows(rows)
        grow, new_cap = self.ex.grow_plan(t.active, n)
        if grow > 0:
            if self.waiting_for_memory or new_cap is None:
                self.backpressure += 1
                return False
            need_new = self.ex.merge_bytes_at(t.main, new_cap)
            others = max((x.need_cap for x in self.tables.values() if x is not t), default=0)
            if self.in_use() + grow + max(need_new, others) > self.budget:
                self.backpressure += 1
                return False
        self.ex.append(t.active, rows)
        if grow > 0:
            self._refresh_need(t)
        self.appended_rows += n
        self._note_use()
        self._maybe_trigger(tid, t)
        return True

    def _maybe_trigger(self, tid: int, t: TableState):
        """Merge trigger of Section 4: request a merge of the table once its
        active delta holds more than merge_trigger times the main's rows (one
        request per table at a time)."""
        if self.merge_trigger is None or t.merging is not None:
            return
        if any(r.table == tid for r in self.queue):
            return
        n_main = self.ex.main_rows(t.main) / max(1, self.ex.columns(t.main))
        if self.ex.delta_rows(t.active) > self.merge_trigger * n_main:
            self.submit_merge(tid)
            self.auto_requests += 1

    # ---- requests -----------------------------------------------------------

    def submit_merge(self, tid: int) -> MergeRequest:
        with self.lock:
            r = MergeRequest(tid, self.clock())
            self.queue.append(r)
            return r

    def cancel(self, r: MergeRequest) -> bool:
        """Cancel a request that has not been admitted (nothing changes)."""
        with self.lock:
            if r.status == "queued" and r in self.queue:
                self.queue.remove(r)
                r.status = "cancelled"
                return True
            return False

    def resident_bytes(self) -> int:
        # while a table merges, its second buffer is the merge's snapshot
        total = 0
        for t in self.tables.values():
            other = t.second if t.second is not None else t.merging.snapshot
            total += (self.ex.main_bytes(t.main) + self.ex.delta_bytes(t.active)
                      + self.ex.delta_bytes(other))
        return total

    def in_use(self) -> int:
        return self.resident_bytes() + self.reserved

    def _note_use(self):
        self.peak_in_use = max(self.peak_in_use, self.in_use())

    # ---- progress -----------------------------------------------------------

    def poll(self) -> int:
        """Commit finished merges, then admit what fits.  Returns the number
        of commits."""
        with self.lock:
            return self._poll()

    def _poll(self) -> int:
        commits = 0
        still = []
        for r in self.running:
            if self.ex.finished(r.job):
                self._commit(r)
                commits += 1
            else:
                still.append(r)
        self.running = still
        self._admit()
        return commits

    def _admit(self):
        blocked_tables = set()
        waited = False
        for r in list(self.queue):
            if len(self.running) >= self.max_inflight:
                waited = True
                break
            t = self.tables[r.table]
            if t.merging is not None or r.table in blocked_tables:
                blocked_tables.add(r.table)     # one merge per table at a time
                continue
            need = self.ex.merge_bytes_at(t.main, self.ex.delta_rows(t.active))
            if self.in_use() + need > self.budget:
                if not self.running:
                    # nothing will free memory: this request can never run
                    self.queue.remove(r)
                    r.status = "rejected"
                    self.rejected += 1
                    continue
                waited = True
                break                           # arrival order: nothing overtakes
            # freeze the active delta as the snapshot, appends go to the second
            snap, t.active, t.second = t.active, t.second, None
            r.snapshot = snap
            r.reserved = need
            self.reserved += need
            r.rows = (self.ex.main_rows(t.main)
                      + self.ex.delta_rows(snap) * self.ex.columns(t.main))
            r.job = self.ex.launch(t.main, snap)
            r.admitted = self.clock()
            r.status = "running"
            t.merging = r
            self._refresh_need(t)            # the new active delta is the (small) second one
            self.queue.remove(r)
            self.running.append(r)
            self._note_use()
        self.waiting_for_memory = waited and len(self.running) < self.max_inflight
        if waited:
            self.admission_waits += 1

    def _commit(self, r: MergeRequest):
        t = self.tables[r.table]
        done = getattr(self.ex, "completion_time", None)
        r.completed = done(r.job) if done is not None else None
        new_main = self.ex.result(r.job)
        old = t.main
        t.main = new_main                       # atomic swap of the table's main
        self.ex.free_main(old)
        self.ex.clear_delta(r.snapshot)
        t.second = r.snapshot                   # the emptied snapshot is the next second delta
        t.merging = None
        t.merges += 1
        self._refresh_need(t)                # the new main is larger
        self.reserved -= r.reserved
        r.committed = self.clock()
        r.status = "committed"
        r.job = None
        self.done.append(r)
        self._note_use()

    def drain(self, timeout: float = 600.0, progress=None):
        """Run until every request is committed, rejected or the timeout
        passes; `progress(server)` is called about once a second."""
        end = self.clock() + timeout
        last = self.clock()
        while (self.queue or self.running) and self.clock() < end:
            if not self.poll():
                self.ex.idle()
            if progress is not None and self.clock() - last >= 1.0:
                last = self.clock()
                progress(self)

    # ---- statistics ------------------------------------------------------------

    def stats(self) -> dict:
        with self.lock:
            return self._stats()

    def _stats(self) -> dict:
        lat = np.array([r.latency for r in self.done], dtype=np.float64)
        wall = self.clock() - self.t0
        rows = sum(r.rows for r in self.done)
        return {
            "merges": len(self.done),
            "p50_ms": float(np.percentile(lat, 50) * 1e3) if lat.size else None,
            "p99_ms": float(np.percentile(lat, 99) * 1e3) if lat.size else None,
            "max_ms": float(lat.max() * 1e3) if lat.size else None,
            "tuples_s": rows / wall if wall > 0 else None,
            "merged_rows": rows,
            "appended_rows": self.appended_rows,
            "admission_waits": self.admission_waits,
            "backpressure": self.backpressure,
            "rejected": self.rejected,
            "auto_requests": self.auto_requests,
            "peak_in_use_bytes": self.peak_in_use,
            "budget_bytes": self.budget,
            "wall_s": wall,
        }


# ---------------------------------------------------------------------------
# GPU executor: tables resident in HBM, merges through the C ABI
# ---------------------------------------------------------------------------

@dataclass
class GpuMain:
    cols: list                   # per column: ColumnInput (u_m, codes, n_main, w, delta unused)
    nbytes: int = 0


@dataclass
class GpuDelta:
    groups: dict                 # vtype -> device tensor (n_cols_of_type, cap[, 16])
    index: list                  # per column: (vtype, row in its group)
    cap: int
    rows: int = 0
    nbytes: int = 0
    fence: object = None         # event after the last append copy
    init_cap: int = 0
    row_bytes: int = 0           # bytes of one row over all columns


class GpuExecutor:
    """Resident tables on one GPU.  Appends are host-to-device copies on an
    append stream; each admitted merge is one batched launch sequence over the
    table's columns on a stream of a pool (one whose last merge has finished,
    if any, so a short merge does not queue behind a long one), with that
    stream's own library context (a context stages a batch's descriptors in
    one host buffer, so a shared context would make each launch wait for the
    previous launch's copy on another stream); commit reads the result scalars
    once per merge."""

    def __init__(self, n_streams: int = 4, device: int = 0, plain: bool = False):
        import torch
        import paper_1109_6885_amd as cm
        self.torch, self.cm = torch, cm
        self.device = device
        # plain: each merge is one mc_merge_column call per column, in order
        # on the merge's stream with one workspace sized for its largest
        # column (the comparison of the batched form with the plain one)
        self.plain = plain
        self.t0_event = None  # device-clock origin for completion times
        self.append_stream = torch.cuda.Stream(device=device)
        self.streams = [torch.cuda.Stream(device=device) for _ in range(n_streams)]
        self.ctxs = [cm.Context(device) for _ in range(n_streams)]
        self.last_done = [None] * n_streams  # event of each stream's last merge
        self.next = 0
        self.ctx = cm.context(device)  # default tuning, for the bounds

    # mains
    def make_main(self, cols) -> GpuMain:
        nb = sum(c.u_m.numel() * c.u_m.element_size() + c.main_codes.numel() * 8 for c in cols)
        return GpuMain(cols, nb)

    def main_bytes(self, m): return m.nbytes
    def main_rows(self, m): return sum(c.n_main for c in m.cols)
    def columns(self, m): return len(m.cols)
    def free_main(self, m): m.cols = []

    # deltas
    def _alloc_groups(self, counts, cap):
        torch = self.torch
        groups, nb = {}, 0
        for vt, n in counts.items():
            shape = (n, cap, 16) if vt == "str16" else (n, cap)
            dt = {"u32": torch.int32, "u64": torch.int64, "str16": torch.uint8}[vt]
            groups[vt] = torch.empty(shape, dtype=dt, device=f"cuda:{self.device}")
            nb += groups[vt].numel() * groups[vt].element_size()
        return groups, nb

    def new_delta(self, m: GpuMain, cap: int) -> GpuDelta:
        counts = collections.Counter(c.vtype for c in m.cols)
        groups, nb = self._alloc_groups(counts, cap)
        index, seen = [], collections.Counter()
        for c in m.cols:
            index.append((c.vtype, seen[c.vtype]))
            seen[c.vtype] += 1
        row_bytes = sum(self.cm.VALUE_LEN[c.vtype] for c in m.cols)
        return GpuDelta(groups, index, cap, 0, nb, None, cap, row_bytes)

    def delta_rows(self, d): return d.rows
    def delta_capacity(self, d): return d.cap
    def delta_bytes(self, d): return d.nbytes
    def batch_rows(self, rows): return rows["n"]

    def grow_plan(self, d: GpuDelta, n: int):
        """(bytes to allocate, new capacity) for appending n rows; (0, cap) if
        they fit."""
        if d.rows + n <= d.cap:
            return 0, d.cap
        new_cap = max(2 * d.cap, d.rows + n)
        if new_cap >= (1 << 30):
            return 1, None                     # past the library's delta limit
        return (new_cap - d.cap) * d.row_bytes, new_cap

    def append(self, d: GpuDelta, rows):
        """rows: {"n": r, vtype: pinned host tensor (n_cols_of_type, r[, 16])}.
        Doubles the delta's capacity first when needed."""
        n = rows["n"]
        torch = self.torch
        with torch.cuda.stream(self.append_stream):
            if d.rows + n > d.cap:
                new_cap = max(2 * d.cap, d.rows + n)
                counts = {vt: g.shape[0] for vt, g in d.groups.items()}
                groups, nb = self._alloc_groups(counts, new_cap)
                for vt, g in d.groups.items():
                    groups[vt][:, :d.rows].copy_(g[:, :d.rows], non_blocking=True)
                    g.record_stream(self.append_stream)
                d.groups, d.cap, d.nbytes = groups, new_cap, nb
            for vt, g in d.groups.items():
                g[:, d.rows:d.rows + n].copy_(rows[vt], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.append_stream)
        d.fence = ev
        d.rows += n
        return True

    def clear_delta(self, d: GpuDelta):
        """Empty the delta; a grown buffer shrinks back to its first size."""
        d.rows = 0
        if d.cap > d.init_cap:
            for g in d.groups.values():
                g.record_stream(self.append_stream)
            counts = {vt: g.shape[0] for vt, g in d.groups.items()}
            d.groups, d.nbytes = self._alloc_groups(counts, d.init_cap)
            d.cap = d.init_cap
        d.fence = None

    def _inputs(self, m: GpuMain, d: GpuDelta):
        out = []
        for c, (vt, i) in zip(m.cols, d.index):
            delta = d.groups[vt][i, :d.rows]
            out.append(self.cm.ColumnInput(c.vtype, c.u_m, c.main_codes, c.n_main, c.w, delta))
        return out

    def merge_bytes_at(self, m: GpuMain, rows: int) -> int:
        """Worst-case bytes of merging `rows` delta rows into main m: every
        column's U' and codes capacity (mc_merge_bounds) plus the batched
        workspace (mc_merge_batched_bounds).  Host-only arithmetic in the
        library; cached per (main, rows)."""
        key = (id(m), rows)
        cache = m.__dict__.setdefault("_need", {})
        if key in cache:
            return cache[key]
        cm = self.cm
        ins = []
        total = 0
        plain_scratch = 0
        for c in m.cols:
            d = cm.McColumnIn()
            d.type = cm.TYPE_CODES[c.vtype]
            d.bitwidth = c.w
            d.main_dict = 256 if c.u_m.numel() else None     # sizing never reads memory
            d.main_dict_len = int(c.u_m.shape[0])
            d.main_codes = 256 if c.n_main else None
            d.main_rows = c.n_main
            d.delta_values = 256 if rows else None
            d.delta_rows = rows
            ins.append(d)
            dc, words, sb = cm.bounds_of(d)
            total += dc * cm.VALUE_LEN[c.vtype] + max(words, 2) * 8 + cm.RESULT_BYTES
            plain_scratch = max(plain_scratch, sb)
        # the workspace each route really needs: one column at a time (plain)
        # or every column at once (batched)
        total += plain_scratch if self.plain else cm.batched_bounds_of(ins, self.ctx)
        if len(cache) > 64:
            cache.clear()
        cache[key] = total
        return total

    def _pick_stream(self) -> int:
        n = len(self.streams)
        for k in range(n):
            i = (self.next + k) % n
            e = self.last_done[i]
            if e is None or e.query():
                return i
        return self.next % n

    def launch(self, m: GpuMain, d: GpuDelta):
        torch, cm = self.torch, self.cm
        si = self._pick_stream()
        self.next = si + 1
        s = self.streams[si]
        cols = self._inputs(m, d)
        descs = [c.descriptor() for c in cols]  # built once for the bounds and the launch
        # (one allocation per column's U' and codes: the caching allocator
        # reuses those; one allocation of all of them, gigabytes that rarely
        # fit a cached block, went to the device allocator and stalled merges)
        with torch.cuda.stream(s):
            if d.fence is not None:
                s.wait_event(d.fence)          # the snapshot's appends have landed
            res = torch.zeros(len(cols) * cm.RESULT_BYTES, dtype=torch.uint8,
                              device=f"cuda:{self.device}")
            outs = []
            for j, (col, desc) in enumerate(zip(cols, descs)):
                dict_cap, words, _ = cm.bounds_of(desc)
                outs.append(cm.MergeOutput(
                    col.vtype, cm.value_tensor_empty(col.vtype, dict_cap),
                    torch.empty(max(words, 2), dtype=torch.int64, device=f"cuda:{self.device}"),
                    None, None, res[j * cm.RESULT_BYTES:(j + 1) * cm.RESULT_BYTES],
                    col.n_main + int(col.delta.shape[0])))
            if self.plain:
                scratch = cm.alloc_scratch(max(cm.bounds_of(dd)[2] for dd in descs))
                for col, out in zip(cols, outs):
                    cm.merge_column(col, out=out, scratch=scratch, stream=s, ctx=self.ctxs[si])
            else:
                scratch = cm.alloc_scratch(cm.batched_bounds_of(descs, self.ctx))
                cm.merge_columns_batched(cols, outs=outs, scratch=scratch, stream=s,
                                         ctx=self.ctxs[si], descs=descs)
            done = torch.cuda.Event(enable_timing=self.t0_event is not None)
            done.record(s)
            self.last_done[si] = done
        return {"cols": cols, "outs": outs, "res": res, "scratch": scratch, "done": done,
                "stream": s}

    def finished(self, job) -> bool:
        return job["done"].query()

    def start_clock(self, host_now: float):
        """Record the device-clock origin (after a synchronize) matching the
        host clock reading host_now: completion times are then host-clock
        seconds of the merges' last kernels."""
        torch = self.torch
        torch.cuda.synchronize(self.device)
        self.t0_event = torch.cuda.Event(enable_timing=True)
        self.t0_event.record(torch.cuda.current_stream(self.device))
        self.t0_event.synchronize()
        self.t0_host = host_now

    def completion_time(self, job):
        if self.t0_event is None:
            return None
        return self.t0_host + self.t0_event.elapsed_time(job["done"]) / 1e3

    def result(self, job) -> GpuMain:
        cm = self.cm
        raw = job["res"].cpu().numpy()
        new_cols = []
        for j, (col, out) in enumerate(zip(job["cols"], job["outs"])):
            r = cm.McResult.from_buffer_copy(raw[j * cm.RESULT_BYTES:(j + 1) * cm.RESULT_BYTES].tobytes())
            if r.error:
                raise RuntimeError(f"merge of column {j} reported device error {r.error}")
            rows = col.n_main + int(col.delta.shape[0])
            new_cols.append(cm.ColumnInput(col.vtype, out.new_dict[: r.new_dict_len],
                                           out.new_codes, rows, int(r.new_bitwidth), None))
        job["scratch"] = None
        return self.make_main(new_cols)

    def idle(self):
        time.sleep(0.0002)


# ---------------------------------------------------------------------------
# Helpers for building resident tables and append batches
# ---------------------------------------------------------------------------

def gpu_main_from_columns(ex: GpuExecutor, cols) -> GpuMain:
    """Resident main from host columns (workloads.Column, delta ignored)."""
    cm = ex.cm
    dcols = [cm.ColumnInput(c.vtype, cm.to_device(c.u_m), cm.to_device(c.main_packed), c.n_main,
                            c.w, None) for c in cols]
    return ex.make_main(dcols)


def append_batch(ex: GpuExecutor, main: GpuMain, values_by_type: dict, n: int) -> dict:
    """An append batch of n rows for every column of `main`: values_by_type
    maps a value type to a host array (columns of that type, n[, 16]), which
    is copied into pinned memory once."""
    torch = ex.torch
    out = {"n": n}
    for vt, arr in values_by_type.items():
        a = np.ascontiguousarray(arr)
        if a.dtype == np.uint32:
            a = a.view(np.int32)
        elif a.dtype == np.uint64:
            a = a.view(np.int64)
        out[vt] = torch.from_numpy(a).pin_memory()
    return out
