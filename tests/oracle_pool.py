"""Oracle merges of the batched workload's columns in worker processes.

The oracle is single-threaded by design (its sort keeps the comparator's
state in file-scope variables), so parallel oracle runs use processes, not
threads.  A worker regenerates its column from the column's own seed (the
same bytes the parent generated), merges it with the oracle and returns the
scalars plus SHA-256 digests of U' and of the W' result words, so that only
a few bytes travel back; equal digests mean equal bytes."""
from __future__ import annotations

import hashlib

import numpy as np

import oracle
from workloads import gen


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def oracle_digest(shape) -> dict:
    """shape: one entry of gen.batched_shapes()."""
    col = gen._batched_one(shape)
    ref = oracle.merge_column(col.vtype, col.u_m, col.main_packed, col.n_main, col.w, col.delta)
    return {"n_new": ref["n_new"], "w_new": ref["w_new"], "n_words": ref["n_words"],
            "u_new": digest(ref["u_new"]), "codes": digest(ref["codes"])}
