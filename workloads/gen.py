"""Seeded generators for merge inputs (see package docstring).

Seeds: numpy PCG64 with base seed 11096885.  Configuration k uses seed
BASE_SEED + k; column c of the batched configuration uses
BASE_SEED + 1000 * 4 + c.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

BASE_SEED = 11096885

CONFIG_NAMES = {
    1: "c1: 1M-row u64 column, 10k-entry dictionary, 14-bit codes, 10k delta (50% new)",
    2: "c2: 100M-row u64 column, 1.048M-entry dictionary, 20-bit codes, 1M delta (90% new), width 20->21",
    3: "c3: 100M-row 16-byte string column, 10M-entry dictionary, Zipf 1.1, 24-bit codes, 10M delta (30% of rows from new values)",
    4: "c4: 300 columns, rows log-uniform [1M, 20M], distinct log-uniform [2, 10M], u32/u64/str16, delta 1% (50% new)",
}

_ELEM_DTYPE = {"u32": np.uint32, "u64": np.uint64}


@dataclass
class Column:
    """Inputs of one column merge."""
    vtype: str                 # "u32" | "u64" | "str16"
    u_m: np.ndarray            # sorted unique main dictionary
    main_packed: np.ndarray    # uint64 words, codes at width w
    n_main: int
    w: int
    delta: np.ndarray          # delta values in append order
    meta: dict = field(default_factory=dict)

    @property
    def n_delta(self) -> int:
        return int(self.delta.shape[0])

    @property
    def value_len(self) -> int:
        return {"u32": 4, "u64": 8, "str16": 16}[self.vtype]


# ---------------------------------------------------------------------------
# Value helpers
# ---------------------------------------------------------------------------

def _str_order(a: np.ndarray) -> np.ndarray:
    """Argsort of 16-byte strings in unsigned byte order (big-endian halves).
    Sorting by the high half alone is exact unless two strings share their
    first 8 bytes; only then the two-key sort runs."""
    halves = np.ascontiguousarray(a, dtype=np.uint8).view(">u8").reshape(-1, 2)
    hi = halves[:, 0].astype(np.uint64)
    order = np.argsort(hi, kind="stable")
    hs = hi[order]
    if hs.shape[0] > 1 and np.any(hs[1:] == hs[:-1]):
        lo = halves[:, 1].astype(np.uint64)
        return np.lexsort((lo, hi))
    return order


def _str_keys(a: np.ndarray):
    halves = np.ascontiguousarray(a, dtype=np.uint8).view(">u8").reshape(-1, 2)
    return halves[:, 0].astype(np.uint64), halves[:, 1].astype(np.uint64)


def sort_unique_values(vals: np.ndarray, vtype: str) -> np.ndarray:
    """Sorted distinct values (the input format of a main dictionary)."""
    if vtype != "str16":
        return np.unique(vals)
    if vals.shape[0] == 0:
        return vals.reshape(0, 16).copy()
    order = _str_order(vals)
    s = vals[order]
    keep = np.ones(s.shape[0], dtype=bool)
    keep[1:] = np.any(s[1:] != s[:-1], axis=1)
    return np.ascontiguousarray(s[keep])


def random_values(rng: np.random.Generator, vtype: str, n: int,
                  u64_high: int = 2 ** 63) -> np.ndarray:
    """n values drawn uniformly (not necessarily distinct)."""
    if vtype == "u32":
        return rng.integers(0, 2 ** 32, size=n, dtype=np.uint64).astype(np.uint32)
    if vtype == "u64":
        if u64_high >= 2 ** 64:
            return rng.integers(0, 2 ** 64, size=n, dtype=np.uint64, endpoint=False)
        return rng.integers(0, u64_high, size=n, dtype=np.uint64)
    # printable ASCII bytes 0x20..0x7E
    return rng.integers(0x20, 0x7F, size=(n, 16), dtype=np.uint8)


def _member(x: np.ndarray, ref_sorted: np.ndarray, vtype: str) -> np.ndarray:
    """Boolean mask: which entries of x occur in the sorted distinct ref."""
    if x.shape[0] == 0:
        return np.zeros(0, dtype=bool)
    if ref_sorted is None or ref_sorted.shape[0] == 0:
        return np.zeros(x.shape[0], dtype=bool)
    if vtype != "str16":
        idx = np.searchsorted(ref_sorted, x)
        idx = np.minimum(idx, ref_sorted.shape[0] - 1)
        return ref_sorted[idx] == x
    # strings: sort both together, tag the reference, look for equal neighbours
    allv = np.concatenate([ref_sorted, x], axis=0)
    tag = np.concatenate([np.zeros(ref_sorted.shape[0], np.int8),
                          np.ones(x.shape[0], np.int8)])
    hi, lo = _str_keys(allv)
    order = np.lexsort((tag, lo, hi))          # reference before x on ties
    hs, ls, ts = hi[order], lo[order], tag[order]
    # for each x entry, it is a member iff the last reference entry with the
    # same key exists: propagate "key of last reference seen" forward
    is_ref = ts == 0
    ref_pos = np.where(is_ref, np.arange(order.shape[0]), -1)
    ref_pos = np.maximum.accumulate(ref_pos)
    ok = ref_pos >= 0
    same = np.zeros(order.shape[0], dtype=bool)
    rp = ref_pos[ok]
    same[ok] = (hs[rp] == hs[ok]) & (ls[rp] == ls[ok])
    res = np.zeros(x.shape[0], dtype=bool)
    xs = ~is_ref
    res[order[xs] - ref_sorted.shape[0]] = same[xs]
    return res


def distinct_values(rng: np.random.Generator, vtype: str, n: int,
                    exclude: np.ndarray | None = None,
                    u64_high: int = 2 ** 63) -> np.ndarray:
    """n distinct values, none of them in the sorted array `exclude`,
    in random order."""
    if vtype == "u32" and n > 2 ** 31:
        raise ValueError("too many distinct u32 values requested")
    got = None
    want = n
    while True:
        draw = random_values(rng, vtype, int(want * 1.05) + 16, u64_high)
        if exclude is not None:
            draw = draw[~_member(draw, exclude, vtype)]
        pool = draw if got is None else np.concatenate([got, draw], axis=0)
        got = sort_unique_values(pool, vtype)
        if got.shape[0] >= n:
            break
        want = n - got.shape[0]
    pick = rng.permutation(got.shape[0])[:n]
    return np.ascontiguousarray(got[pick])


def code_width(k: int) -> int:
    """Bits for codes of a k-entry dictionary (input encoding, >= 1)."""
    return max(1, int(k - 1).bit_length()) if k > 1 else 1


# ---------------------------------------------------------------------------
# Packed code vectors (input encoding: LSB-first 64-bit words)
# ---------------------------------------------------------------------------

def pack_codes(codes: np.ndarray, w: int, chunk_groups: int = 1 << 20) -> np.ndarray:
    """Pack codes (< 2^w) at width w: code i at stream bits [i*w, (i+1)*w),
    least significant bit first, stream bit b = bit b%64 of word b//64.
    Works on groups of 64 codes, which fill exactly w words."""
    codes = np.asarray(codes).reshape(-1)
    n = codes.shape[0]
    nwords = (n * w + 63) // 64
    ngroups = (n + 63) // 64
    out = np.zeros(ngroups * w, dtype=np.uint64)
    mask = np.uint64((1 << w) - 1)
    for g0 in range(0, ngroups, chunk_groups):
        g1 = min(ngroups, g0 + chunk_groups)
        c = np.zeros((g1 - g0) * 64, dtype=np.uint64)
        src = codes[g0 * 64: min(n, g1 * 64)].astype(np.uint64)
        c[: src.shape[0]] = src & mask
        c = c.reshape(-1, 64)
        o = out[g0 * w: g1 * w].reshape(-1, w)
        for j in range(64):
            off = j * w
            word, sh = off >> 6, off & 63
            o[:, word] |= c[:, j] << np.uint64(sh)
            if sh + w > 64:
                o[:, word + 1] |= c[:, j] >> np.uint64(64 - sh)
    return out[:nwords]


# ---------------------------------------------------------------------------
# Column generators
# ---------------------------------------------------------------------------

def _zipf_codes(rng, n: int, k: int, s: float, rank_to_code: np.ndarray) -> np.ndarray:
    """n i.i.d. draws of a bounded Zipf(s) over k ranks, mapped to codes.
    Drawn as multinomial counts per rank, then shuffled (same law as
    independent draws)."""
    p = np.arange(1, k + 1, dtype=np.float64) ** (-s)
    p /= p.sum()
    counts = rng.multinomial(n, p)
    out = np.repeat(rank_to_code.astype(np.uint32), counts)
    rng.shuffle(out)
    return out


def random_column(rng: np.random.Generator, vtype: str, n_um: int, n_main: int,
                  n_delta: int, frac_new: float = 0.5, w: int | None = None,
                  zipf_s: float | None = None, new_pool: int | None = None,
                  u64_high: int = 2 ** 63) -> Column:
    """A column with an n_um-entry dictionary, n_main uniform (or Zipf) codes
    and n_delta delta rows, round(frac_new * n_delta) of them new values
    (distinct unless new_pool bounds the pool they are drawn from)."""
    u_m = distinct_values(rng, vtype, n_um, None, u64_high)
    u_m = sort_unique_values(u_m, vtype)
    if w is None:
        w = code_width(n_um)
    # with Zipf frequencies, the same random rank -> code map serves the
    # main rows and the delta rows drawn from the main dictionary
    perm = rng.permutation(n_um) if (zipf_s is not None and n_um > 0) else None
    if n_main > 0:
        if n_um == 0:
            raise ValueError("rows need a dictionary")
        if zipf_s is None:
            codes = rng.integers(0, n_um, size=n_main, dtype=np.uint64).astype(np.uint32)
        else:
            codes = _zipf_codes(rng, n_main, n_um, zipf_s, perm)
    else:
        codes = np.zeros(0, np.uint32)
    packed = pack_codes(codes, w)
    n_new = int(round(frac_new * n_delta))
    n_old = n_delta - n_new
    if n_old > 0 and n_um == 0:
        n_new, n_old = n_delta, 0
    parts = []
    if n_old > 0:
        if zipf_s is None:
            idx = rng.integers(0, n_um, size=n_old)
        else:
            idx = _zipf_codes(rng, n_old, n_um, zipf_s, perm)
        parts.append(u_m[idx])
    if n_new > 0:
        pool_n = n_new if new_pool is None else new_pool
        pool = distinct_values(rng, vtype, pool_n, u_m, u64_high)
        if new_pool is None:
            parts.append(pool)
        else:
            if zipf_s is None:
                idx = rng.integers(0, pool_n, size=n_new)
            else:
                idx = _zipf_codes(rng, n_new, pool_n, zipf_s, rng.permutation(pool_n))
            parts.append(pool[idx])
    if parts:
        delta = np.concatenate(parts, axis=0)
        delta = np.ascontiguousarray(delta[rng.permutation(delta.shape[0])])
    else:
        delta = (np.zeros((0, 16), np.uint8) if vtype == "str16"
                 else np.zeros(0, _ELEM_DTYPE[vtype]))
    return Column(vtype, np.ascontiguousarray(u_m), packed, n_main, w, delta,
                  {"n_new_rows": n_new, "n_old_rows": n_old})


def config_column(k: int) -> Column:
    """The single-column workload configurations 1, 2 and 3."""
    rng = np.random.default_rng(BASE_SEED + k)
    if k == 1:
        col = random_column(rng, "u64", 10_000, 1_000_000, 10_000, 0.5, w=14)
    elif k == 2:
        col = random_column(rng, "u64", 1_048_000, 100_000_000, 1_000_000, 0.9, w=20)
    elif k == 3:
        col = random_column(rng, "str16", 10_000_000, 100_000_000, 10_000_000, 0.3,
                            w=24, zipf_s=1.1, new_pool=3_000_000)
    else:
        raise ValueError(f"no single-column configuration {k}")
    col.meta["config"] = CONFIG_NAMES[k]
    return col


def batched_shapes(ncols: int = 300, scale: float = 1.0, k: int = 4):
    """Per-column (vtype, rows, distinct) of the batched configuration."""
    shapes = []
    for c in range(ncols):
        rng = np.random.default_rng(BASE_SEED + 1000 * k + c)
        rows = int(math.exp(rng.uniform(math.log(1e6), math.log(2e7))) * scale)
        rows = max(rows, 1)
        kd = int(math.exp(rng.uniform(math.log(2), math.log(1e7))))
        kd = max(1, min(kd, rows))
        vtype = ("u32", "u64", "str16")[int(rng.integers(0, 3))]
        shapes.append((vtype, rows, kd, int(rng.integers(0, 2 ** 63))))
    return shapes


def _batched_one(shape):
    vtype, rows, kd, sub = shape
    rng = np.random.default_rng(sub)
    n_delta = rows // 100
    u64_high = 2 ** 64 if vtype == "u64" else 2 ** 63
    return random_column(rng, vtype, kd, rows, n_delta, 0.5, u64_high=u64_high)


def batched_columns(ncols: int = 300, scale: float = 1.0, k: int = 4, workers: int = 1):
    """Columns of the batched configuration: delta = 1% of main rows, half
    drawn from the main dictionary and half new distinct values.  Every
    column has its own seed, so `workers` > 1 (separate processes, started
    fresh) gives the same columns faster."""
    shapes = batched_shapes(ncols, scale, k)
    if workers <= 1:
        return [_batched_one(sh) for sh in shapes]
    import concurrent.futures as cf
    import multiprocessing as mp
    # largest columns first, so the pool's tail is short
    order = sorted(range(len(shapes)), key=lambda i: -shapes[i][1])
    out = [None] * len(shapes)
    with cf.ProcessPoolExecutor(max_workers=workers,
                                mp_context=mp.get_context("spawn")) as ex:
        futs = {ex.submit(_batched_one, shapes[i]): i for i in order}
        for f in cf.as_completed(futs):
            out[futs[f]] = f.result()
    return out
