"""Pins for the CPU oracle (no GPU).

The oracle is checked against things other than itself: the hand example
built from the paper's stated facts (Sections 4.1 and 5.3), a brute-force
merge written with Python sets and sorting, the closed forms that follow
from Eqs. 2-4, the special cases that reduce to library routines, the naive
Step 2(b) of Section 5.2, and an independent bit packer (numpy.packbits).
"""
import json
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st, HealthCheck

import oracle
from workloads import gen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# Independent references
# ---------------------------------------------------------------------------

def packbits_reference(codes, w):
    """Pack via an explicit bit matrix and numpy.packbits (little bit order)."""
    codes = np.asarray(codes, dtype=np.uint64).reshape(-1)
    n = codes.shape[0]
    nwords = (n * w + 63) // 64
    if nwords == 0:
        return np.zeros(0, np.uint64)
    bits = ((codes[:, None] >> np.arange(w, dtype=np.uint64)[None, :]) & np.uint64(1)).astype(np.uint8)
    flat = np.zeros(nwords * 64, np.uint8)
    flat[: n * w] = bits.reshape(-1)
    by = np.packbits(flat, bitorder="little")
    return by.view("<u8").astype(np.uint64)


def unpackbits_reference(words, n, w):
    by = np.asarray(words, dtype="<u8").view(np.uint8)
    flat = np.unpackbits(by, bitorder="little")[: n * w].reshape(n, w).astype(np.uint64)
    return (flat << np.arange(w, dtype=np.uint64)[None, :]).sum(axis=1).astype(np.uint64)


def as_py(values, vtype):
    """Values as Python objects whose natural order is the column order."""
    if vtype == "str16":
        return [bytes(r) for r in np.asarray(values, np.uint8).reshape(-1, 16)]
    return [int(x) for x in np.asarray(values).reshape(-1)]


def brute_force(vtype, u_m, main_codes, n_main, w, delta):
    """U' = sorted set(U_M) | set(D); each row's code = its value's rank."""
    um = as_py(u_m, vtype)
    d = as_py(delta, vtype)
    codes = unpackbits_reference(main_codes, n_main, w) if n_main else np.zeros(0, np.uint64)
    rows = [um[int(c)] for c in codes] + d
    u_new = sorted(set(um) | set(d))
    rank = {v: i for i, v in enumerate(u_new)}
    n = len(u_new)
    w_new = 1 if n <= 1 else (n - 1).bit_length()
    new_codes = [rank[v] for v in rows]
    return u_new, w_new, new_codes


def to_py_bytes(s):
    b = s.encode("ascii")
    return b + b"\0" * (16 - len(b))


def str_array(words):
    return np.frombuffer(b"".join(to_py_bytes(s) for s in words), np.uint8).reshape(-1, 16).copy()


# ---------------------------------------------------------------------------
# The hand example (Sections 4.1 and 5.3)
# ---------------------------------------------------------------------------

def test_hand_example():
    ex = json.load(open(os.path.join(GOLDEN, "hand_example.json")))
    e = ex["expected"]
    u_m = str_array(ex["u_m"])
    # main codes are positions of the main rows' words in U_M
    codes = [ex["u_m"].index(x) for x in ex["main_rows"]]
    assert codes == e["main_codes"]
    packed = oracle.pack_codes(codes, ex["w"])
    assert packed.view(np.uint8)[:3].tobytes().hex() == e["main_packed_bytes"]
    delta = str_array(ex["delta"])
    r = oracle.merge_column("str16", u_m, packed, len(codes), ex["w"], delta)
    assert [bytes(x).rstrip(b"\0").decode() for x in r["u_d"]] == e["u_d"]
    assert r["drank"].tolist() == e["drank"]
    assert oracle.width(len(e["u_d"])) == e["delta_code_width"]
    assert [bytes(x).rstrip(b"\0").decode() for x in r["u_new"]] == e["u_new"]
    assert r["x_m"].tolist() == e["x_m"]
    assert r["x_d"].tolist() == e["x_d"]
    assert r["w_new"] == e["w_new"] and r["n_new"] == 9
    assert oracle.unpack_codes(r["codes"], 12, 4).tolist() == e["new_codes"]
    nbytes = (12 * 4 + 7) // 8
    assert r["codes"].view(np.uint8)[:nbytes].tobytes().hex() == e["new_packed_bytes"]
    # 'hotel' was main code 4 and becomes 6 (Section 4.1)
    assert r["x_m"][4] == 6


# ---------------------------------------------------------------------------
# Width (Eq. 4 with the one-bit floor) and packing
# ---------------------------------------------------------------------------

def test_width_closed_form():
    assert oracle.width(0) == 1 and oracle.width(1) == 1
    for k in range(1, 33):
        assert oracle.width(2 ** k) == k
        assert oracle.width(2 ** k + 1) == k + 1
        assert oracle.width(2 ** k - 1) == (k if k > 1 else 1)
    assert oracle.width(6) == 3 and oracle.width(9) == 4      # Section 4.1
    assert oracle.width(1_948_000) == 21 and oracle.width(1_048_000) == 20


@pytest.mark.parametrize("w", list(range(1, 33)))
def test_pack_against_packbits(w):
    rng = np.random.default_rng(w)
    for n in (0, 1, 63, 64, 65, 127, 128, 129, 300):
        codes = rng.integers(0, 2 ** w, size=n, dtype=np.uint64)
        ref = packbits_reference(codes, w)
        assert np.array_equal(oracle.pack_codes(codes, w), ref)
        assert np.array_equal(oracle.unpack_codes(ref, n, w).astype(np.uint64), codes)
        # the generator's packer must agree too (it writes every input)
        assert np.array_equal(gen.pack_codes(codes, w), ref)


def test_pack_padding_zero():
    # bits beyond n*w in the last word stay zero
    codes = np.full(5, 7, np.uint64)
    p = oracle.pack_codes(codes, 3)
    assert p.shape == (1,) and int(p[0]) == (1 << 15) - 1


# ---------------------------------------------------------------------------
# Brute force on tiny inputs (hypothesis)
# ---------------------------------------------------------------------------

@st.composite
def tiny_columns(draw):
    vtype = draw(st.sampled_from(["u32", "u64", "str16"]))
    seed = draw(st.integers(0, 2 ** 32 - 1))
    rng = np.random.default_rng(seed)
    n_um = draw(st.integers(0, 40))
    n_main = draw(st.integers(0, 200)) if n_um > 0 else 0
    n_delta = draw(st.integers(0, 60))
    frac_new = draw(st.sampled_from([0.0, 0.3, 0.5, 1.0]))
    small = draw(st.booleans())          # small value domain: many collisions
    if small and vtype != "str16":
        u_m = np.unique(rng.integers(0, 50, size=n_um)).astype(np.uint32 if vtype == "u32" else np.uint64)
        n_um = u_m.shape[0]
        if n_um == 0:
            n_main = 0
        w = gen.code_width(n_um) + draw(st.integers(0, 2))
        codes = rng.integers(0, max(n_um, 1), size=n_main)
        delta = rng.integers(0, 60, size=n_delta).astype(u_m.dtype)
        return gen.Column(vtype, u_m, gen.pack_codes(codes, w), n_main, w, delta)
    col = gen.random_column(rng, vtype, n_um, n_main, n_delta, frac_new,
                            u64_high=2 ** 64 if vtype == "u64" else 2 ** 63)
    extra = draw(st.integers(0, 3))
    if extra and col.w + extra <= 32:
        # a caller may store codes wider than needed
        codes = unpackbits_reference(col.main_packed, col.n_main, col.w) if col.n_main else np.zeros(0)
        col = gen.Column(vtype, col.u_m, gen.pack_codes(codes, col.w + extra), col.n_main,
                         col.w + extra, col.delta)
    return col


@settings(max_examples=250, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(tiny_columns())
def test_brute_force(col):
    r = oracle.merge_column(col.vtype, col.u_m, col.main_packed, col.n_main, col.w, col.delta)
    u_new, w_new, new_codes = brute_force(col.vtype, col.u_m, col.main_packed, col.n_main,
                                          col.w, col.delta)
    assert as_py(r["u_new"], col.vtype) == u_new
    assert r["w_new"] == w_new and r["n_new"] == len(u_new)
    n_out = col.n_main + col.n_delta
    assert r["n_words"] == (n_out * w_new + 63) // 64
    assert np.array_equal(r["codes"], packbits_reference(np.array(new_codes, np.uint64), w_new))
    check_invariants(col, r)


def check_invariants(col, r):
    """Invariants that any correct merge satisfies."""
    vt = col.vtype
    u_new = as_py(r["u_new"], vt)
    assert all(a < b for a, b in zip(u_new, u_new[1:]))           # strictly increasing
    um = as_py(col.u_m, vt)
    ud = as_py(r["u_d"], vt)
    x_m, x_d = r["x_m"].tolist(), r["x_d"].tolist()
    assert all(a < b for a, b in zip(x_m, x_m[1:]))
    assert all(a < b for a, b in zip(x_d, x_d[1:]))
    assert all(u_new[x] == v for x, v in zip(x_m, um))
    assert all(u_new[x] == v for x, v in zip(x_d, ud))
    assert set(x_m) | set(x_d) == set(range(len(u_new)))
    # decode(new) == decode(old main) ++ delta
    n_out = col.n_main + col.n_delta
    if n_out:
        codes = unpackbits_reference(r["codes"], n_out, r["w_new"])
        assert int(codes.max()) < len(u_new)
        old = unpackbits_reference(col.main_packed, col.n_main, col.w) if col.n_main else []
        rows = [um[int(c)] for c in old] + as_py(col.delta, vt)
        assert [u_new[int(c)] for c in codes] == rows
        # padding bits in the last word are zero
        used = n_out * r["w_new"]
        if used % 64:
            assert int(r["codes"][-1]) >> (used % 64) == 0


# ---------------------------------------------------------------------------
# Closed forms and special cases
# ---------------------------------------------------------------------------

def _merge(col):
    return oracle.merge_column(col.vtype, col.u_m, col.main_packed, col.n_main, col.w, col.delta)


@pytest.mark.parametrize("vtype", ["u32", "u64", "str16"])
def test_translation_closed_forms(vtype):
    rng = np.random.default_rng(7)
    col = gen.random_column(rng, vtype, 500, 3000, 800, 0.5)
    r = _merge(col)
    um = as_py(col.u_m, vtype)
    ud = as_py(r["u_d"], vtype)
    new = sorted(set(ud) - set(um))
    import bisect
    # X_M[i] = i + #{new delta values below U_M[i]}
    assert r["x_m"].tolist() == [i + bisect.bisect_left(new, v) for i, v in enumerate(um)]
    # X_D[k] = #{U_M below U_D[k]} + #{new delta values below U_D[k]}
    assert r["x_d"].tolist() == [bisect.bisect_left(um, v) + bisect.bisect_left(new, v) for v in ud]
    assert r["n_new"] == len(set(um) | set(ud))                    # Eq. 3


@pytest.mark.parametrize("vtype", ["u32", "u64", "str16"])
def test_empty_delta_is_identity(vtype):
    rng = np.random.default_rng(11)
    col = gen.random_column(rng, vtype, 300, 5000, 0)
    r = _merge(col)
    assert r["x_m"].tolist() == list(range(300))
    assert r["w_new"] == col.w
    # with an exact input width the packed stream is byte-identical
    assert np.array_equal(r["codes"], col.main_packed)


@pytest.mark.parametrize("vtype", ["u32", "u64", "str16"])
def test_delta_subset_of_main(vtype):
    rng = np.random.default_rng(12)
    col = gen.random_column(rng, vtype, 300, 2000, 700, 0.0)
    r = _merge(col)
    assert r["x_m"].tolist() == list(range(300))
    assert np.array_equal(r["codes"][: col.main_packed.shape[0] - 1], col.main_packed[:-1])
    if vtype == "str16":
        return
    delta_codes = unpackbits_reference(r["codes"], 2700, r["w_new"])[2000:]
    assert np.array_equal(delta_codes, np.searchsorted(col.u_m, col.delta).astype(np.uint64))


def test_all_new_above_and_below():
    um = np.array([100, 200, 300, 400], np.uint64)
    codes = gen.pack_codes(np.array([0, 1, 2, 3, 3, 2, 1, 0]), 2)
    above = np.array([1000, 900, 1000, 950], np.uint64)
    r = oracle.merge_column("u64", um, codes, 8, 2, above)
    assert r["x_m"].tolist() == [0, 1, 2, 3]
    assert r["x_d"].tolist() == [4, 5, 6]              # |U_M| + k
    below = np.array([5, 1, 5, 3], np.uint64)
    r = oracle.merge_column("u64", um, codes, 8, 2, below)
    assert r["x_m"].tolist() == [3, 4, 5, 6]           # i + |U_D|
    assert r["x_d"].tolist() == [0, 1, 2]


@pytest.mark.parametrize("vtype", ["u32", "u64", "str16"])
def test_empty_main_is_unique_inverse(vtype):
    rng = np.random.default_rng(13)
    col = gen.random_column(rng, vtype, 0, 0, 400, 0.6, new_pool=150)
    r = _merge(col)
    if vtype == "str16":
        keys = [bytes(x) for x in col.delta]
        uniq = sorted(set(keys))
        inv = [uniq.index(k) for k in keys]
        assert as_py(r["u_new"], vtype) == uniq
    else:
        uniq, inv = np.unique(col.delta, return_inverse=True)
        assert np.array_equal(r["u_new"], uniq)
    got = unpackbits_reference(r["codes"], 400, r["w_new"])
    assert got.tolist() == list(inv)


def test_single_value_dictionary_uses_one_bit():
    um = np.array([42], np.uint32)
    codes = gen.pack_codes(np.zeros(70), 1)
    r = oracle.merge_column("u32", um, codes, 70, 1, np.array([42, 42], np.uint32))
    assert r["n_new"] == 1 and r["w_new"] == 1
    assert r["n_words"] == 2 and r["codes"].tolist() == [0, 0]


def test_everything_empty():
    r = oracle.merge_column("u64", np.zeros(0, np.uint64), np.zeros(0, np.uint64), 0, 1,
                            np.zeros(0, np.uint64))
    assert r["n_new"] == 0 and r["w_new"] == 1 and r["n_words"] == 0


@pytest.mark.parametrize("vtype", ["u32", "u64", "str16"])
def test_naive_route_agrees(vtype):
    """Section 5.2's decode-and-search route gives the same codes."""
    rng = np.random.default_rng(21)
    col = gen.random_column(rng, vtype, 700, 4000, 900, 0.5)
    r = _merge(col)
    naive = oracle.reencode_naive(vtype, col.u_m, col.main_packed, col.n_main, col.w,
                                  col.delta, r["u_new"], r["w_new"])
    assert np.array_equal(naive, r["codes"])


def test_invalid_inputs_rejected():
    um = np.array([1, 2, 3], np.uint64)
    codes = gen.pack_codes(np.array([0, 1, 2]), 2)
    with pytest.raises(oracle.OracleError):          # not sorted
        oracle.merge_column("u64", np.array([1, 3, 2], np.uint64), codes, 3, 2, um)
    with pytest.raises(oracle.OracleError):          # duplicate entry
        oracle.merge_column("u64", np.array([1, 2, 2], np.uint64), codes, 3, 2, um)
    with pytest.raises(oracle.OracleError):          # code outside the dictionary
        oracle.merge_column("u64", um, gen.pack_codes(np.array([0, 3, 2]), 2), 3, 2, um)
    with pytest.raises(oracle.OracleError):          # width too small for |U_M|
        oracle.merge_column("u64", np.arange(5, dtype=np.uint64), codes, 3, 2, um)
    with pytest.raises(oracle.OracleError):          # width out of range
        oracle.merge_column("u64", um, codes, 3, 33, um)


def test_config1_closed_form():
    """c1: 10,000 main values and 5,000 distinct new values -> |U'| = 15,000."""
    col = gen.config_column(1)
    r = _merge(col)
    assert r["n_new"] == 15_000 and r["w_new"] == 14
    assert r["n_words"] == (1_010_000 * 14 + 63) // 64
    # sampled rows decode to the right values
    rng = np.random.default_rng(0)
    rows = rng.integers(0, 1_010_000, size=200)
    for i in rows:
        c = oracle.unpack(r["codes"], int(i), 14)
        if i < 1_000_000:
            v = col.u_m[oracle.unpack(col.main_packed, int(i), 14)]
        else:
            v = col.delta[i - 1_000_000]
        assert r["u_new"][c] == v


def test_planted_mistakes_are_caught():
    """Each plausible slip in a merge (dropped tie rule, off-by-one rank,
    swapped tables) makes the brute-force comparison fail."""
    rng = np.random.default_rng(5)
    col = gen.random_column(rng, "u64", 50, 300, 80, 0.5)
    r = _merge(col)
    u_new, w_new, new_codes = brute_force("u64", col.u_m, col.main_packed, col.n_main,
                                          col.w, col.delta)
    good = packbits_reference(np.array(new_codes, np.uint64), w_new)
    assert np.array_equal(r["codes"], good)
    # (1) equal values appended twice -> ranks shift
    dup = sorted(as_py(col.u_m, "u64") + as_py(r["u_d"], "u64"))
    assert dup != u_new
    # (2) ranks off by one
    assert not np.array_equal(packbits_reference(np.array(new_codes, np.uint64) + 1 & ((1 << w_new) - 1), w_new), good)
    # (3) main re-encoded through X_D instead of X_M
    codes = unpackbits_reference(col.main_packed, col.n_main, col.w)
    wrong = [int(r["x_d"][int(c) % len(r["x_d"])]) for c in codes]
    assert wrong != new_codes[: col.n_main]
