"""The multi-threaded CPU merge (Section 6.2's scheme) against the oracle,
byte for byte: random shapes and value types, 1 to 8 threads (more threads
than rows included), empty main / delta, heavy duplicates, a bad code."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import cpu_parallel
import oracle
from test_oracle import tiny_columns
from workloads import gen


@pytest.fixture(scope="module", autouse=True)
def built():
    cpu_parallel.build(force=True)
    oracle.build()


def check(col, threads):
    got = cpu_parallel.merge_column(col.vtype, col.u_m, col.main_packed, col.n_main, col.w,
                                    col.delta, threads)
    ref = oracle.merge_column(col.vtype, col.u_m, col.main_packed, col.n_main, col.w, col.delta)
    assert got["n_new"] == ref["n_new"] and got["w_new"] == ref["w_new"]
    assert got["n_words"] == ref["n_words"]
    assert np.array_equal(got["u_new"], ref["u_new"])
    assert np.array_equal(got["codes"], ref["codes"])
    assert np.array_equal(got["x_m"], ref["x_m"])
    assert np.array_equal(got["x_d"], ref["x_d"])


@pytest.mark.parametrize("vtype", ["u32", "u64", "str16"])
@pytest.mark.parametrize("threads", [1, 3, 8])
@pytest.mark.parametrize("shape", [(1, 1, 1, 0.0), (300, 4096, 4096, 0.5), (777, 12_289, 9_001, 0.9),
                                   (0, 0, 500, 1.0), (3, 1000, 0, 0.0), (20_000, 9_000, 30_000, 0.1),
                                   (5, 7, 3, 0.5)])
def test_matches_oracle(vtype, threads, shape):
    rng = np.random.default_rng(hash((vtype, threads, shape)) % (2 ** 32))
    check(gen.random_column(rng, vtype, *shape), threads)


@pytest.mark.parametrize("vtype", ["u32", "u64", "str16"])
def test_heavy_duplicates(vtype):
    rng = np.random.default_rng(17)
    col = gen.random_column(rng, vtype, 2000, 30_000, 40_000, 0.3, zipf_s=1.1, new_pool=500)
    check(col, 6)


def test_bad_code_is_reported():
    u_m = np.array([1, 5, 9], np.uint64)
    packed = gen.pack_codes(np.array([0, 3, 2], np.uint32), 2)  # code 3 >= |U_M|
    with pytest.raises(cpu_parallel.CpuMergeError):
        cpu_parallel.merge_column("u64", u_m, packed, 3, 2, np.array([4], np.uint64), 2)


def test_reused_outputs():
    """Output buffers reused across calls give the same result as fresh ones;
    buffers sized for another merge are refused."""
    rng = np.random.default_rng(23)
    col = gen.random_column(rng, "u64", 500, 20_000, 7_000, 0.5)
    o = cpu_parallel.alloc_outputs("u64", len(col.u_m), col.n_main, len(col.delta))
    o["out"][:] = ~np.uint64(0)  # stale contents must not leak into the result
    ref = oracle.merge_column(col.vtype, col.u_m, col.main_packed, col.n_main, col.w, col.delta)
    for threads in (4, 2):
        got = cpu_parallel.merge_column(col.vtype, col.u_m, col.main_packed, col.n_main, col.w,
                                        col.delta, threads, outputs=o)
        assert np.array_equal(got["codes"], ref["codes"])
        assert np.array_equal(got["x_d"], ref["x_d"])
    small = cpu_parallel.alloc_outputs("u64", 10, 10, 10)
    with pytest.raises(cpu_parallel.CpuMergeError):
        cpu_parallel.merge_column(col.vtype, col.u_m, col.main_packed, col.n_main, col.w,
                                  col.delta, 2, outputs=small)


@settings(max_examples=200, deadline=None, suppress_health_check=list(HealthCheck))
@given(tiny_columns(), st.integers(1, 9))
def test_hypothesis_tiny_columns(col, threads):
    """The oracle's brute-force strategy at 1 to 9 threads (often more threads
    than rows or dictionary entries)."""
    check(col, threads)
