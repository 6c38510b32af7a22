"""Seeded synthetic inputs for the column merge.

This package only *creates inputs*: sorted unique main dictionaries, packed
main code vectors and delta value arrays shaped like the workloads of the
paper's evaluation (Section 7: values drawn uniformly at random, 4- to
16-byte values, main partitions of 1M to 1B rows, deltas of about 1% of the
main) and like the five workload configurations of the benchmark.  It holds
no step of the merge itself.  Both the CPU oracle and the GPU library consume
the same bytes produced here.

Value arrays:
  u32   -> 1-D uint32
  u64   -> 1-D uint64
  str16 -> 2-D uint8 (n, 16), bytes in [0x20, 0x7E], ordered as unsigned bytes
"""
from .gen import (  # noqa: F401
    BASE_SEED,
    Column,
    pack_codes,
    sort_unique_values,
    random_values,
    random_column,
    config_column,
    batched_columns,
    CONFIG_NAMES,
)
