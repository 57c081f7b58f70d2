"""Host-side accounting in bench.py, checked against counts made by hand on small batches."""
import importlib.util
import os

import numpy as np

from helpers import ROOT
from paper_2406_10158_amd import workload as wl

spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
bench = importlib.util.module_from_spec(spec)
spec.loader.exec_module(bench)


def _batch(txns):
    """txns: list of [(table, row, field, kind, arg), ...]"""
    lengths, cols = [], [[] for _ in range(5)]
    for ops in txns:
        lengths.append(len(ops))
        for op in ops:
            for c, v in zip(cols, op):
                c.append(v)
    return wl._pack(lengths, *[np.array(c, np.int64) for c in cols], {})


def test_counts_single_op_rows():
    # txn0: read r1, add r2; txn1: add r3 -> 3 ops, 3 row groups, 2 written
    b = _batch([[(0, 1, 0, wl.READ, 0), (0, 2, 0, wl.ADD, 5)], [(0, 3, 0, wl.ADD, 1)]])
    acc = bench.access_counts(b)
    assert acc["value_loads"] == 3 and acc["word_loads"] == 2 * 1  # 3 values; read row word + its validation
    assert acc["word_atomics"] == 2              # two write rows locked
    assert acc["value_stores"] == 2 and acc["word_stores"] == 2  # two values, two publishing words
    assert acc["stream_bytes"] == 3 * 24 + 2 * 40
    # per op 32 B, per group 8 B, per write 8 B, per written group 8 B, per read group 8 B, per txn 40 B
    assert bench.algorithmic_bytes(b) == 3 * 32 + 3 * 8 + 2 * 8 + 2 * 8 + 1 * 8 + 2 * 40


def test_counts_multi_field_row_groups():
    # one txn touching row 7 twice (adjacent: one row access, written) and row 9 once (read)
    b = _batch([[(0, 7, 0, wl.READ, 0), (0, 7, 1, wl.ADD, 2), (0, 9, 0, wl.READ, 0)]])
    acc = bench.access_counts(b)
    assert acc["word_atomics"] == 1               # row 7 locked once
    assert acc["value_loads"] == 3 and acc["word_loads"] == 2 * 1  # 3 values; row 9 word + validation
    assert acc["value_stores"] == 1 and acc["word_stores"] == 1
    # the same row in two different transactions is two accesses
    b2 = _batch([[(0, 7, 0, wl.ADD, 1)], [(0, 7, 0, wl.ADD, 1)]])
    assert bench.access_counts(b2)["word_atomics"] == 2


def test_counts_scale_with_the_generated_workload():
    b = wl.kv_batch(10_000, 10, 2_000, ops=16, read_ratio=0.5, seed=3)
    acc = bench.access_counts(b)
    writes = int((b.kind != wl.READ).sum())
    assert acc["word_atomics"] == writes          # one op per row: every write row is one group
    assert acc["value_loads"] == b.total_ops and acc["word_loads"] == 2 * (b.total_ops - writes)
