"""Algorithmic cache lines per operation, from the sequential oracle.

TEST INFRASTRUCTURE (see oracle/__init__.py): this script only calls the
oracle.  It prints, for the benchmark's table shapes at each load, the mean
number of 128-byte lines an operation reads (bucket snapshots) and writes
(buckets it modifies), counted by the sequential model at a reduced slot
count with the same bucket shape, load and hit ratio.  The benchmark quotes
these figures as its per-operation algorithmic traffic.

usage: python oracle/lines_per_op.py [log2_slots]
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import oracle  # noqa: E402
import synth  # noqa: E402

LOADS = (0.5, 0.7, 0.8, 0.9, 0.95)


def cuckoo_shape(log2_slots: int, B: int, S: int, compact: bool, load: float, w: int = 37) -> dict:
    t = oracle.Table(oracle.CUCKOO, w, log2_slots, B, S, compact=compact, seed=11)
    bucket_lines = max(1, B * S // 8 // 128)
    n = int(load * (1 << log2_slots))
    keys = synth.distinct_keys(w, 0x5EED, 0, n).numpy().astype(np.uint64)
    out, lput = t.insert(keys, lines=True)
    nq = 1 << (log2_slots - 1)
    q = synth.find_queries(w, 0x5EED, n, nq, 0.5, 3).numpy().astype(np.uint64)
    _, lfind = t.find(q, lines=True)
    return {
        "scheme": "cuckoo", "B": B, "S": S, "compact": compact, "load": load,
        "full": int((out == oracle.FULL).sum()),
        # sequential put: one bucket read per round and one slot (one line) written per round
        "put_read_lines": float(lput.mean()), "put_write_lines": float(lput.mean()) / bucket_lines,
        "find_read_lines": float(lfind.mean()), "bucket_lines": bucket_lines,
    }


def iceberg_shape(log2_slots0: int, B0: int, S0: int, S1: int, compact: bool, load: float, w: int) -> dict:
    t = oracle.Table(oracle.ICEBERG, w, log2_slots0, B0, S0, log2_slots1=log2_slots0 - 3, B1=B0 // 2, s1=S1,
                     compact=compact, seed=11)
    cap = (1 << log2_slots0) + (1 << (log2_slots0 - 3))
    n = int(load * cap)
    keys = synth.distinct_keys(w, 0x5EED, 0, n).numpy().astype(np.uint64)
    out, lput = t.insert(keys, lines=True)
    nq = 1 << (log2_slots0 - 1)
    q = synth.find_queries(w, 0x5EED, n, nq, 0.5, 3).numpy().astype(np.uint64)
    _, lfind = t.find(q, lines=True)
    return {
        "scheme": "iceberg", "B0": B0, "S0": S0, "S1": S1, "compact": compact, "load": load,
        "full": int((out == oracle.FULL).sum()),
        "put_read_lines": float(lput.mean()), "put_write_lines": float((out == oracle.PUT).mean()),
        "find_read_lines": float(lfind.mean()),
    }


def main():
    L = int(sys.argv[1]) if len(sys.argv) > 1 else 22
    rows = []
    for load in LOADS:
        rows.append(cuckoo_shape(L, 32, 32, True, load))
        rows.append(cuckoo_shape(L, 32, 64, False, load))
    for row in rows:
        print(json.dumps(row))


if __name__ == "__main__":
    main()
