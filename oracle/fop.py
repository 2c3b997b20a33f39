"""Find-or-put on the static cuckoo table by sorting the batch.

TEST INFRASTRUCTURE ONLY (see the package docstring).

This is the baseline of the paper's find-or-put experiment (Sec. 5,
"Find-or-put"): the cuckoo table has no concurrent find-or-put of its own, so
the batch is sorted to expose duplicates, every distinct key is looked up
once, and every distinct key that is not stored is inserted once with the
cuckoo put.  The oracle takes those steps on its sequential cuckoo table
(Alg. 4 applied one key at a time); numpy's unique is the sort.

Answers per input position: FOUND for a key stored before the batch; for
any other key, the put's answer (PUT, or FULL once an eviction chain runs
past the bound) at its first occurrence in the batch and FOUND at the later
occurrences (FULL again if the first one was FULL).  The distinct keys are
put in increasing key order, the order the sort leaves them in.
"""
from __future__ import annotations

import numpy as np

from . import FOUND, FULL, PUT


def cuckoo_find_or_put(table, keys) -> np.ndarray:
    """Apply one sorted find-or-put batch to the oracle cuckoo `table` and
    return the answer byte of every input position."""
    k = np.asarray(keys, dtype=np.uint64)
    if k.size == 0:
        return np.zeros(0, np.uint8)
    distinct, first, which = np.unique(k, return_index=True, return_inverse=True)
    stored = table.find(distinct).astype(bool)
    missing = np.nonzero(~stored)[0]  # increasing key order
    per_key = np.full(distinct.size, FOUND, np.uint8)
    if missing.size:
        per_key[missing] = table.insert(distinct[missing])
    out = per_key[which.reshape(-1)]
    later = np.ones(k.size, bool)
    later[first] = False
    out[later & (out == PUT)] = FOUND
    return out


__all__ = ["cuckoo_find_or_put", "PUT", "FOUND", "FULL"]
