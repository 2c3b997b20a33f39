"""Pins of the oracle's sorted find-or-put on the cuckoo table (the baseline
of the paper's find-or-put experiment, Sec. 5).

Below the failure load the answers are fixed by set semantics alone: the
first occurrence of a key not yet stored is PUT, every other operation is
FOUND (Theorem 1 (c), (d) and the closing corollary of Appendix A).  The
tests replay each batch one operation at a time on a Python set and compare;
above the failure load they check the accounting that any run of the method
must satisfy.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from oracle.fop import cuckoo_find_or_put


def _set_semantics(S: set, keys) -> list[int]:
    out = []
    for k in (int(x) for x in keys):
        if k in S:
            out.append(oracle.FOUND)
        else:
            S.add(k)
            out.append(oracle.PUT)
    return out


def _decoded(t: oracle.Table) -> np.ndarray:
    ok, msg, dec = t.check()
    assert ok, msg
    return dec


@pytest.mark.parametrize("w,log2_slots,B,s", [(12, 8, 8, 32), (16, 10, 16, 32), (37, 12, 32, 64)])
def test_sorted_fop_is_set_semantics(w, log2_slots, B, s):
    rng = np.random.default_rng(w)
    t = oracle.Table(oracle.CUCKOO, w, log2_slots, B, s, seed=5, compact=s == 32)
    domain = rng.choice(1 << min(w, 40), size=int(0.8 * (1 << log2_slots)), replace=False).astype(np.uint64)
    S: set = set()
    for batch in range(4):
        # repeats inside the batch and keys stored by earlier batches
        keys = domain[rng.integers(0, (batch + 1) * domain.size // 4, size=domain.size // 3)]
        want = _set_semantics(S, keys)
        got = cuckoo_find_or_put(t, keys)
        assert got.tolist() == want
        assert sorted(int(x) for x in _decoded(t)) == sorted(S)


def test_sorted_fop_all_duplicates_and_empty():
    t = oracle.Table(oracle.CUCKOO, 20, 8, 8, 32, seed=1)
    assert cuckoo_find_or_put(t, np.zeros(0, np.uint64)).size == 0
    keys = np.full(50, 777, np.uint64)
    out = cuckoo_find_or_put(t, keys)
    assert out[0] == oracle.PUT and (out[1:] == oracle.FOUND).all()
    assert (cuckoo_find_or_put(t, keys) == oracle.FOUND).all()
    assert _decoded(t).tolist() == [777]


def test_sorted_fop_over_capacity_accounting():
    """Past the failure load: FULL drops one carried key per FULL answer, so
    the stored set is a subset of everything offered and is smaller than it
    by exactly the number of FULL first occurrences."""
    w = 14
    t = oracle.Table(oracle.CUCKOO, w, 7, 8, 32, seed=3, C=16)
    rng = np.random.default_rng(2)
    pre = rng.choice(1 << w, size=90, replace=False).astype(np.uint64)
    assert (t.insert(pre) == oracle.PUT).all()
    keys = np.concatenate([rng.choice(1 << w, size=120).astype(np.uint64), pre[:20]])
    rng.shuffle(keys)
    out = cuckoo_find_or_put(t, keys)
    dec = _decoded(t)
    offered = np.union1d(pre, keys)
    _, first = np.unique(keys, return_index=True)
    n_full = int((out[first] == oracle.FULL).sum())
    assert n_full > 0
    assert np.isin(dec, offered).all()
    assert dec.size == offered.size - n_full
    # keys stored before the batch are FOUND (they are looked up before any put)
    assert (out[np.isin(keys, pre)] == oracle.FOUND).all()
    # later occurrences repeat FULL or turn PUT into FOUND
    later = np.ones(keys.size, bool)
    later[first] = False
    assert not (out[later] == oracle.PUT).any()


def test_map_definition_worked_example():
    """Put-if-absent: the first value offered for a key stays."""
    from oracle import sets
    M: dict = {}
    out = sets.insert_values(M, [5, 9, 5, 7, 9], [50, 90, 51, 70, 91])
    assert out.tolist() == [oracle.PUT, oracle.PUT, oracle.FOUND, oracle.PUT, oracle.FOUND]
    assert M == {5: 50, 9: 90, 7: 70}
    found, vals = sets.find_values(M, [7, 8, 5])
    assert found.tolist() == [1, 0, 1] and vals.tolist() == [70, 0, 50]


def test_map_answers_equal_set_answers():
    from oracle import sets
    rng = np.random.default_rng(3)
    keys = rng.integers(0, 200, size=500).astype(np.uint64)
    vals = rng.integers(0, 1 << 40, size=500).astype(np.uint64)
    M: dict = {}
    out = sets.insert_values(M, keys, vals)
    want, S = sets.insert(np.zeros(0, np.uint64), keys)
    assert np.array_equal(out, want)
    assert sorted(M) == S.tolist()
    # each stored value is the one offered at the key's first occurrence
    _, first = np.unique(keys, return_index=True)
    assert all(M[int(keys[i])] == int(vals[i]) for i in first)
