"""Pins of the oracle's delete by tombstone (Sec. 2.2 "Lookup" and Sec. 3
"Limitations": a deleted key leaves a non-empty marker so that the non-empty
slots of a bucket stay consecutive and lookups keep their early exit).

The answers and the final set are fixed by set semantics; the tests replay
random insert / delete / find sequences one operation at a time on a Python
set, on tiny key domains where every key of the domain can be queried, and
run the table checker after every batch.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from oracle import sets


def _check(t):
    ok, msg, dec = t.check()
    assert ok, msg
    return dec


@pytest.mark.parametrize("scheme", [oracle.CUCKOO, oracle.ICEBERG])
def test_delete_matches_set_semantics_tiny_domain(scheme):
    w = 11
    if scheme == oracle.CUCKOO:
        t = oracle.Table(scheme, w, 8, 8, 32, seed=4, C=64)
    else:
        t = oracle.Table(scheme, w, 8, 16, 16, log2_slots1=6, B1=8, s1=16, seed=4)
    rng = np.random.default_rng(scheme + 10)
    domain = np.arange(1 << w, dtype=np.uint64)
    S: set = set()
    deleted = 0
    for step in range(40):
        kind = step % 3
        if kind == 0:  # inserts of fresh keys (cuckoo needs absent, distinct keys)
            cand = np.setdiff1d(rng.choice(domain, 12, replace=False), np.array(sorted(S), np.uint64))
            # tombstones hold their slots until the table is rebuilt
            if len(S) + t.tombstones() + cand.size > 0.5 * t.capacity():
                continue
            out = t.insert(cand)
            assert (out == oracle.PUT).all()
            S.update(int(x) for x in cand)
        elif kind == 1:  # deletes: stored keys, absent keys and repeats
            stored = np.array(sorted(S), np.uint64)
            pick = np.concatenate([rng.choice(stored, min(6, stored.size), replace=False) if stored.size else
                                   np.zeros(0, np.uint64), rng.choice(domain, 4)])
            pick = np.concatenate([pick, pick[:2]])
            want = []
            for k in (int(x) for x in pick):
                want.append(1 if k in S else 0)
                S.discard(k)
            got = t.delete(pick)
            assert got.tolist() == want
            deleted += int(sum(want))
        else:
            assert np.array_equal(t.find(domain), np.isin(domain, np.array(sorted(S), np.uint64)).astype(np.uint8))
        dec = _check(t)
        assert sorted(int(x) for x in dec) == sorted(S)
        assert t.occupied() == len(S)
    assert deleted > 0
    if scheme == oracle.ICEBERG:
        assert t.tombstones() == deleted  # iceberg never reuses a tombstone


def test_delete_set_definition():
    S = np.array([3, 5, 9], np.uint64)
    out, after = sets.delete(S, [5, 7, 5, 3])
    assert out.tolist() == [1, 0, 0, 1]
    assert after.tolist() == [9]


def test_iceberg_reinsert_after_delete():
    t = oracle.Table(oracle.ICEBERG, 18, 8, 16, 16, log2_slots1=6, B1=8, s1=32, seed=2)
    keys = np.arange(100, 160, dtype=np.uint64)
    assert (t.insert(keys) == oracle.PUT).all()
    assert (t.delete(keys[:20]) == 1).all()
    assert (t.find(keys[:20]) == 0).all() and (t.find(keys[20:]) == 1).all()
    # find-or-put puts a deleted key again (into a later slot) and finds the rest
    out = t.insert(keys)
    assert (out[:20] == oracle.PUT).all() and (out[20:] == oracle.FOUND).all()
    assert t.occupied() == 60 and t.tombstones() == 20
    _check(t)


def test_cuckoo_put_overwrites_tombstone_victims():
    """Fill a tiny cuckoo table, delete most keys, then insert new ones: the
    evictions land on tombstones, which end the chain (nothing to carry)."""
    w = 16
    t = oracle.Table(oracle.CUCKOO, w, 6, 8, 32, seed=9, C=32)
    rng = np.random.default_rng(3)
    keys = rng.choice(1 << w, 60, replace=False).astype(np.uint64)
    out = t.insert(keys)
    stored = keys[out == oracle.PUT]
    _check(t)
    gone = stored[: stored.size * 3 // 4]
    assert (t.delete(gone) == 1).all()
    tomb_before = t.tombstones()
    fresh = np.setdiff1d(rng.choice(1 << w, 200, replace=False).astype(np.uint64), keys)[:30]
    out2 = t.insert(fresh)
    assert (out2 == oracle.PUT).all()
    assert t.tombstones() < tomb_before  # some victims were tombstones
    want = np.union1d(np.setdiff1d(stored, gone), fresh)
    assert np.array_equal(_check(t), want)
    assert np.array_equal(t.find(want), np.ones(want.size, np.uint8))


def test_checker_accepts_tombstone_rejects_other_unoccupied_values():
    t = oracle.Table(oracle.ICEBERG, 18, 8, 16, 16, log2_slots1=6, B1=8, s1=32, seed=2)
    t.insert(np.arange(1, 40, dtype=np.uint64))
    t.delete(np.arange(1, 10, dtype=np.uint64))
    img0, img1 = t.export(0), t.export(1)
    ok, msg, _ = oracle.check_images(t.cfg, img0, img1)
    assert ok, msg
    v = img0.view(np.uint16)
    tomb = np.nonzero(v == 1)[0]
    assert tomb.size > 0
    bad = img0.copy()
    bad.view(np.uint16)[tomb[0]] = 3  # occupancy bit clear but not the tombstone
    ok, msg, _ = oracle.check_images(t.cfg, bad, img1)
    assert not ok and "occupancy" in msg
    # a tombstone after an EMPTY slot breaks the prefix rule like any other value
    bad = img0.copy()
    b0 = bad.view(np.uint16).reshape(-1, 16)
    row = int(np.nonzero((b0 == 0).any(axis=1))[0][0])
    b0[row, 15] = 1
    ok, msg, _ = oracle.check_images(t.cfg, bad, img1)
    assert not ok and "after an empty" in msg
