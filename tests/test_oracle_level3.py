"""Pins of the oracle's third iceberg level (Sec. 2.3: linked lists outside
the table, chosen by h_0(k), take the keys whose primary and secondary
buckets are all full, so inserts do not fail; Sec. 3 Limitations names slab
lists as the way to build it).

Set semantics fix every answer while the slab pool has room; the tests replay
batches one operation at a time on a Python set over whole tiny key domains,
run the checker (which now also walks the lists) after every batch, and
plant corruptions in the level-3 images that it must reject.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle


def _table(w=14, pool=64, log2_lists=3, s0=16, s1=16, seed=3):
    # 2^7 + 2^4 slots in levels 1-2: tiny, so most of a domain overflows
    return oracle.Table(oracle.ICEBERG, w, 7, 16, s0, log2_slots1=4, B1=8, s1=s1, seed=seed,
                        log2_lists=log2_lists, pool_slabs=pool)


def _replay(S: set, keys):
    out = []
    for k in (int(x) for x in keys):
        if k in S:
            out.append(oracle.FOUND)
        else:
            S.add(k)
            out.append(oracle.PUT)
    return out


@pytest.mark.parametrize("s0,s1,log2_lists", [(16, 16, 3), (16, 32, 0), (32, 32, 5), (64, 64, 2)])
def test_level3_set_semantics_beyond_two_level_capacity(s0, s1, log2_lists):
    w = 14
    t = _table(w, pool=200, log2_lists=log2_lists, s0=s0, s1=s1)
    rng = np.random.default_rng(s0 + s1 + log2_lists)
    domain = np.arange(1 << w, dtype=np.uint64)
    S: set = set()
    for batch in range(6):
        keys = rng.choice(domain, 120)  # with repeats; 6 x 120 draws overfill 144 table slots
        want = _replay(S, keys)
        got = t.insert(keys)
        assert got.tolist() == want
        ok, msg, dec = t.check()
        assert ok, msg
        assert dec.tolist() == sorted(S)
        assert t.occupied() == len(S)
    assert len(S) > t.capacity()  # more keys than levels 1-2 hold: level 3 took the rest
    assert t.l3_used() > 0
    member = np.isin(domain, np.array(sorted(S), np.uint64)).astype(np.uint8)
    assert np.array_equal(t.find(domain), member)


def test_level3_pool_exhaustion_gives_full_and_absent():
    t = _table(pool=3, log2_lists=1)
    keys = np.arange(1, 400, dtype=np.uint64)
    out = t.insert(keys)
    full = keys[out == oracle.FULL]
    assert full.size > 0 and t.l3_used() == 3
    stored = keys[out == oracle.PUT]
    assert stored.size == t.occupied()
    assert (t.find(full) == 0).all() and (t.find(stored) == 1).all()
    ok, msg, dec = t.check()
    assert ok, msg
    assert np.array_equal(dec, np.sort(stored))


def test_level3_delete_and_reinsert():
    t = _table(pool=100, log2_lists=2)
    keys = np.arange(1, 260, dtype=np.uint64)
    assert (t.insert(keys) == oracle.PUT).all()
    assert t.l3_used() > 0
    gone = keys[::3]
    assert (t.delete(gone) == 1).all()
    assert (t.find(gone) == 0).all() and (t.find(np.setdiff1d(keys, gone)) == 1).all()
    out = t.insert(gone)
    assert (out == oracle.PUT).all()
    ok, msg, dec = t.check()
    assert ok, msg
    assert np.array_equal(dec, keys)


def _corrupt(t, fn):
    imgs = [t.export(0), t.export(1), t.export(2), t.export(3)]
    fn(imgs)
    return oracle.check_images(t.cfg, *imgs)


def test_checker_rejects_level3_corruptions():
    t = _table(pool=40, log2_lists=2)
    t.insert(np.arange(1, 300, dtype=np.uint64))
    ok, msg, _ = t.check()
    assert ok, msg
    used = t.l3_used()
    slot_words = 32  # 16-bit primary slots -> 32-bit level-3 slots, 32 per 128-byte slab

    def pool32(imgs):
        return imgs[2].view(np.uint32).reshape(-1, slot_words)

    # a key of level 3 copied into an unused slab that is on no list
    def orphan(imgs):
        p = pool32(imgs)
        p[used, 0] = p[0, 0]
    ok, msg, _ = _corrupt(t, orphan)
    assert not ok and "no list" in msg

    # a list whose head points at a slab already on another list
    def shared(imgs):
        h = imgs[3].view(np.uint32)
        nz = np.nonzero(h)[0]
        h[(nz[0] + 1) % h.size] = h[nz[0]]
    ok, msg, _ = _corrupt(t, shared)
    assert not ok

    # a hole in the middle of a slab
    def hole(imgs):
        p = pool32(imgs)
        p[0, 3] = 0
    ok, msg, _ = _corrupt(t, hole)
    assert not ok and "empty" in msg

    # a level-3 key whose primary bucket has an empty slot (order property)
    def primary_hole(imgs):
        v = imgs[0].view(np.uint16).reshape(-1, 16)
        v[:, 15] = 0
    ok, msg, _ = _corrupt(t, primary_hole)
    assert not ok

    # slab id out of range
    def bad_id(imgs):
        h = imgs[3].view(np.uint32)
        h[np.nonzero(h)[0][0]] = 41
    ok, msg, _ = _corrupt(t, bad_id)
    assert not ok and "out of range" in msg
