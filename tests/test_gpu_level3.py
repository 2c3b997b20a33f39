"""GPU parity of the third iceberg level (Sec. 2.3: lists outside the table,
chosen by h_0(k), hold the keys whose primary and secondary buckets are full;
Sec. 3 Limitations: slab lists) against the oracle.

The tables are tiny on purpose, so that most keys overflow into the lists and
many lanes race to link slabs.  Bars: per distinct key one PUT and FOUND for
the rest (which duplicate wins is timing-dependent); no FULL while the pool
has room; the decoded key set equals the oracle's; lookups bit-exact; the
checker walks every list (distinct slabs, slots filled in list order, keys in
their own list only behind full buckets, slabs on no list untouched).
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import paper_2406_09255_amd as cpht
import synth
from oracle import sets
from tests.helpers import check_table, host_u64, oracle_table, to_dev

pytestmark = pytest.mark.gpu

KEY_SEED = 0x1E3E13


def _dev(keys_h, w, gpu):
    return to_dev(torch.from_numpy(keys_h.astype(np.int64)), w, gpu)


SHAPES = [
    # w, L0, L1, B0, S0, S1, G, log2_lists, pool
    (18, 10, 7, 16, 16, 16, 2, 3, 400),
    (22, 12, 9, 32, 16, 32, 2, 6, 600),
    (32, 11, 8, 16, 32, 32, 4, 1, 400),
    (40, 10, 7, 16, 64, 64, 8, 2, 800),
    (34, 11, 8, 32, 32, 32, 8, 4, 500),
]


def _table(w, L0, L1, B0, S0, S1, G, lists, pool, seed=7):
    return cpht.Table(scheme=cpht.ICEBERG, key_bits=w, log2_slots0=L0, log2_slots1=L1, bucket0=B0,
                      bucket1=B0 // 2, slot_bits0=S0, slot_bits1=S1, compact=0 if S0 == 64 else 1, subtile=G,
                      log2_lists=lists, pool_slabs=pool, seed=seed)


@pytest.mark.parametrize("shape", SHAPES, ids=[f"{s[4]}_{s[5]}_B{s[3]}_g{s[6]}_l{s[7]}" for s in SHAPES])
def test_level3_matches_oracle(gpu, shape):
    w, L0, L1, B0, S0, S1, G, lists, pool = shape
    t = _table(*shape)
    o = oracle_table(t)
    cap = t.count()[1]
    # 2.5 x the two-level capacity in distinct keys, in batches with 30 % repeats
    n_distinct = int(2.5 * cap)
    pool_keys = host_u64(synth.distinct_keys(w, KEY_SEED + w, 0, n_distinct))
    rng = np.random.default_rng(w + S0)
    S = np.zeros(0, np.uint64)
    issued = 0
    for b in range(4):
        fresh = pool_keys[issued: issued + n_distinct // 4]
        issued += fresh.size
        rep = pool_keys[rng.integers(0, issued, size=fresh.size * 3 // 7)]
        batch = np.concatenate([fresh, rep])
        batch = batch[rng.permutation(batch.size)]
        got = t.insert(_dev(batch, w, gpu)).cpu().numpy()
        want = o.insert(batch)
        assert (want != oracle.FULL).all() and (got != cpht.FULL).all()
        ok, msg = sets.check_insert_outcomes(S, batch, got)
        assert ok, f"batch {b}: {msg}"
        S = np.union1d(S, batch)
        assert np.array_equal(check_table(t), S)
        assert t.count()[0] == S.size == o.occupied()
    assert S.size > cap and t.level3_used() > 0
    q = np.concatenate([pool_keys, host_u64(synth.distinct_keys(w, KEY_SEED + w, n_distinct, 5000))])
    assert np.array_equal(t.find(_dev(q, w, gpu)).cpu().numpy(), o.find(q))


def test_level3_one_list_link_races(gpu):
    """All overflow into a single list: every lane that finds the last slab
    full races to link the next one; only the lane that reserves the link
    takes a slab, so the pool holds exactly the slabs on the list."""
    w = 28
    t = _table(w, 8, 5, 16, 32, 32, 2, 0, 2000)
    keys = synth.distinct_keys(w, KEY_SEED, 0, 20000)
    out = t.insert(to_dev(keys, w, gpu)).cpu().numpy()
    assert (out == cpht.PUT).all()
    assert np.array_equal(check_table(t), np.sort(host_u64(keys)))
    used = t.level3_used()
    heads = t.export(3).view(np.uint32)
    pool = t.export(2).view(np.uint32).reshape(-1, 32)
    chain, id_ = 0, int(heads[0])
    while id_:
        chain += 1
        id_ = int(pool[id_ - 1, 31])
    assert chain == used  # no slab taken outside the list
    l3_keys = int(((pool[:, :31] >> 31) == 1).sum())
    assert l3_keys > 0 and used == -(-l3_keys // 31)  # slabs filled in order, only the last one partly
    assert int(t.find(to_dev(keys, w, gpu)).sum().item()) == 20000


def test_level3_pool_exhaustion(gpu):
    w = 20
    t = _table(w, 9, 6, 16, 16, 32, 2, 2, 12)
    o = oracle_table(t)
    keys_h = host_u64(synth.distinct_keys(w, KEY_SEED + 1, 0, 3000))
    got = t.insert(_dev(keys_h, w, gpu)).cpu().numpy()
    want = o.insert(keys_h)
    full = keys_h[got == cpht.FULL]
    stored = keys_h[got == cpht.PUT]
    assert full.size > 0 and (want == oracle.FULL).sum() > 0
    assert stored.size + full.size == keys_h.size
    assert t.count()[0] == stored.size
    assert t.level3_used() == 12
    assert np.array_equal(check_table(t), np.sort(stored))
    assert int(t.find(_dev(full, w, gpu)).sum().item()) == 0
    # at most the bucket slots and every key slot of the pool (lost link races
    # leave slabs unused, so the parallel run may store fewer than the oracle)
    assert stored.size <= t.count()[1] + 12 * 31
    assert int((want == oracle.PUT).sum()) <= t.count()[1] + 12 * 31


def test_level3_delete_mixed_and_reinsert(gpu):
    w = 32
    t = _table(w, 10, 7, 32, 32, 32, 4, 3, 500)
    o = oracle_table(t)
    keys_h = host_u64(synth.distinct_keys(w, KEY_SEED + 2, 0, 4000))
    assert (t.insert(_dev(keys_h, w, gpu)) == cpht.PUT).all()
    o.insert(keys_h)
    gone = keys_h[::3]
    got = t.delete(_dev(gone, w, gpu)).cpu().numpy()
    assert (got == 1).all() and (o.delete(gone) == 1).all()
    S = np.setdiff1d(keys_h, gone)
    assert np.array_equal(check_table(t), S)
    assert np.array_equal(t.find(_dev(keys_h, w, gpu)).cpu().numpy(), o.find(keys_h))
    # a mixed batch over the overflowing table: finds of stored keys, finds of
    # deleted keys, find-or-puts of deleted and fresh keys
    fresh = host_u64(synth.distinct_keys(w, KEY_SEED + 2, 4000, 800))
    kk = np.concatenate([S[:1500], gone, fresh])
    ops = np.concatenate([np.zeros(1500, np.uint8), np.ones(gone.size + fresh.size, np.uint8)])
    perm = np.random.default_rng(5).permutation(kk.size)
    kk, ops = kk[perm], ops[perm]
    got = t.mixed(_dev(kk, w, gpu), torch.from_numpy(ops).to(gpu)).cpu().numpy()
    want, S_after, racy = sets.mixed(S, kk, ops)
    fixed = ~racy
    assert np.array_equal(got[fixed & (ops == 0)], want[fixed & (ops == 0)])
    ok, msg = sets.check_insert_outcomes(S, kk[ops == 1], got[ops == 1])
    assert ok, msg
    assert np.array_equal(check_table(t), S_after)


def test_level3_config_checks(gpu):
    with pytest.raises(cpht.CphtError):  # 64-bit slots with 32-lane sub-tiles: no level 3
        _table(40, 12, 9, 64, 64, 64, 32, 2, 10)
    _table(40, 16, 14, 32, 32, 32, 4, 9, 10)  # levels 1-2 and the lists fit
    with pytest.raises(cpht.CphtError):  # w - log2_lists + 1 must fit the 32-bit slab slots
        _table(40, 16, 14, 32, 32, 32, 4, 2, 10)
    c = cpht.default_config(cpht.ICEBERG)
    c.key_bits, c.log2_slots0, c.log2_slots1, c.pool_slabs, c.log2_lists = 20, 10, 7, 10, 2
    with pytest.raises(cpht.CphtError):  # no level 3 inside table sets
        cpht.MultiTable([c, c], max_keys=100)
    t = _table(18, 10, 7, 16, 16, 16, 2, 3, 50)
    assert t.nimages == 4 and t.level_bytes(2) == 50 * 128 and t.level_bytes(3) == 8 * 4
    t2 = cpht.Table(scheme=cpht.ICEBERG, key_bits=18, log2_slots0=10, log2_slots1=7, bucket0=16, bucket1=8,
                    slot_bits0=16, slot_bits1=16)
    with pytest.raises(cpht.CphtError):
        t2.level3_used()
