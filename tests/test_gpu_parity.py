"""GPU parity tests: the HIP library (through the C-ABI) against the oracle.

Bars (all exact, the method is integer work):
  * the key split a_i(k) / stored form: bit-exact per key;
  * find answers after a completed build/insert: bit-exact per key;
  * the decoded key set of the GPU table equals the oracle's set;
  * insert outcomes: per distinct key, PUT exactly once for new keys and
    FOUND otherwise (which duplicate gets the PUT is timing-dependent);
  * at and above the failure load: the checker invariants of Appendix A
    (well-formed, no duplicates, order property), Theorem 1 (e) for FULL
    answers, and outcome accounting; fill factors are reported beside the
    sequential oracle's.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import paper_2406_09255_amd as cpht
import synth
from oracle import sets
from tests.helpers import check_table, host_u64, images, oracle_cfg, oracle_table, to_dev

pytestmark = pytest.mark.gpu

KEY_SEED = 0x5EED0001
Q_SEED = 0x5EED0002


def _sync():
    torch.cuda.synchronize()


def cuckoo(w, log2_slots, B, S=32, compact=1, seed=1, H=2, C=256, subtile=0):
    return cpht.Table(scheme=cpht.CUCKOO, key_bits=w, log2_slots0=log2_slots, bucket0=B, slot_bits0=S,
                      n_hash=H, max_chain=C, compact=compact, seed=seed, subtile=subtile)


def iceberg(w, log2_slots0, B0, S0, S1, log2_slots1=None, compact=1, seed=1, subtile=0):
    if log2_slots1 is None:
        log2_slots1 = log2_slots0 - 3
    return cpht.Table(scheme=cpht.ICEBERG, key_bits=w, log2_slots0=log2_slots0, log2_slots1=log2_slots1,
                      bucket0=B0, bucket1=B0 // 2, slot_bits0=S0, slot_bits1=S1, compact=compact, seed=seed,
                      subtile=subtile)


# ---------------------------------------------------------------------------
# the split (quotienting permutation)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("w,log2_slots,B,S,compact", [
    (32, 17, 32, 32, 1), (37, 20, 32, 32, 1), (37, 20, 16, 64, 0), (20, 12, 8, 32, 1), (60, 14, 16, 64, 1),
])
def test_split_cuckoo_bit_exact(gpu, w, log2_slots, B, S, compact):
    t = cuckoo(w, log2_slots, B, S, compact=compact, seed=0xC0FFEE + w)
    o = oracle_table(t)
    keys = synth.distinct_keys(w, KEY_SEED, 0, 5000)
    dk = to_dev(keys, w, gpu)
    for j in range(2):
        a, e = t.split(j, dk)
        _sync()
        oa, oe = o.split(j, host_u64(keys))
        assert np.array_equal(a.cpu().numpy().astype(np.uint64), oa)
        assert np.array_equal(e.cpu().numpy().astype(np.uint64), oe)


@pytest.mark.parametrize("w,L0,S0,S1,compact", [(34, 24, 16, 32, 1), (32, 18, 32, 32, 1), (24, 18, 16, 16, 1),
                                                 (50, 18, 64, 64, 0)])
def test_split_iceberg_bit_exact(gpu, w, L0, S0, S1, compact):
    t = iceberg(w, L0, 32, S0, S1, compact=compact, seed=77 + w)
    o = oracle_table(t)
    keys = synth.distinct_keys(w, KEY_SEED, 0, 4097)
    dk = to_dev(keys, w, gpu)
    for i in range(3):
        a, e = t.split(i, dk)
        _sync()
        oa, oe = o.split(i, host_u64(keys))
        assert np.array_equal(a.cpu().numpy().astype(np.uint64), oa), i
        assert np.array_equal(e.cpu().numpy().astype(np.uint64), oe), i


# ---------------------------------------------------------------------------
# compact cuckoo: bulk build + find
# ---------------------------------------------------------------------------

def test_c1_cuckoo_build_then_find(gpu):
    """Cuckoo H=2, 2^17 slots in 2^12 buckets of 32 x 32-bit slots, w=32:
    bulk insert 104,857 keys (load 0.8), then 10^5 finds with 50 % hits."""
    w, n = 32, 104857
    t = cuckoo(w, 17, 32, 32, seed=1)
    keys = synth.distinct_keys(w, KEY_SEED, 0, n)
    out = t.bulk_build(to_dev(keys, w, gpu))
    _sync()
    assert (out.cpu().numpy() == cpht.PUT).all()
    S = np.sort(host_u64(keys))
    dec = check_table(t)
    assert np.array_equal(dec, S)
    occ, cap = t.count()
    assert (occ, cap) == (n, 1 << 17)
    q = synth.find_queries(w, KEY_SEED, n, 100000, 0.5, Q_SEED)
    f = t.find(to_dev(q, w, gpu)).cpu().numpy()
    assert np.array_equal(f, sets.find(S, host_u64(q)))
    # the sequential model answers the same on its own table
    o = oracle_table(t)
    assert (o.insert(S) == oracle.PUT).all()
    assert np.array_equal(o.find(host_u64(q)), f)


@pytest.mark.parametrize("S,compact", [(32, 1), (64, 0)])
@pytest.mark.parametrize("B", [8, 16, 32])
@pytest.mark.parametrize("load", [0.5, 0.8, 0.9, 0.95])
def test_cuckoo_scaled_c2(gpu, S, compact, B, load):
    """Static build then finds, 2^20 slots, 37-bit keys, compact 32-bit vs
    non-compact 64-bit slots; finds 50 % hit / 50 % miss."""
    w, L2 = 37, 20
    n = int(load * (1 << L2))
    t = cuckoo(w, L2, B, S, compact=compact, seed=1000 + B)
    keys = synth.distinct_keys(w, KEY_SEED + B, 0, n)
    out = t.bulk_build(to_dev(keys, w, gpu)).cpu().numpy()
    S_in = np.sort(host_u64(keys))
    dec = check_table(t)
    nfull = int((out == cpht.FULL).sum())
    assert set(np.unique(out)) <= {cpht.PUT, cpht.FULL}
    assert dec.size == n - nfull  # every FULL drops exactly one carried key
    assert np.isin(dec, S_in).all()
    if nfull == 0:
        assert np.array_equal(dec, S_in)
    occ, _ = t.count()
    assert occ == dec.size
    q = synth.find_queries(w, KEY_SEED + B, n, 1 << 16, 0.5, Q_SEED)
    f = t.find(to_dev(q, w, gpu)).cpu().numpy()
    assert np.array_equal(f, sets.find(dec, host_u64(q)))


def test_cuckoo_forced_chain_failure(gpu):
    """C = 1 forces FULL as soon as a bucket is full: no key may be lost
    beyond the dropped carried keys, and the table stays well formed."""
    w = 24
    t = cuckoo(w, 12, 8, 32, seed=5, C=1)
    n = 4000
    keys = synth.distinct_keys(w, KEY_SEED, 0, n)
    out = t.bulk_build(to_dev(keys, w, gpu)).cpu().numpy()
    dec = check_table(t)
    nfull = int((out == cpht.FULL).sum())
    assert nfull > 0
    assert dec.size == n - nfull
    assert np.isin(dec, host_u64(keys)).all()


def test_cuckoo_three_hashes(gpu):
    w, n = 30, 60000
    t = cuckoo(w, 16, 16, 32, seed=9, H=3)
    keys = synth.distinct_keys(w, KEY_SEED, 0, n)
    out = t.bulk_build(to_dev(keys, w, gpu)).cpu().numpy()
    assert (out == cpht.PUT).all()
    dec = check_table(t)
    assert np.array_equal(dec, np.sort(host_u64(keys)))
    q = synth.find_queries(w, KEY_SEED, n, 30000, 0.5, Q_SEED)
    assert np.array_equal(t.find(to_dev(q, w, gpu)).cpu().numpy(), sets.find(dec, host_u64(q)))


@pytest.mark.parametrize("subtile", [2, 4, 8])
def test_cuckoo_subtile_widths_agree(gpu, subtile):
    w, n = 32, 90000
    t = cuckoo(w, 17, 32, 32, seed=3, subtile=subtile)
    keys = synth.distinct_keys(w, KEY_SEED, 0, n)
    out = t.bulk_build(to_dev(keys, w, gpu)).cpu().numpy()
    assert (out == cpht.PUT).all()
    assert np.array_equal(check_table(t), np.sort(host_u64(keys)))


# ---------------------------------------------------------------------------
# compact iceberg: find-or-put, find, mixed batches
# ---------------------------------------------------------------------------

def _ice_w(log2_slots0, B0, S0, log2_slots1, S1, compact, cap=34):
    """Largest key width <= cap that fits both levels' slots."""
    nb0 = log2_slots0 - int(np.log2(B0))
    nb1 = log2_slots1 - int(np.log2(B0 // 2))
    if not compact:
        return min(cap, S0 - 1, S1 - 2)
    return min(cap, nb0 + S0 - 1, nb1 + S1 - 2)


ICE_SHAPES = [(8, 16, 32), (16, 16, 32), (32, 16, 32), (64, 16, 32), (32, 16, 16), (32, 32, 32),
              (16, 32, 32), (32, 64, 64), (8, 64, 64)]


@pytest.mark.parametrize("B0,S0,S1", ICE_SHAPES)
def test_iceberg_fop_batches(gpu, B0, S0, S1):
    """Three find-or-put batches with 30 % duplicate keys, then finds; the
    table holds well under its failure load, so every outcome is fixed by the
    set semantics."""
    L0, L1 = 16, 13
    compact = 0 if S0 == 64 else 1
    w = _ice_w(L0, B0, S0, L1, S1, compact)
    t = iceberg(w, L0, B0, S0, S1, L1, compact=compact, seed=31 + B0)
    S_cur = np.zeros(0, np.uint64)
    issued = 0
    for b in range(3):
        keys, nf = synth.insert_stream_with_duplicates(w, KEY_SEED, issued, 15000 + 1237 * b, 0.3, 100 + b)
        issued += nf
        out = t.insert(to_dev(keys, w, gpu)).cpu().numpy()
        ok, msg = sets.check_insert_outcomes(S_cur, host_u64(keys), out)
        assert ok, f"batch {b}: {msg}"
        _, S_cur = sets.insert(S_cur, host_u64(keys))
        dec = check_table(t)
        assert np.array_equal(dec, S_cur)
    occ, cap = t.count()
    assert occ == S_cur.size
    q = synth.find_queries(w, KEY_SEED, issued, 40000, 0.5, Q_SEED)
    f = t.find(to_dev(q, w, gpu)).cpu().numpy()
    assert np.array_equal(f, sets.find(S_cur, host_u64(q)))
    o = oracle_table(t)
    o.insert(S_cur)
    assert np.array_equal(o.find(host_u64(q)), f)


def test_iceberg_same_key_everywhere(gpu):
    """Every lane of the grid find-or-puts the same key: exactly one PUT."""
    w = 34
    t = iceberg(w, 18, 32, 32, 32, seed=2)
    k = torch.full((1 << 16,), 123456789, dtype=torch.int64)
    out = t.insert(to_dev(k, w, gpu)).cpu().numpy()
    assert (out == cpht.PUT).sum() == 1 and (out == cpht.FOUND).sum() == out.size - 1
    assert check_table(t).tolist() == [123456789]


def test_iceberg_hot_keys(gpu):
    """A few keys repeated thousands of times across waves and XCDs, together
    with distinct keys: one PUT per key."""
    w = 34
    t = iceberg(w, 18, 32, 32, 32, seed=4)
    distinct = synth.distinct_keys(w, KEY_SEED, 0, 20000)
    hot = distinct[:7].repeat(3000)
    keys = torch.cat([distinct, hot])[synth.permutation(11, 20000 + 21000)]
    out = t.insert(to_dev(keys, w, gpu)).cpu().numpy()
    ok, msg = sets.check_insert_outcomes(np.zeros(0, np.uint64), host_u64(keys), out)
    assert ok, msg
    assert np.array_equal(check_table(t), np.sort(host_u64(distinct)))


@pytest.mark.parametrize("S0,S1", [(16, 32), (32, 32)])
def test_iceberg_until_full(gpu, S0, S1):
    """Insert twice the capacity: FULL answers appear.  Checked: invariants,
    Theorem 1 (e) for every FULL key, one PUT or all-FULL per new key, and
    #PUT equal to the occupied slots; fill factor reported beside the
    sequential oracle's."""
    w = 22
    L0, L1, B0 = 10, 7, 8
    t = iceberg(w, L0, B0, S0, S1, L1, seed=8)
    keys, _ = synth.insert_stream_with_duplicates(w, KEY_SEED, 0, 2 * ((1 << L0) + (1 << L1)), 0.2, 5)
    hk = host_u64(keys)
    out = t.insert(to_dev(keys, w, gpu)).cpu().numpy()
    dec = check_table(t)
    assert (out == cpht.FULL).any()
    uk, inv = np.unique(hk, return_inverse=True)
    puts = np.bincount(inv, weights=(out == cpht.PUT), minlength=uk.size)
    fulls = np.bincount(inv, weights=(out == cpht.FULL), minlength=uk.size)
    cnt = np.bincount(inv, minlength=uk.size)
    assert ((puts == 1) | (fulls == cnt)).all()
    assert (puts <= 1).all()
    assert np.array_equal(dec, np.sort(uk[puts == 1]))
    occ, cap = t.count()
    assert occ == int(puts.sum())
    img0, img1 = images(t)
    ok, msg = oracle.check_full(oracle_cfg(t), img0, img1, uk[fulls > 0])
    assert ok, msg
    o = oracle_table(t)
    o.insert(hk)
    print(f"fill at end: gpu {occ / cap:.4f}  oracle {o.occupied() / o.capacity():.4f}")


def test_iceberg_mixed_batch(gpu):
    """Mixed find / find-or-put batches (50/50) on a pre-filled table: inserts
    follow the set semantics per key; finds of keys present before the batch
    answer 1, of keys absent after it answer 0, and of keys inserted by the
    batch itself may answer either."""
    w = 30
    t = iceberg(w, 20, 32, 16, 32, seed=12)
    pre = synth.distinct_keys(w, KEY_SEED, 0, 60000)
    t.insert(to_dev(pre, w, gpu))
    S_cur = np.sort(host_u64(pre))
    issued = 60000
    for b in range(3):
        n = 50000 + 313 * b
        ins, nf = synth.insert_stream_with_duplicates(w, KEY_SEED, issued, n, 0.3, 40 + b)
        issued += nf
        q = synth.find_queries(w, KEY_SEED, issued, n, 0.5, 50 + b)
        keys = torch.cat([ins, q])
        ops = torch.cat([torch.ones(n, dtype=torch.uint8), torch.zeros(n, dtype=torch.uint8)])
        perm = synth.permutation(60 + b, 2 * n)
        keys, ops = keys[perm], ops[perm]
        out = t.mixed(to_dev(keys, w, gpu), ops.to(gpu)).cpu().numpy()
        hk, ho = host_u64(keys), ops.numpy()
        seq, S_after, racy = sets.mixed(S_cur, hk, ho)
        ins_m = ho == 1
        ok, msg = sets.check_insert_outcomes(S_cur, hk[ins_m], out[ins_m])
        assert ok, msg
        fixed = (~ins_m) & ~racy
        assert np.array_equal(out[fixed], seq[fixed])
        assert np.isin(out[racy], [0, 1]).all()
        S_cur = S_after
        assert np.array_equal(check_table(t), S_cur)


# ---------------------------------------------------------------------------
# edge cases
# ---------------------------------------------------------------------------

def test_empty_batches(gpu):
    t = iceberg(26, 16, 32, 16, 32)
    e = torch.empty(0, dtype=torch.int32, device=gpu)
    assert t.insert(e).numel() == 0
    assert t.find(e).numel() == 0
    assert t.mixed(e, torch.empty(0, dtype=torch.uint8, device=gpu)).numel() == 0
    assert t.count()[0] == 0
    c = cuckoo(32, 12, 32)
    assert c.bulk_build(torch.empty(0, dtype=torch.int32, device=gpu)).numel() == 0


@pytest.mark.parametrize("n", [1, 7, 63, 64, 65, 255, 257, 1000 + 37])
def test_ragged_batch_sizes(gpu, n):
    w = 26
    t = iceberg(w, 16, 32, 16, 32, seed=n)
    keys = synth.distinct_keys(w, KEY_SEED, 0, n)
    out = t.insert(to_dev(keys, w, gpu)).cpu().numpy()
    assert (out == cpht.PUT).all()
    assert np.array_equal(check_table(t), np.sort(host_u64(keys)))
    c = cuckoo(w, 16, 32, 32, seed=n)
    out = c.bulk_build(to_dev(keys, w, gpu)).cpu().numpy()
    assert (out == cpht.PUT).all()
    f = c.find(to_dev(keys, w, gpu)).cpu().numpy()
    assert (f == 1).all()


def test_single_bucket_levels(gpu):
    """Degenerate shapes: one primary bucket and one secondary bucket (both
    secondary permutations then address the same bucket)."""
    w = 12
    t = iceberg(w, 3, 8, 32, 32, log2_slots1=2)
    keys = synth.distinct_keys(w, KEY_SEED, 0, 40)
    out = t.insert(to_dev(keys, w, gpu)).cpu().numpy()
    dec = check_table(t)
    assert (out == cpht.PUT).sum() == 12 and (out == cpht.FULL).sum() == 28
    assert np.array_equal(dec, np.sort(host_u64(keys)[out == cpht.PUT]))
    f = t.find(to_dev(keys, w, gpu)).cpu().numpy()
    assert np.array_equal(f, (out == cpht.PUT).astype(np.uint8))


def test_zero_bit_remainders(gpu):
    """The address takes every key bit (w = log2 #buckets, so the remainder
    has no bits, Sec. 2.4): a slot then holds only the occupancy bit and the
    hash tag, and since each permutation is a bijection every key owns its
    own primary (iceberg) or first (cuckoo) bucket.  The whole key domain
    goes in with PUT, no key moves or overflows, and every lookup hits."""
    w = 10
    keys = synth.distinct_keys(w, KEY_SEED, 0, 1 << w)
    dk = to_dev(keys, w, gpu)
    t = iceberg(w, 15, 32, 16, 16, log2_slots1=12)  # 2^10 primary buckets
    o = oracle_table(t)
    out = t.insert(dk).cpu().numpy()
    assert (out == cpht.PUT).all() and (o.insert(host_u64(keys)) == oracle.PUT).all()
    assert np.array_equal(check_table(t), np.arange(1 << w, dtype=np.uint64))
    for got, want in zip(images(t), [o.export(0), o.export(1)]):
        assert np.array_equal(got, want)  # the placement is forced: images are bit-exact
    assert (t.insert(dk).cpu().numpy() == cpht.FOUND).all()
    assert (t.find(dk).cpu().numpy() == 1).all()
    c = cuckoo(w, 15, 32, 32)  # 2^10 buckets of 32 slots
    oc = oracle_table(c)
    assert (c.bulk_build(dk).cpu().numpy() == cpht.PUT).all()
    oc.insert(host_u64(keys))
    # the bucket of every key is forced (one key per bucket, hash 0); the put
    # may take any empty slot of it, so compare each bucket's one stored form
    got = images(c)[0].view(np.uint32).reshape(-1, 32)
    want = oc.export(0).view(np.uint32).reshape(-1, 32)
    assert ((got != 0).sum(1) == 1).all() and ((want != 0).sum(1) == 1).all()
    assert np.array_equal(got.max(1), want.max(1))
    assert np.array_equal(check_table(c), np.arange(1 << w, dtype=np.uint64))
    assert (c.find(dk).cpu().numpy() == 1).all()


@pytest.mark.parametrize("scheme", ["cuckoo", "iceberg"])
def test_full_width_64_bit_keys(gpu, scheme):
    """w = 64: keys use every bit of their word (the permutations work mod
    2^64); compact 64-bit slots store the 64 - log2 #buckets remainder bits."""
    w = 64
    if scheme == "cuckoo":
        t = cuckoo(w, 16, 16, 64)
    else:
        t = iceberg(w, 16, 32, 64, 64, log2_slots1=13)
    o = oracle_table(t)
    keys = synth.distinct_keys(w, KEY_SEED, 0, int(0.85 * (1 << 16)))
    kh = host_u64(keys)
    assert (kh >> np.uint64(63)).any()  # keys with the top bit set are in the batch
    out = (t.bulk_build if scheme == "cuckoo" else t.insert)(to_dev(keys, w, gpu)).cpu().numpy()
    assert (out == cpht.PUT).all() and (o.insert(kh) == oracle.PUT).all()
    assert np.array_equal(check_table(t), np.sort(kh))
    q = synth.find_queries(w, KEY_SEED, kh.size, 30000, 0.5, 9)
    assert np.array_equal(t.find(to_dev(q, w, gpu)).cpu().numpy(), o.find(host_u64(q)))


def test_clear_and_reseed(gpu):
    w = 32
    t = cuckoo(w, 16, 32, 32, seed=1)
    keys = synth.distinct_keys(w, KEY_SEED, 0, 50000)
    dk = to_dev(keys, w, gpu)
    t.bulk_build(dk)
    for seed in (2, 3):
        t.clear(seed)
        assert t.count()[0] == 0
        out = t.bulk_build(dk).cpu().numpy()
        assert (out == cpht.PUT).all()
        assert t.config.seed == seed
        assert np.array_equal(check_table(t), np.sort(host_u64(keys)))


def test_unsupported_configs_rejected(gpu):
    with pytest.raises(cpht.CphtError):
        cuckoo(40, 12, 32, 32)  # 40 - 7 = 33 remainder bits + tag + occupancy > 32
    with pytest.raises(cpht.CphtError):
        cuckoo(32, 12, 32, 16)  # no 16-bit cuckoo slots
    with pytest.raises(cpht.CphtError):
        iceberg(34, 10, 32, 16, 32)  # 34 - 5 = 29 remainder bits in a 16-bit slot
    t = cuckoo(32, 12, 32, 32)
    with pytest.raises(cpht.CphtError):
        t.mixed(torch.zeros(4, dtype=torch.int32, device=gpu), torch.zeros(4, dtype=torch.uint8, device=gpu))


# ---------------------------------------------------------------------------
# contention: many keys of one batch aimed at the same few buckets
# ---------------------------------------------------------------------------

def _keys_in_buckets(t, level, perm_index, w, nbuckets, count, seed):
    """Distinct keys whose bucket under perm_index is one of `nbuckets`
    buckets (selected with the oracle's own split)."""
    o = oracle_table(t)
    cand = host_u64(synth.distinct_keys(w, seed, 0, 1 << 21))
    a, _ = o.split(perm_index, cand)
    chosen = np.unique(a)[:nbuckets]
    pick = cand[np.isin(a, chosen)][:count]
    assert pick.size == count
    return torch.from_numpy(pick.astype(np.int64))


@pytest.mark.parametrize("S0,S1", [(16, 32), (32, 32), (16, 16)])
def test_iceberg_colliding_primary_buckets(gpu, S0, S1):
    """Keys of a batch share 6 primary buckets, so claims collide, primaries
    overflow into the secondary level and some keys come back FULL; keys are
    also repeated.  Outcomes must still follow Theorem 1."""
    w = 26 if S1 == 32 else 23
    t = iceberg(w, 16, 32, S0, S1, seed=71)
    base = _keys_in_buckets(t, 0, 0, w, 6, 600, 3)
    keys = torch.cat([base, base[:200], base[::3]])[synth.permutation(5, 600 + 200 + 200)]
    hk = host_u64(keys)
    out = t.insert(to_dev(keys, w, gpu)).cpu().numpy()
    dec = check_table(t)
    uk, inv = np.unique(hk, return_inverse=True)
    puts = np.bincount(inv, weights=(out == cpht.PUT), minlength=uk.size)
    fulls = np.bincount(inv, weights=(out == cpht.FULL), minlength=uk.size)
    cnt = np.bincount(inv, minlength=uk.size)
    assert (puts <= 1).all() and ((puts == 1) | (fulls == cnt)).all()
    assert np.array_equal(dec, np.sort(uk[puts == 1]))
    img0, img1 = images(t)
    ok, msg = oracle.check_full(oracle_cfg(t), img0, img1, uk[fulls > 0])
    assert ok, msg
    f = t.find(to_dev(keys, w, gpu)).cpu().numpy()
    assert np.array_equal(f, np.isin(hk, dec).astype(np.uint8))


def test_cuckoo_colliding_first_buckets(gpu):
    """600 keys whose first bucket is one of 8 buckets: 256 fit there, the
    rest are placed by evictions; no key may be lost."""
    w = 30
    t = cuckoo(w, 16, 32, 32, seed=72)
    keys = _keys_in_buckets(t, 0, 0, w, 8, 600, 4)
    out = t.bulk_build(to_dev(keys, w, gpu)).cpu().numpy()
    dec = check_table(t)
    nfull = int((out == cpht.FULL).sum())
    assert dec.size == 600 - nfull and np.isin(dec, host_u64(keys)).all()
    assert nfull == 0
    f = t.find(to_dev(keys, w, gpu)).cpu().numpy()
    assert (f == 1).all()


def test_iceberg_high_load_parity(gpu):
    """Fill a compact iceberg table (2^20 + 2^17 slots, B0 = 32) in 8 batches
    of distinct keys to load 0.875; every batch must match the set semantics
    unless FULL appears, and finds after each batch are bit-exact."""
    w = 30
    t = iceberg(w, 20, 32, 16, 32, seed=73)
    cap = (1 << 20) + (1 << 17)
    S_cur = np.zeros(0, np.uint64)
    per = cap // 8
    for b in range(7):
        keys = synth.distinct_keys(w, KEY_SEED, b * per, per)
        out = t.insert(to_dev(keys, w, gpu)).cpu().numpy()
        hk = host_u64(keys)
        if (out == cpht.FULL).any():
            break
        ok, msg = sets.check_insert_outcomes(S_cur, hk, out)
        assert ok, msg
        _, S_cur = sets.insert(S_cur, hk)
        q = synth.find_queries(w, KEY_SEED, (b + 1) * per, 1 << 16, 0.5, b)
        f = t.find(to_dev(q, w, gpu)).cpu().numpy()
        assert np.array_equal(f, sets.find(S_cur, host_u64(q)))
    assert np.array_equal(check_table(t), S_cur)
    assert S_cur.size >= 6 * per
