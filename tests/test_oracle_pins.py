"""Pins of the CPU oracle against facts that do not come from the oracle.

Each test ties one part of the oracle to something fixed by the paper or by
mathematics: published generator outputs, the worked examples of Sec. 5.1
and Figure 5, bijectivity and inverses checked exhaustively, brute force on
tiny key domains, the set semantics of Theorem 1, and planted corruptions
that the table checker must reject.
"""
from __future__ import annotations

import os

import numpy as np
import pytest

import oracle
from oracle import sets

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_lines(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [l.strip() for l in f if l.strip() and not l.startswith("#")]


def _rng(seed):
    return np.random.default_rng(seed)


# ---------------------------------------------------------------------------
# splitmix64 and the permutation family (Sec. 2.4)
# ---------------------------------------------------------------------------

def test_splitmix64_published_outputs():
    want = [int(v, 16) for v in _golden_lines("splitmix64_seed0.txt")]
    assert [oracle.sm64(0, i) for i in range(3)] == want


def test_multiplicative_inverse_mod_2w():
    r = _rng(1)
    for w in list(range(1, 65)):
        for _ in range(20):
            m = int(r.integers(0, 2**63)) * 2 + 1
            m &= (1 << w) - 1 if w < 64 else (1 << 64) - 1
            m |= 1
            inv = oracle.mulinv(m, w)
            assert (m * inv) % (1 << w) == 1 % (1 << w), (w, m)


@pytest.mark.parametrize("w", list(range(1, 21)))
def test_permutation_is_a_bijection_exhaustive(w):
    x = np.arange(1 << w, dtype=np.uint64)
    for i in range(3):
        for seed in (0, 1, 0xDEADBEEF):
            y = oracle.perm(w, seed, i, x)
            assert y.max() < (1 << w)
            assert np.unique(y).size == x.size
            assert np.array_equal(oracle.perm(w, seed, i, y, inverse=True), x)


@pytest.mark.parametrize("w", [24, 31, 32, 33, 34, 37, 40, 52, 63, 64])
def test_permutation_round_trip_random(w):
    r = _rng(w)
    x = r.integers(0, 2**63, size=200000, dtype=np.int64).astype(np.uint64) * np.uint64(2)
    x ^= r.integers(0, 2, size=x.size, dtype=np.int64).astype(np.uint64)
    if w < 64:
        x &= np.uint64((1 << w) - 1)
    for i in range(3):
        y = oracle.perm(w, 99, i, x)
        if w < 64:
            assert (y < np.uint64(1 << w)).all()
        assert np.array_equal(oracle.perm(w, 99, i, y, inverse=True), x)


def test_permutations_differ_by_index_and_seed():
    x = np.arange(4096, dtype=np.uint64)
    a = oracle.perm(32, 1, 0, x)
    assert not np.array_equal(a, oracle.perm(32, 1, 1, x))
    assert not np.array_equal(a, oracle.perm(32, 2, 0, x))


@pytest.mark.parametrize("w,nb", [(32, 12), (37, 22), (20, 10)])
def test_addresses_spread_uniformly(w, nb):
    """Consecutive keys must land in buckets like uniform draws (chi-square,
    mean and variance of the counts); taking the address from the key itself
    instead of pi(k) would pile consecutive keys into a few buckets."""
    n = 16 << nb if nb <= 12 else 1 << 22
    x = np.arange(n, dtype=np.uint64)
    a, _ = oracle.split(w, nb, 5, 0, x)
    counts = np.bincount(a.astype(np.int64), minlength=1 << nb)
    exp = n / (1 << nb)
    chi2 = ((counts - exp) ** 2 / exp).sum()
    dof = (1 << nb) - 1
    assert abs(chi2 - dof) < 6 * np.sqrt(2 * dof), chi2


def test_split_joins_back():
    """k = pi^-1(a(k) . r(k)) (Sec. 2.4)."""
    w, nb = 37, 22
    x = _rng(3).integers(0, 1 << w, size=100000, dtype=np.int64).astype(np.uint64)
    a, r = oracle.split(w, nb, 17, 1, x)
    joined = (a << np.uint64(w - nb)) | r
    assert np.array_equal(oracle.perm(w, 17, 1, joined, inverse=True), x)


# ---------------------------------------------------------------------------
# worked examples of the paper
# ---------------------------------------------------------------------------

def test_width_example_sec_5_1():
    for line in _golden_lines("width_example.txt"):
        log2_slots, B, s, t, nb, wmax = map(int, line.split())
        assert log2_slots - int(np.log2(B)) == nb
        assert oracle.max_key_bits(log2_slots, B, s, t) == wmax
    # the same rule decides which small tables the model accepts
    oracle.Table(oracle.ICEBERG, 10 + 15, 15, 32, 16, log2_slots1=12, B1=16, s1=32)
    with pytest.raises(ValueError):
        oracle.Table(oracle.ICEBERG, 10 + 16, 15, 32, 16, log2_slots1=12, B1=16, s1=32)


def test_memory_ratio_sec_5_1():
    """Compact 32-bit vs 64-bit slots use half the memory; 16-bit primary /
    32-bit secondary iceberg uses (2^27*16 + 2^24*32)/((2^27+2^24)*64) = 5/18
    (the text prints 9/32; the arithmetic gives 5/18)."""
    from fractions import Fraction

    assert Fraction(32, 64) == Fraction(1, 2)
    r = Fraction(2**27 * 16 + 2**24 * 32, (2**27 + 2**24) * 64)
    assert r == Fraction(5, 18)
    t = oracle.Table(oracle.ICEBERG, 20, 13, 32, 16, log2_slots1=10, B1=16, s1=32)
    u = oracle.Table(oracle.ICEBERG, 20, 13, 32, 64, log2_slots1=10, B1=16, s1=64, compact=False)
    got = Fraction(sum(t.export(x).size for x in (0, 1)), sum(u.export(x).size for x in (0, 1)))
    assert got == Fraction(5, 18)


def test_figure5_slot_order():
    lines = _golden_lines("fig5_slot_order.txt")
    B0, B1 = (int(f.split("=")[1]) for f in lines[0].split())
    want = [tuple(map(int, l.split()[1:])) for l in lines[1:]]
    assert oracle.order_list(B0, B1) == want
    # pairwise: the order is strict and total on distinct slots
    for i, a in enumerate(want):
        for j, b in enumerate(want):
            assert oracle.order_less(a, b) == (i < j)


# ---------------------------------------------------------------------------
# sequential models against the plain set semantics (Theorem 1)
# ---------------------------------------------------------------------------

def _stream(r, domain_bits, n, dup_frac):
    fresh = r.choice(1 << domain_bits, size=n, replace=False).astype(np.uint64)
    out = fresh.copy()
    dup = r.random(n) < dup_frac
    dup[0] = False
    idx = np.nonzero(dup)[0]
    out[idx] = out[(r.random(idx.size) * idx).astype(np.int64)]
    return out


@pytest.mark.parametrize("B0,s0,s1", [(32, 16, 32), (8, 32, 32), (16, 64, 64)])
def test_iceberg_model_matches_set_semantics(B0, s0, s1):
    r = _rng(B0 + s0)
    compact = s0 != 64
    t = oracle.Table(oracle.ICEBERG, 24, 14, B0, s0, log2_slots1=11, B1=B0 // 2, s1=s1, compact=compact, seed=4)
    S = np.zeros(0, np.uint64)
    for b in range(3):
        keys = _stream(r, 24, 3000, 0.3)
        out = t.insert(keys)
        want, S = sets.insert(S, keys)
        assert np.array_equal(out, want)
        ok, msg, dec = t.check()
        assert ok, msg
        assert np.array_equal(dec, S)
    q = r.integers(0, 1 << 24, size=20000).astype(np.uint64)
    q[:5000] = S[r.integers(0, S.size, 5000)]
    assert np.array_equal(t.find(q), sets.find(S, q))
    assert t.occupied() == S.size


@pytest.mark.parametrize("B,s,compact", [(32, 32, True), (8, 32, True), (16, 64, False)])
def test_cuckoo_model_loses_no_key(B, s, compact):
    r = _rng(B)
    t = oracle.Table(oracle.CUCKOO, 30, 16, B, s, compact=compact, seed=6)
    keys = r.choice(1 << 30, size=int(0.85 * (1 << 16)), replace=False).astype(np.uint64)
    out = t.insert(keys)
    assert (out == oracle.PUT).all()
    ok, msg, dec = t.check()
    assert ok, msg
    assert np.array_equal(dec, np.sort(keys))
    q = np.concatenate([keys[:3000], r.integers(0, 1 << 30, 3000).astype(np.uint64)])
    assert np.array_equal(t.find(q), sets.find(np.sort(keys), q))


def test_mixed_model_is_sequential_semantics():
    r = _rng(8)
    t = oracle.Table(oracle.ICEBERG, 22, 14, 32, 16, log2_slots1=11, B1=16, s1=32, seed=3)
    keys = _stream(r, 22, 6000, 0.4)
    ops = (r.random(keys.size) < 0.5).astype(np.uint8)
    out = t.mixed(keys, ops)
    want, S, racy = sets.mixed(np.zeros(0, np.uint64), keys, ops)
    assert np.array_equal(out, want)


def test_fill_factors_reached():
    """Sec. 5.2: cuckoo tables with 32-slot buckets reach fill factor 0.95;
    the 2-level iceberg table with B0 = 32 reaches 0.9 but not 0.95 (a soft
    pin: it depends on the permutations and the chain bound)."""
    r = _rng(9)
    keys = r.choice(1 << 34, size=1 << 18, replace=False).astype(np.uint64)
    c = oracle.Table(oracle.CUCKOO, 34, 18, 32, 32, seed=2)
    n95 = int(0.95 * (1 << 18))
    assert (c.insert(keys[:n95]) == oracle.PUT).all()
    ice = oracle.Table(oracle.ICEBERG, 34, 18, 32, 32, log2_slots1=15, B1=16, s1=32, seed=2)
    cap = (1 << 18) + (1 << 15)
    more = r.choice(1 << 34, size=cap, replace=False).astype(np.uint64)
    out = ice.insert(more)
    first_full = int(np.argmax(out == oracle.FULL)) if (out == oracle.FULL).any() else cap
    ff = first_full / cap
    assert 0.9 <= ff < 0.95, ff


# ---------------------------------------------------------------------------
# brute force over a whole tiny key domain
# ---------------------------------------------------------------------------

def _buckets_full_without(img, s, B, bucket, stored):
    """Raw-image test: bucket `bucket` of a level has no EMPTY slot and does
    not hold `stored` (slots little endian, s bits)."""
    sb = s // 8
    raw = img[bucket * B * sb:(bucket + 1) * B * sb].reshape(B, sb).astype(np.uint64)
    vals = (raw << (np.arange(sb, dtype=np.uint64) * np.uint64(8))).sum(axis=1)
    return bool((vals != 0).all() and not (vals == stored).any())


def test_iceberg_brute_force_tiny_domain():
    """Every key of a 2^10 domain, in random order, into 4 primary buckets of
    4 slots and 2 secondary buckets of 2 slots.  After the run: a key is
    found iff some insert of it returned PUT; each FULL key has three full
    buckets without it (checked directly on the raw image); the table holds
    exactly the PUT keys."""
    w = 10
    t = oracle.Table(oracle.ICEBERG, w, 4, 4, 32, log2_slots1=2, B1=2, s1=32, seed=21)
    keys = _rng(10).permutation(1 << w).astype(np.uint64)
    out = t.insert(keys)
    assert set(np.unique(out)) <= {oracle.PUT, oracle.FULL}
    put = np.sort(keys[out == oracle.PUT])
    assert put.size == 16 + 4  # every slot filled
    ok, msg, dec = t.check()
    assert ok, msg
    assert np.array_equal(dec, put)
    domain = np.arange(1 << w, dtype=np.uint64)
    assert np.array_equal(t.find(domain), np.isin(domain, put).astype(np.uint8))
    img0, img1 = t.export(0), t.export(1)
    for k in keys[out == oracle.FULL][:200]:
        k = int(k)
        for lvl, i, B in ((0, 0, 4), (1, 1, 2), (1, 2, 2)):
            b = t.bucket_of(lvl, i, k)
            e = t.stored_form(lvl, i, k, 0 if i < 2 else 1)
            assert _buckets_full_without(img0 if lvl == 0 else img1, 32, B, b, e)


# ---------------------------------------------------------------------------
# the Theorem 1 (e) checker for FULL answers
# ---------------------------------------------------------------------------

# a tiny iceberg shape: 4 primary buckets of 4 x 32-bit slots (2 address
# bits, 8 payload bits), 2 secondary buckets of 2 x 32-bit slots (1 address
# bit, 9 payload bits, 1 tag bit), 10-bit keys
_TINY = dict(w=10, L0=4, B0=4, L1=2, B1=2, seed=31)


def _tiny_iceberg(seed):
    c = _TINY
    return oracle.Table(oracle.ICEBERG, c["w"], c["L0"], c["B0"], 32, log2_slots1=c["L1"], B1=c["B1"], s1=32,
                        seed=seed)


def _words(img):
    return img.view(np.uint32)


def _places(k, seed):
    """(level, first word, slots, stored form) of key k's three buckets,
    computed from the permutation and the documented slot layout
    (occupancy bit 31 | tag << payload bits | payload), not from the
    oracle's table code."""
    c = _TINY
    out = []
    for i, (lvl, L, B, tag) in enumerate(((0, c["L0"], c["B0"], 0), (1, c["L1"], c["B1"], 0),
                                         (1, c["L1"], c["B1"], 1))):
        nb = L - int(np.log2(B))
        a, r = oracle.split(c["w"], nb, seed, i, [k])
        p = c["w"] - nb
        out.append((lvl, int(a[0]) * B, B, (1 << 31) | (tag << p) | int(r[0])))
    return out


def _full_verdict_brute(imgs, k, seed):
    """Theorem 1 (e) for key k straight from the images: its primary bucket
    and both secondary buckets hold no EMPTY slot and not its stored form."""
    for lvl, at, B, e in _places(k, seed):
        words = _words(imgs[lvl])[at:at + B]
        if (words == 0).any() or (words == e).any():
            return False
    return True


@pytest.mark.parametrize("fill", [6, 12, 17, 20, 1 << 10])
def test_check_full_equals_brute_force_over_the_domain(fill):
    """For every key of the 2^10 domain, or_check_full accepts the key as a
    legitimate FULL answer exactly when the raw images say its three buckets
    are full without it; at several fills, so both full and non-full buckets,
    stored and absent keys occur."""
    seed = _TINY["seed"] + fill
    t = _tiny_iceberg(seed)
    keys = _rng(fill).permutation(1 << _TINY["w"]).astype(np.uint64)[:fill]
    out = t.insert(keys)
    imgs = [t.export(0), t.export(1)]
    accepted = 0
    for k in range(1 << _TINY["w"]):
        want = _full_verdict_brute(imgs, k, seed)
        got, msg = oracle.check_full(t.cfg, imgs[0], imgs[1], [k])
        assert got == want, f"fill {fill}, key {k}: checker says {got} ({msg}), images say {want}"
        accepted += got
    if fill == 1 << 10:  # every slot is taken: exactly the keys answered FULL are accepted
        assert accepted == int((out == oracle.FULL).sum()) == (1 << 10) - 20
    elif fill < 16:  # some primary bucket still has room: keys aimed there are rejected
        assert accepted < (1 << 10) - fill


def test_check_full_rejects_planted_violations():
    """On the whole-domain image (every slot full), for FULL keys: the
    checker accepts the oracle's own FULL answers and rejects each planted
    violation of Theorem 1 (e): the key stored in its primary bucket, in its
    first secondary bucket (tag 0) or in its second (tag 1); an EMPTY slot in
    any of the three buckets.  A stored form with the other secondary's tag
    is some other key, not a violation."""
    seed = _TINY["seed"]
    t = _tiny_iceberg(seed)
    keys = _rng(12).permutation(1 << _TINY["w"]).astype(np.uint64)
    out = t.insert(keys)
    full = keys[out == oracle.FULL]
    img0, img1 = t.export(0), t.export(1)
    ok, msg = oracle.check_full(t.cfg, img0, img1, full)
    assert ok, msg
    ok, _ = oracle.check_full(t.cfg, img0, img1, keys[out == oracle.PUT][:1])
    assert not ok  # a stored key is no FULL answer
    for k in full[:25]:
        k = int(k)
        places = _places(k, seed)
        for which, (lvl, at, B, e) in enumerate(places):
            for plant in ("store", "empty"):
                imgs = [img0.copy(), img1.copy()]
                words = _words(imgs[lvl])
                words[at + (k % B)] = e if plant == "store" else 0
                ok, msg = oracle.check_full(t.cfg, imgs[0], imgs[1], [k])
                assert not ok, f"key {k}: planted {plant} in bucket {which} accepted"
        # the second secondary bucket holding the key's payload under tag 0
        # (the first secondary's tag) stores another key: still a valid FULL
        lvl, at, B, e = places[2]
        p = _TINY["w"] - (_TINY["L1"] - 1)
        imgs = [img0.copy(), img1.copy()]
        _words(imgs[1])[at] = e & ~np.uint64(1 << p)
        ok, msg = oracle.check_full(t.cfg, imgs[0], imgs[1], [k])
        assert ok, f"key {k}: the other tag's form was taken for the key: {msg}"


def test_cuckoo_brute_force_tiny_domain():
    w = 10
    t = oracle.Table(oracle.CUCKOO, w, 5, 4, 32, seed=22, C=64)
    keys = _rng(11).permutation(1 << w)[:28].astype(np.uint64)
    out = t.insert(keys)
    ok, msg, dec = t.check()
    assert ok, msg
    nfull = int((out == oracle.FULL).sum())
    assert dec.size == keys.size - nfull
    assert np.isin(dec, keys).all()
    domain = np.arange(1 << w, dtype=np.uint64)
    assert np.array_equal(t.find(domain), np.isin(domain, dec).astype(np.uint8))


def test_zero_bit_remainder_images_are_forced():
    """When the bucket address takes all w key bits the remainder is empty
    and each permutation is a bijection onto the buckets, so the whole domain
    fills exactly slot 0 of every primary (first-hash) bucket with the bare
    occupancy bit and hash tag 0, whatever the permutation: the images are
    fixed without reference to the oracle's hashing."""
    w = 10
    t = oracle.Table(oracle.ICEBERG, w, 15, 32, 16, log2_slots1=12, B1=16, s1=16, seed=3)
    domain = np.arange(1 << w, dtype=np.uint64)
    assert (t.insert(_rng(4).permutation(domain)) == oracle.PUT).all()
    img0 = t.export(0).view(np.uint16).reshape(1 << w, 32)
    assert (img0[:, 0] == 0x8000).all() and (img0[:, 1:] == 0).all()
    assert (t.export(1) == 0).all()
    assert (t.insert(domain) == oracle.FOUND).all() and (t.find(domain) == 1).all()
    c = oracle.Table(oracle.CUCKOO, w, 15, 32, 32, seed=4)
    assert (c.insert(_rng(5).permutation(domain)) == oracle.PUT).all()
    img = c.export(0).view(np.uint32).reshape(1 << w, 32)
    assert (img[:, 0] == 0x80000000).all() and (img[:, 1:] == 0).all()
    assert (c.find(domain) == 1).all()


# ---------------------------------------------------------------------------
# line counts (the per-operation bucket reads used for the roofline)
# ---------------------------------------------------------------------------

def test_lines_per_op_closed_forms():
    # empty table: every find reads exactly one bucket; 32 x 32-bit = 128 B = 1 line
    c = oracle.Table(oracle.CUCKOO, 32, 14, 32, 32)
    _, ln = c.find(np.arange(1000, dtype=np.uint64), lines=True)
    assert (ln == 1).all()
    # non-compact 32 x 64-bit bucket = 256 B = 2 lines
    u = oracle.Table(oracle.CUCKOO, 32, 14, 32, 64, compact=False)
    _, ln = u.find(np.arange(1000, dtype=np.uint64), lines=True)
    assert (ln == 2).all()
    # iceberg with every primary bucket full: a miss reads the primary and both secondaries
    t = oracle.Table(oracle.ICEBERG, 20, 6, 8, 32, log2_slots1=6, B1=4, s1=32, seed=1)
    t.insert(np.arange(1 << 20, dtype=np.uint64)[:2000])
    occ0 = t.export(0).view(np.uint32)
    assert (occ0 != 0).all()
    probe = np.arange(1 << 19, (1 << 19) + 100, dtype=np.uint64)
    f, ln = t.find(probe, lines=True)
    assert (ln[f == 0] == 3).all()


# ---------------------------------------------------------------------------
# the checker rejects planted mistakes
# ---------------------------------------------------------------------------

def _ice_table():
    t = oracle.Table(oracle.ICEBERG, 20, 10, 8, 32, log2_slots1=8, B1=4, s1=32, seed=5)
    keys = _rng(12).choice(1 << 20, size=1100, replace=False).astype(np.uint64)
    t.insert(keys)
    return t


def _slots(img):
    return img.view(np.uint32).copy()


def test_checker_accepts_oracle_tables():
    ok, msg, _ = _ice_table().check()
    assert ok, msg


def test_checker_rejects_duplicate():
    t = _ice_table()
    s0, s1 = _slots(t.export(0)), _slots(t.export(1))
    b = int(np.nonzero((s0.reshape(-1, 8) != 0).sum(1) == 3)[0][0])  # bucket with 3 keys
    s0[b * 8 + 3] = s0[b * 8 + 0]  # same key twice in one bucket
    ok, msg, _ = oracle.check_images(t.cfg, s0.view(np.uint8), s1.view(np.uint8))
    assert not ok


def test_checker_rejects_hole():
    t = _ice_table()
    s0, s1 = _slots(t.export(0)), _slots(t.export(1))
    b = int(np.nonzero((s0.reshape(-1, 8) != 0).sum(1) >= 3)[0][0])
    s0[b * 8 + 1] = 0
    ok, msg, _ = oracle.check_images(t.cfg, s0.view(np.uint8), s1.view(np.uint8))
    assert not ok and "after an empty" in msg


def test_checker_rejects_secondary_key_with_room_in_primary():
    t = _ice_table()
    s0, s1 = _slots(t.export(0)), _slots(t.export(1))
    full = np.nonzero((s0.reshape(-1, 8) != 0).all(1))[0]
    # free the last slot of every full primary bucket: keys in the secondary
    # level now violate the order property
    for b in full:
        s0[b * 8 + 7] = 0
    ok, msg, _ = oracle.check_images(t.cfg, s0.view(np.uint8), s1.view(np.uint8))
    assert not ok and "order property" in msg


def test_checker_rejects_wrong_tag():
    t = _ice_table()
    s0, s1 = _slots(t.export(0)), _slots(t.export(1))
    i = int(np.nonzero(s1)[0][0])
    pbits = 20 - (8 - 2)
    s1[i] ^= np.uint32(1 << pbits)  # flip the secondary index tag
    ok, msg, _ = oracle.check_images(t.cfg, s0.view(np.uint8), s1.view(np.uint8))
    assert not ok


def test_checker_rejects_cuckoo_early_exit_violation():
    t = oracle.Table(oracle.CUCKOO, 20, 10, 8, 32, seed=7)
    keys = _rng(13).choice(1 << 20, size=600, replace=False).astype(np.uint64)
    t.insert(keys)
    s0 = _slots(t.export(0))
    ok, _, _ = oracle.check_images(t.cfg, s0.view(np.uint8))
    assert ok
    # move a hash-1 key's primary bucket below full by clearing its last slot
    pbits = 20 - 7
    tag1 = np.nonzero((s0 >> np.uint32(pbits)) & np.uint32(1))[0]
    assert tag1.size > 0
    slot = int(tag1[0])
    b = slot // 8
    r = int(s0[slot]) & ((1 << pbits) - 1)
    key = int(oracle.perm(20, t.cfg.seed, 1, np.array([(b << pbits) | r], np.uint64), inverse=True)[0])
    a0 = t.bucket_of(0, 0, key)
    s0[a0 * 8 + 7] = 0
    ok, msg, _ = oracle.check_images(t.cfg, s0.view(np.uint8))
    assert not ok


def test_checker_accepts_cuckoo_bucket_with_holes():
    """Alg. 4 claims some empty slot, not necessarily the first, so a cuckoo
    bucket may have an empty slot before a filled one; the checker accepts
    that (and the key set is unchanged), while the same hole in an iceberg
    bucket is still rejected (test_checker_rejects_hole)."""
    t = oracle.Table(oracle.CUCKOO, 20, 10, 8, 32, seed=7)
    keys = _rng(13).choice(1 << 20, size=600, replace=False).astype(np.uint64)
    t.insert(keys)
    s0 = _slots(t.export(0))
    ok, msg, want = oracle.check_images(t.cfg, s0.view(np.uint8))
    assert ok, msg
    rows = s0.reshape(-1, 8)
    filled = (rows != 0).sum(1)
    b = int(np.nonzero((filled >= 2) & (filled < 8))[0][0])
    rows[b, 7], rows[b, 0] = rows[b, 0], 0  # slot 0 moves to the last (empty) slot
    ok, msg, got = oracle.check_images(t.cfg, s0.view(np.uint8))
    assert ok, msg
    assert np.array_equal(np.sort(got), np.sort(want))


def test_insert_outcome_checker_rejects_double_put():
    keys = np.array([5, 5, 6], np.uint64)
    assert sets.check_insert_outcomes(np.zeros(0, np.uint64), keys, np.array([1, 2, 1], np.uint8))[0]
    assert not sets.check_insert_outcomes(np.zeros(0, np.uint64), keys, np.array([1, 1, 1], np.uint8))[0]
    assert not sets.check_insert_outcomes(np.array([6], np.uint64), keys, np.array([1, 2, 1], np.uint8))[0]
