"""Every interleaving of concurrent compact cuckoo puts (Sec. 4.4, Alg. 4) at
the kernel's step granularity, on tiny tables: per-slot snapshot reads that
may be stale, CAS claims with known-occupied masks, eviction swaps whose
evicted word is decoded under its own hash index, victims in every row.  No
key is lost or stored twice, the early-exit invariant of the lookup holds,
every put succeeds where there is room (also when a claim takes any free
slot of the snapshot, not the first), and the planted mistakes are caught:
decoding the evicted word with the carried key's hash index, and forgetting
lost claims (which lets a stale line be claimed again and again)."""
import pytest

from oracle.interleave_cuckoo import CuckooScenario, check

# keys: name -> ((a_0, r_0), (a_1, r_1))


def contention(**kw):
    """Three puts on one 2-slot bucket whose second buckets are empty."""
    keys = {"k1": ((0, 1), (1, 1)), "k2": ((0, 2), (1, 2)), "k3": ((0, 3), (1, 3))}
    return CuckooScenario(B=2, n_buckets=2, H=2, C=8, keys=keys, ops=["k1", "k2", "k3"],
                          expect_no_full=True, **kw)


def evictions(**kw):
    """Two puts into bucket 0, which holds two keys stored under hash 1 (so
    their first buckets, bucket 2, are full); evicting them pushes keys out of
    bucket 2 into the empty bucket 3."""
    keys = {
        "p1": ((2, 5), (0, 5)), "p2": ((2, 6), (0, 6)),   # stored in bucket 0 under hash 1
        "p3": ((2, 7), (3, 7)), "p4": ((2, 8), (3, 8)),   # stored in bucket 2 under hash 0
        "k1": ((0, 1), (1, 1)), "k2": ((0, 2), (1, 2)),   # put concurrently
    }
    prefill = {0: "p1", 1: "p2", 4: "p3", 5: "p4"}
    tags = {0: 1, 1: 1, 4: 0, 5: 0}
    return CuckooScenario(B=2, n_buckets=4, H=2, C=10, keys=keys, ops=["k1", "k2"], prefill=prefill,
                          prefill_tags=tags, expect_no_full=True, **kw)


def over_capacity(**kw):
    """Three puts, two one-slot buckets: at least one FULL, one dropped key each."""
    keys = {"k1": ((0, 1), (1, 1)), "k2": ((0, 2), (1, 2)), "k3": ((0, 3), (1, 3))}
    return CuckooScenario(B=1, n_buckets=2, H=2, C=4, keys=keys, ops=["k1", "k2", "k3"], **kw)


def stale_prefill(**kw):
    """One put into a bucket whose first slot is taken (a stale read may show it EMPTY)."""
    keys = {"p": ((0, 9), (1, 9)), "k": ((0, 1), (1, 1))}
    return CuckooScenario(B=2, n_buckets=2, H=2, C=6, keys=keys, ops=["k"], prefill={0: "p"},
                          expect_no_full=True, **kw)


@pytest.mark.parametrize("make", [contention, evictions, over_capacity, stale_prefill])
def test_cuckoo_put_interleavings_are_correct(make):
    ok, errors, states, terminal = check(make())
    assert ok, errors
    assert terminal > 0


@pytest.mark.parametrize("make", [contention, evictions, over_capacity, stale_prefill])
def test_cuckoo_put_claiming_any_free_slot_is_correct(make):
    """Claims spread over the snapshot's free slots (every choice explored):
    holes may remain in a bucket, and still no key is lost or stored twice,
    the lookup's early-exit invariant holds and no put fails with room."""
    ok, errors, states, terminal = check(make(claim_any=True))
    assert ok, errors
    assert terminal > 0


def test_spread_claims_leave_holes_in_some_interleaving():
    """With claims spread over free slots, some terminal table has an EMPTY
    slot before an occupied one in a bucket (so the non-empty slots of a
    cuckoo bucket need not form a prefix), which the lookup tolerates."""
    from oracle.interleave_cuckoo import CuckooChecker

    keys = {"k1": ((0, 1), (1, 1))}
    c = CuckooChecker(CuckooScenario(B=2, n_buckets=2, H=2, C=4, keys=keys, ops=["k1"], claim_any=True,
                                     expect_no_full=True))
    terminals = []
    orig = c._check_terminal
    c._check_terminal = lambda st: (terminals.append(st[0]), orig(st))
    assert c.run() and not c.errors
    assert any(tb[0] is None and tb[1] is not None for tb in terminals)


def test_evictions_really_happen_in_the_scenarios():
    """The eviction scenario reaches terminal states with keys under hash 1
    moved (so the decode path is exercised)."""
    ok, errors, states, terminal = check(evictions())
    assert ok and states > 1000


@pytest.mark.parametrize("make", [evictions])
def test_planted_decode_with_carried_index_is_caught(make):
    ok, errors, _, _ = check(make(bug_decode_with_carried_j=True))
    assert not ok
    assert "lost or made up" in errors[0] or "no key's form" in errors[0] or "stored twice" in errors[0]


@pytest.mark.parametrize("make", [stale_prefill, contention])
def test_planted_forgotten_claims_are_caught(make):
    ok, errors, _, _ = check(make(bug_no_known=True))
    assert not ok
    assert "FULL with room" in errors[0]


def test_without_stale_reads_forgetting_claims_is_harmless():
    """Only stale reads make the known-occupied mask necessary (a fresh
    re-read shows the lost slot taken)."""
    ok, errors, _, _ = check(stale_prefill(bug_no_known=True, stale_reads=False))
    assert ok, errors
