"""The third iceberg level's list protocol under every interleaving
(explicit-state model checking with stale reads; see oracle/interleave_l3.py).

The kernel reserves a list head or slab link by CAS before taking a slab
from the pool; the checker confirms that this keeps every list a chain of
distinct slabs filled in order, with one copy and one PUT per key, FULL only
once the pool is used up, no slab taken outside the list, and termination --
and that plausible mistakes are caught.
"""
from __future__ import annotations

import pytest

from oracle.interleave_l3 import L3Scenario, check


@pytest.mark.parametrize("keys,slots,pool", [
    ((1, 2, 3), 1, 3),       # every insert needs its own slab: three racing links
    ((1, 1, 2), 2, 2),       # a repeated key racing a fresh one across a full slab
    ((1, 2, 3), 2, 1),       # the pool runs out: FULL
    ((1, 1, 1), 1, 2),       # three inserts of one key
    ((1, 2), 1, 1),          # one slab for two keys: one of them FULL
    ((1, 2, 3, 4), 1, 3),    # four racing links, the last one finds the pool used up
    ((1, 1, 2, 2), 2, 2),    # two repeated keys over two slabs
])
def test_link_protocol_all_interleavings(keys, slots, pool):
    ok, errors, states = check(L3Scenario(slots=slots, pool=pool, keys=keys))
    assert ok, errors
    assert states > 10


def test_link_protocol_without_stale_reads():
    ok, errors, _ = check(L3Scenario(slots=2, pool=3, keys=(1, 2, 3), stale_reads=False))
    assert ok, errors


def test_allocating_before_reserving_strands_slabs():
    """The first design: every lane that finds the tail full takes a slab and
    then races to link it; the losers' slabs are never linked."""
    ok, errors, _ = check(L3Scenario(slots=1, pool=3, keys=(1, 2, 3), bug_alloc_first=True))
    assert not ok and any("on no list" in e or "FULL" in e for e in errors), errors


def test_claiming_the_last_empty_slot_is_caught():
    ok, errors, _ = check(L3Scenario(slots=2, pool=2, keys=(1, 1), bug_last_empty=True))
    assert not ok, errors


def test_skipping_the_found_check_is_caught():
    ok, errors, _ = check(L3Scenario(slots=2, pool=2, keys=(1, 1), bug_skip_found=True))
    assert not ok, errors
