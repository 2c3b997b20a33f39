"""The autotuner's host logic: which compiled variants are candidates at a
shape, and how a winner is picked from measured times (no device needed).
Its measurements run in tests/test_gpu_tune.py."""
from __future__ import annotations

import pytest

import paper_2406_09255_amd as cpht
from paper_2406_09255_amd import tune


@pytest.mark.parametrize("scheme,w,e", [(cpht.ICEBERG, 32, 10), (cpht.ICEBERG, 32, 20), (cpht.ICEBERG, 37, 27),
                                        (cpht.CUCKOO, 37, 27), (cpht.CUCKOO, 32, 12)])
def test_candidates_are_feasible_and_line_sized(scheme, w, e):
    cands = tune.candidates(scheme, w, e)
    assert cands, "every shape here has feasible variants"
    seen = set()
    for c in cands:
        assert cpht.check_config(c) is not None
        assert c.bucket0 * c.slot_bits0 // 8 <= 128  # a primary bucket fits one cache line
        if scheme == cpht.ICEBERG:
            assert c.slot_bits1 >= c.slot_bits0 and c.log2_slots1 == e - 3
        seen.add((c.bucket0, c.slot_bits0, c.slot_bits1, c.subtile))
    assert len(seen) == len(cands)  # one per compiled variant
    # every compiled variant that fits is offered
    fits = 0
    for v in cpht.variants(scheme):
        if v["key64"] != int(w > 32) or v["bucket0"] * v["slot_bits0"] // 8 > 128:
            continue
        if scheme == cpht.ICEBERG and v["slot_bits1"] < v["slot_bits0"]:
            continue
        c = cpht.default_config(scheme)
        c.key_bits, c.log2_slots0 = w, e
        c.bucket0, c.slot_bits0, c.subtile = v["bucket0"], v["slot_bits0"], v["subtile"]
        if scheme == cpht.ICEBERG:
            c.log2_slots1, c.bucket1, c.slot_bits1 = e - 3, v["bucket1"], v["slot_bits1"]
        fits += cpht.check_config(c) is not None
    assert fits == len(cands)


def test_wide_keys_drop_narrow_slots():
    """37-bit keys at 2^27 slots: 64-slot buckets leave 21 address bits and a
    16-bit remainder, which with the occupancy bit overflows a 16-bit slot;
    32-slot buckets leave 15 remainder bits, which fit."""
    cands = tune.candidates(cpht.ICEBERG, 37, 27)
    assert not any(c.slot_bits0 == 16 and c.bucket0 == 64 for c in cands)
    assert any(c.slot_bits0 == 16 and c.bucket0 == 32 for c in cands)


def test_pick_drops_failures_and_prefers_memory_within_tie():
    # (ms or None, bits per slot, preferred)
    entries = [(10.0, 64.0, False), (None, 16.0, False), (10.2, 32.0, False), (12.0, 17.8, False)]
    assert tune.pick(entries, tie=0.03) == 2  # 10.2 is within 3 % of 10.0 and uses half the memory
    assert tune.pick(entries, tie=0.01) == 0  # not within 1 %: the fastest wins
    assert tune.pick(entries, tie=0.25) == 3  # within 25 %: the smallest footprint


def test_pick_breaks_memory_ties_by_preference_then_time():
    entries = [(10.0, 32.0, False), (10.1, 32.0, True), (10.05, 32.0, False)]
    assert tune.pick(entries) == 1
    entries = [(10.0, 32.0, False), (10.1, 32.0, False), (10.05, 32.0, False)]
    assert tune.pick(entries) == 0


def test_pick_raises_when_nothing_reaches_the_load():
    with pytest.raises(RuntimeError):
        tune.pick([(None, 32.0, False), (None, 16.0, True)])


@pytest.mark.parametrize("w", [12, 32, 37, 64])
def test_timing_keys_are_distinct_words(w):
    import torch

    gen = torch.Generator().manual_seed(5)
    n = 1 << 12
    k = tune._random_keys(n, w, gen, "cpu")
    assert k.dtype == (torch.int32 if w <= 32 else torch.int64)
    assert torch.unique(k).numel() == n
    if w < 32:
        assert int(k.min()) >= 0 and int(k.max()) < (1 << w)
