"""Every interleaving of small concurrent find-or-put sets, at the kernel's
step granularity with stale (non-coherent) reads, satisfies Theorem 1 of
Appendix A; planted mistakes in the algorithm are caught."""
import pytest

from oracle.interleave import Scenario, check

A, B, C, X, Y = "A", "B", "C", "X", "Y"


def _full_primary(B0, bucket=0):
    # fill primary bucket `bucket` with keys that belong there (stored forms of other keys)
    return {bucket * B0 + y: (f"P{y}", 0) for y in range(B0)}


SCENARIOS = {
    "dup_and_other_empty_table": Scenario(B0=2, B1=1, n_primary=1, n_secondary=2,
                                          ops=[(A, 0, 0, 1), (A, 0, 0, 1), (B, 0, 0, 1)]),
    "overflow_to_level2": Scenario(B0=2, B1=2, n_primary=1, n_secondary=2,
                                   ops=[(A, 0, 0, 1), (A, 0, 0, 1), (B, 0, 1, 0)], prefill=_full_primary(2)),
    "level2_full": Scenario(B0=1, B1=1, n_primary=1, n_secondary=2,
                            ops=[(A, 0, 0, 1), (B, 0, 0, 1), (C, 0, 1, 0)], prefill=_full_primary(1)),
    "aliased_secondaries": Scenario(B0=1, B1=2, n_primary=1, n_secondary=1,
                                    ops=[(A, 0, 0, 0), (A, 0, 0, 0), (B, 0, 0, 0)], prefill=_full_primary(1)),
    "half_word_claims": Scenario(B0=2, B1=1, n_primary=1, n_secondary=2, half_words=True,
                                 ops=[(A, 0, 0, 1), (A, 0, 0, 1), (B, 0, 0, 1)]),
    "half_word_partly_full": Scenario(B0=4, B1=1, n_primary=1, n_secondary=2, half_words=True,
                                      ops=[(A, 0, 0, 1), (B, 0, 1, 0), (A, 0, 0, 1)],
                                      prefill={0: ("P0", 0)}),
    "two_levels_mixed": Scenario(B0=2, B1=1, n_primary=2, n_secondary=2,
                                 ops=[(A, 0, 0, 1), (B, 0, 1, 0), (C, 1, 0, 1)], prefill={0: ("P0", 0)}),
}


@pytest.mark.parametrize("name", sorted(SCENARIOS))
def test_theorem1_holds_in_every_interleaving(name):
    ok, errors, states, terminal = check(SCENARIOS[name])
    assert ok, errors
    assert terminal > 1  # concurrency produced more than one outcome path


def test_coherent_reads_subset():
    sc = SCENARIOS["dup_and_other_empty_table"]
    sc2 = Scenario(**{**sc.__dict__, "stale_reads": False})
    ok, errors, states_c, _ = check(sc2)
    ok2, _, states_s, _ = check(sc)
    assert ok and ok2 and states_s > states_c


def test_forgetting_failed_claims_livelocks_under_stale_reads():
    sc = Scenario(B0=2, B1=1, n_primary=1, n_secondary=2, ops=[(A, 0, 0, 1), (B, 0, 0, 1)], bug_no_known=True)
    ok, errors, _, _ = check(sc)
    assert not ok and "non-termination" in errors[0]


def test_claiming_the_last_empty_slot_breaks_the_order_property():
    sc = Scenario(B0=2, B1=1, n_primary=1, n_secondary=2, ops=[(A, 0, 0, 1)], bug_last_empty=True)
    ok, errors, _, _ = check(sc)
    assert not ok and "order property" in errors[0]


def test_skipping_the_secondary_found_check_duplicates_keys():
    sc = Scenario(B0=1, B1=2, n_primary=1, n_secondary=2, ops=[(A, 0, 0, 1), (A, 0, 0, 1)],
                  prefill=_full_primary(1), bug_skip_found2=True)
    ok, errors, _, _ = check(sc)
    assert not ok and ("twice" in errors[0] or "PUT" in errors[0])


def test_tie_break_is_a_convention_not_a_safety_condition():
    """Sending ties to bucket 1 is another well-order; Theorem 1 still holds
    under it.  Figure 5 pins the paper's choice (ties to bucket 2)."""
    sc = Scenario(B0=1, B1=2, n_primary=1, n_secondary=2, ops=[(A, 0, 0, 1), (B, 0, 1, 0), (A, 0, 0, 1)],
                  prefill=_full_primary(1), bug_tie_to_1=True)
    ok, errors, _, _ = check(sc)
    assert ok, errors
