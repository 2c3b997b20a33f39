"""GPU parity of the sorted find-or-put on the cuckoo table (the baseline of
the paper's find-or-put experiment, Sec. 5) against the oracle.

The answers are unique below the failure load (the first occurrence of a new
key is PUT because the sort is stable, every other operation is FOUND), so
they are compared element by element; the decoded key set of the GPU table
must equal the oracle's.  Batch sizes straddle the sort's 4096-key tiles with
ragged tails; key widths cover 32-bit words (four 8-bit digit rounds) and
64-bit words up to the full 64 bits (eight rounds).
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import paper_2406_09255_amd as cpht
import synth
from oracle.fop import cuckoo_find_or_put
from tests.helpers import check_table, host_u64, oracle_table, to_dev

pytestmark = pytest.mark.gpu

KEY_SEED = 0x50F7


def cuckoo(w, log2_slots, B, S=32, compact=1, seed=1):
    return cpht.Table(scheme=cpht.CUCKOO, key_bits=w, log2_slots0=log2_slots, bucket0=B, slot_bits0=S,
                      n_hash=2, max_chain=256, compact=compact, seed=seed)


def _oracle_set(o: oracle.Table) -> list[int]:
    ok, msg, dec = o.check()
    assert ok, msg
    return sorted(int(x) for x in dec)


def _gpu_set(t: cpht.Table) -> list[int]:
    return sorted(int(x) for x in check_table(t))


@pytest.mark.parametrize("w,log2_slots,B,S,compact,n", [
    (32, 14, 32, 32, 1, 3 * 4096 + 17),
    (37, 16, 32, 32, 1, 4096),
    (37, 15, 16, 64, 0, 20001),
    (64, 14, 16, 64, 1, 9000),
    (20, 12, 8, 32, 1, 4095),
])
def test_sorted_fop_matches_oracle(gpu, w, log2_slots, B, S, compact, n):
    t = cuckoo(w, log2_slots, B, S, compact, seed=0xF0 + w)
    o = oracle_table(t)
    slots = 1 << log2_slots
    pool = synth.distinct_keys(w, KEY_SEED + w, 0, int(0.75 * slots))
    pool_h = host_u64(pool)
    # stored before: the first fifth of the pool, by the static build
    pre = pool[: pool.numel() // 5]
    assert (t.bulk_build(to_dev(pre, w, gpu)) == cpht.PUT).all()
    assert (o.insert(host_u64(pre)) == oracle.PUT).all()
    rng = np.random.default_rng(w * 1000 + n)
    ws = torch.empty(t.sorted_fop_workspace(n), dtype=torch.uint8, device=gpu)
    for batch in range(3):
        # draws with repeats from a growing prefix of the pool (stored and new keys)
        hi = min(pool_h.size, pool_h.size // 5 + (batch + 1) * pool_h.size // 4)
        idx = rng.integers(0, hi, size=n)
        keys_h = pool_h[idx]
        dk = to_dev(torch.from_numpy(keys_h.astype(np.int64)), w, gpu)
        got = t.sorted_fop(dk, workspace=ws).cpu().numpy()
        want = cuckoo_find_or_put(o, keys_h)
        assert (want != oracle.FULL).all()
        bad = np.nonzero(got != want)[0]
        assert bad.size == 0, f"batch {batch}: {bad.size} answers differ, first at {bad[:5]}: " \
                              f"got {got[bad[:5]]} want {want[bad[:5]]}"
        assert _gpu_set(t) == _oracle_set(o)
    # lookups agree afterwards
    q = to_dev(torch.from_numpy(pool_h.astype(np.int64)), w, gpu)
    assert np.array_equal(t.find(q).cpu().numpy(), o.find(pool_h))


def test_sorted_fop_first_occurrence_is_put_across_tiles(gpu):
    """Few distinct keys spread over many tiles: the stable sort must keep
    the earliest input position of each key at the head of its run."""
    w = 37
    t = cuckoo(w, 16, 32)
    distinct = synth.distinct_keys(w, KEY_SEED, 0, 300)
    rng = np.random.default_rng(9)
    n = 11 * 4096 + 123
    idx = rng.integers(0, 300, size=n)
    keys_h = host_u64(distinct)[idx]
    got = t.sorted_fop(to_dev(torch.from_numpy(keys_h.astype(np.int64)), w, gpu)).cpu().numpy()
    _, first = np.unique(keys_h, return_index=True)
    want = np.full(n, cpht.FOUND, np.uint8)
    want[first] = cpht.PUT
    assert np.array_equal(got, want)


def test_sorted_fop_single_key_and_all_duplicates(gpu):
    w = 32
    t = cuckoo(w, 12, 32)
    one = torch.tensor([12345], dtype=torch.int32, device=gpu)
    assert t.sorted_fop(one).tolist() == [cpht.PUT]
    assert t.sorted_fop(one).tolist() == [cpht.FOUND]
    same = torch.full((3 * 4096 + 5,), 777, dtype=torch.int32, device=gpu)
    out = t.sorted_fop(same).cpu().numpy()
    assert out[0] == cpht.PUT and (out[1:] == cpht.FOUND).all()
    assert t.count()[0] == 2
    empty = torch.empty(0, dtype=torch.int32, device=gpu)
    assert t.sorted_fop(empty).numel() == 0
    assert t.count()[0] == 2


def test_sorted_fop_rejects_iceberg_and_small_workspace(gpu):
    ice = cpht.Table(scheme=cpht.ICEBERG, key_bits=32, log2_slots0=12, log2_slots1=9, bucket0=32, bucket1=16,
                     slot_bits0=32, slot_bits1=32)
    k = torch.arange(10, dtype=torch.int32, device=gpu)
    with pytest.raises(cpht.CphtError) as e:
        ice.sorted_fop(k)
    assert e.value.code == 7  # CPHT_E_STATE
    t = cuckoo(32, 12, 32)
    need = t.sorted_fop_workspace(10)
    small = torch.empty(need, dtype=torch.uint8, device=gpu)
    out = torch.zeros(10, dtype=torch.uint8, device=gpu)
    L = cpht.lib()
    # through the C-ABI: too few bytes, then a misaligned workspace
    assert L.cpht_sorted_fop(t._h, k.data_ptr(), 10, out.data_ptr(), small.data_ptr(), need - 1, None) == 1
    assert L.cpht_sorted_fop(t._h, k.data_ptr(), 10, out.data_ptr(), small.data_ptr() + 8, need - 8, None) == 1
    torch.cuda.synchronize()
    assert t.count()[0] == 0 and int(out.sum().item()) == 0
    with pytest.raises(ValueError):
        t.sorted_fop(k, workspace=small[: need - 256])


def test_sorted_fop_past_failure_accounting(gpu):
    """Over capacity: answers are interleaving-dependent, but every FULL
    drops exactly one carried key, keys stored before stay FOUND, and the
    table passes the checker."""
    w = 32
    t = cuckoo(w, 10, 8)
    o = oracle_table(t)
    pre = synth.distinct_keys(w, KEY_SEED + 5, 0, 700)
    assert (t.bulk_build(to_dev(pre, w, gpu)) == cpht.PUT).all()
    pool = host_u64(synth.distinct_keys(w, KEY_SEED + 5, 0, 1400))
    rng = np.random.default_rng(4)
    keys_h = pool[rng.integers(0, pool.size, size=5000)]
    got = t.sorted_fop(to_dev(torch.from_numpy(keys_h.astype(np.int64)), w, gpu)).cpu().numpy()
    dec = np.array(_gpu_set(t), dtype=np.uint64)
    offered = np.union1d(host_u64(pre), keys_h)
    _, first = np.unique(keys_h, return_index=True)
    n_full = int((got[first] == cpht.FULL).sum())
    assert n_full > 0
    assert np.isin(dec, offered).all()
    assert dec.size == offered.size - n_full
    assert (got[np.isin(keys_h, host_u64(pre))] == cpht.FOUND).all()
    later = np.ones(keys_h.size, bool)
    later[first] = False
    assert not (got[later] == cpht.PUT).any()
    # the sequential oracle on the same batch, for the record: same accounting
    o.insert(host_u64(pre))
    want = cuckoo_find_or_put(o, keys_h)
    assert int((want[first] == oracle.FULL).sum()) > 0
