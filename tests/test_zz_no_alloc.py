"""The allocation-free sorted find-or-put (cpht_sorted_fop_noalloc) against
the sorted find-or-put that takes a caller workspace (cpht_sorted_fop), and
both against the oracle, through the C-ABI.

Two tables with the same configuration and seed receive the same batches:
one through each entry point.  Below the failure load every answer is unique
(the stable sort makes the first occurrence of a new key the PUT), so the two
answer arrays must be identical element by element and equal to the oracle's
sorted find-or-put; the decoded key sets must equal the oracle's.  Two calls
in a row, the first at the maximum batch (2^20 keys, the scratch array's
limit), the second smaller, so the second call runs over what the first left
in the shared scratch.
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

MAX_KEYS = 1 << 20


def _cuckoo(w, log2_slots, seed):
    return cpht.Table(scheme=cpht.CUCKOO, key_bits=w, log2_slots0=log2_slots, bucket0=32, slot_bits0=32,
                      n_hash=2, max_chain=256, seed=seed)


@pytest.mark.parametrize("w,log2_slots", [(37, 21), (32, 21)])
def test_noalloc_matches_workspace_call_and_oracle(gpu, w, log2_slots):
    seed = 0xA110C + w
    ta, tb = _cuckoo(w, log2_slots, seed), _cuckoo(w, log2_slots, seed)
    o = oracle_table(ta)
    pool = synth.distinct_keys(w, 0x5EED + w, 0, int(0.7 * (1 << log2_slots)))
    pool_h = host_u64(pool)
    pre = to_dev(pool[: pool.numel() // 5], w, gpu)
    assert (ta.bulk_build(pre) == cpht.PUT).all() and (tb.bulk_build(pre) == cpht.PUT).all()
    assert (o.insert(host_u64(pool[: pool.numel() // 5])) == oracle.PUT).all()
    rng = np.random.default_rng(w)
    for call, (n, hi) in enumerate(((MAX_KEYS, (pool_h.size * 3) // 5), (3 * 4096 + 17, pool_h.size))):
        keys_h = pool_h[rng.integers(0, hi, size=n)]  # repeats, stored and new keys
        dk = to_dev(torch.from_numpy(keys_h.astype(np.int64)), w, gpu)
        got_a = ta.sorted_fop(dk).cpu().numpy()
        out_b = torch.full((n,), 0xEE, dtype=torch.uint8, device=gpu)
        got_b = tb.sorted_fop_noalloc(dk, out_b).cpu().numpy()
        want = cuckoo_find_or_put(o, keys_h)
        assert (want != oracle.FULL).all()
        bad = np.nonzero(got_b != got_a)[0]
        assert bad.size == 0, f"call {call}: {bad.size} answers differ from the workspace call, first at {bad[:5]}"
        bad = np.nonzero(got_b != want)[0]
        assert bad.size == 0, f"call {call}: {bad.size} answers differ from the oracle, first at {bad[:5]}"
        dec_o = o.check()
        assert dec_o[0], dec_o[1]
        want_set = np.sort(dec_o[2])
        assert np.array_equal(np.sort(check_table(tb)), want_set)
        assert np.array_equal(np.sort(check_table(ta)), want_set)
    q = to_dev(torch.from_numpy(pool_h.astype(np.int64)), w, gpu)
    assert np.array_equal(tb.find(q).cpu().numpy(), o.find(pool_h))


def test_noalloc_limits(gpu):
    t = _cuckoo(37, 16, 3)
    out = torch.empty(MAX_KEYS + 1, dtype=torch.uint8, device=gpu)
    too_many = torch.zeros(MAX_KEYS + 1, dtype=torch.int64, device=gpu)
    with pytest.raises(cpht.CphtError) as e:
        t.sorted_fop_noalloc(too_many, out)
    assert e.value.code == 1  # CPHT_E_ARG
    # an empty batch is accepted and writes nothing
    t.sorted_fop_noalloc(too_many[:0], out[:0])
    ice = cpht.Table(scheme=cpht.ICEBERG, key_bits=20, log2_slots0=14, log2_slots1=11, bucket0=32, bucket1=16,
                     slot_bits0=16, slot_bits1=32, seed=4)
    with pytest.raises(cpht.CphtError) as e:
        ice.sorted_fop_noalloc(torch.zeros(8, dtype=torch.int32, device=gpu), out[:8])
    assert e.value.code == 7  # CPHT_E_STATE


def test_noalloc_in_a_captured_graph(gpu):
    """The call the entry point is for: captured in a HIP graph (nothing to
    allocate during capture) and replayed three times.  Between the replays
    an eager allocation-free call on another table overwrites the shared
    scratch, so each replay must start from whatever the last call left
    there; every replay gives the eager call's answers and key set."""
    from tests.test_gpu_graphs import _capture

    w = 37
    t = _cuckoo(w, 18, 0x6D)
    other = _cuckoo(w, 18, 0x6E)
    n_before = 1 << 16
    t.bulk_build(synth.distinct_keys(w, 0x6D, 0, n_before, device=gpu))
    torch.cuda.synchronize()
    img = t.export(0)
    keys, _ = synth.find_or_put_batch(w, 0x6D, n_before, 1 << 16, 1 << 18, 5, device=gpu)
    assert keys.numel() <= MAX_KEYS
    out = torch.empty(keys.numel(), dtype=torch.uint8, device=gpu)
    other_out = torch.empty(5000, dtype=torch.uint8, device=gpu)
    t.sorted_fop_noalloc(keys, out)  # eager: the answers and key set every replay must give
    torch.cuda.synchronize()
    want = out.clone()
    want_set = check_table(t)
    g = _capture(lambda s: t.sorted_fop_noalloc(keys, out, stream=s))
    for rep in range(3):
        other.sorted_fop_noalloc(keys[rep * 5000:(rep + 1) * 5000], other_out)
        t.import_image(0, img)
        out.fill_(0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert int((out != want).sum()) == 0, rep
        assert np.array_equal(check_table(t), want_set), rep
