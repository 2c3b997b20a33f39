"""Parity at the benchmark's full sizes, in the launch configuration bench.py
times.  Expected answers come from the plain definition, made cheap by how
the inputs are built: keys phi(i < n) are inserted, phi(i >= n) never are, so
every find's answer is fixed by the index it was drawn from; the full
2^27-slot cuckoo table is also run through the oracle's table checker."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import paper_2406_09255_amd as cpht
import synth
from tests.helpers import check_table, oracle_cfg

pytestmark = pytest.mark.gpu

SEED = 0xF0F0


def _count(mask: torch.Tensor) -> int:
    """Number of set entries (assertions compare plain ints: a failure report
    never formats a tensor of this size)."""
    return int(mask.sum().item())


def _diff(a: torch.Tensor, b: torch.Tensor) -> int:
    return _count(a != b)


def _queries(w, n, nq, seed, dev):
    """nq queries, half hits phi(i < n), half misses phi(i >= n), with the truth."""
    hit = synth.uniform_below(seed, nq, 2, dev) == 1
    hidx = synth.uniform_below(seed + 1, nq, 1 << 30, dev) * n >> 30
    midx = n + torch.arange(nq, device=dev)
    idx = torch.where(hit, hidx, midx)
    return synth.feistel(w, SEED, idx), hit.to(torch.uint8)


def test_c2_compact_cuckoo_full_size(gpu):
    """2^27 slots, 32 x 32-bit buckets, 37-bit keys, load 0.9, 2^26 finds."""
    w, L = 37, 27
    n = int(0.9 * (1 << L))
    t = cpht.Table(scheme=cpht.CUCKOO, key_bits=w, log2_slots0=L, bucket0=32, slot_bits0=32, seed=77)
    keys = synth.distinct_keys(w, SEED, 0, n, device=gpu)
    out = t.bulk_build(keys)
    n_put = _count(out == cpht.PUT)
    assert n_put == n
    assert t.count() == (n, 1 << L)
    q, truth = _queries(w, n, 1 << 26, 5, gpu)
    bad = _diff(t.find(q), truth)
    assert bad == 0, f"{bad} find answers differ"
    ok, msg, dec = oracle.check_images(oracle_cfg(t), t.export(0))
    assert ok, msg
    assert dec.size == n
    # the decoded set is exactly the inserted set: compare sorted arrays
    want = np.sort(keys.cpu().numpy().astype(np.uint64))
    assert np.array_equal(dec, want)


def test_c2_plain_cuckoo_full_size(gpu):
    w, L = 37, 27
    n = int(0.9 * (1 << L))
    t = cpht.Table(scheme=cpht.CUCKOO, key_bits=w, log2_slots0=L, bucket0=32, slot_bits0=64, compact=0, seed=78)
    keys = synth.distinct_keys(w, SEED, 0, n, device=gpu)
    out = t.bulk_build(keys)
    n_put = _count(out == cpht.PUT)
    assert n_put == n
    q, truth = _queries(w, n, 1 << 26, 6, gpu)
    bad = _diff(t.find(q), truth)
    assert bad == 0, f"{bad} find answers differ"


def test_c3_iceberg_full_size_batches(gpu):
    """2^28 + 2^25 slots, 16/32-bit, 34-bit keys, filled to load 0.85 in
    batches of 2^20 with 30 % duplicate inserts: one PUT per distinct key,
    the count equals the distinct keys, every inserted key is found and
    2^24 never-inserted keys are not."""
    w, L0 = 34, 28
    cap = (1 << L0) + (1 << (L0 - 3))
    t = cpht.Table(scheme=cpht.ICEBERG, key_bits=w, log2_slots0=L0, log2_slots1=L0 - 3, bucket0=32, bucket1=16,
                   slot_bits0=16, slot_bits1=32, seed=79)
    target = int(0.85 * cap)
    batch = 1 << 20
    issued, puts, full, b = 0, 0, 0, 0
    out = torch.empty(batch, dtype=torch.uint8, device=gpu)
    while issued < target:
        keys, nf = synth.insert_stream_with_duplicates(w, SEED, issued, batch, 0.3, 1000 + b, device=gpu)
        t.insert(keys, out)
        puts += int((out == cpht.PUT).sum().item())
        full += int((out == cpht.FULL).sum().item())
        issued += nf
        b += 1
    assert full == 0
    assert puts == issued
    assert t.count()[0] == issued
    for a in range(0, issued, 1 << 26):
        k = synth.distinct_keys(w, SEED, a, min(1 << 26, issued - a), device=gpu)
        missed = _count(t.find(k) != 1)
        assert missed == 0, f"{missed} inserted keys not found"
    miss = synth.distinct_keys(w, SEED, 1 << 33, 1 << 24, device=gpu)
    false_hits = _count(t.find(miss) != 0)
    assert false_hits == 0


def test_c3_iceberg_mixed_stream_full_size(gpu):
    """The dynamic-operation stream the benchmark times, batch for batch:
    2^28 + 2^25 slots (16/32-bit, 34-bit keys), mixed batches of 2^20
    operations (half find-or-puts with 30 % repeats, half finds with 50 %
    hits) from load 0 to 0.9, one launch per batch in order on one stream.
    The truth comes from the index each key was drawn from (keys = phi(index)):
    for every distinct inserted key, exactly one PUT, in the first batch that
    inserts it; a find answers 1 if an earlier batch inserted its key, 0 if no
    batch up to its own did (either way if its own batch does); the count is
    the number of distinct inserted keys, all of which are found afterwards."""
    w, L0 = 34, 28
    cap = (1 << L0) + (1 << (L0 - 3))
    keys, ops, idx, n_fresh = synth.mixed_batches(w, 0xC2C2C2C2 + 3, cap, 0.9, 1 << 20, device=gpu)
    nb, batch = keys.shape
    t = cpht.Table(scheme=cpht.ICEBERG, key_bits=w, log2_slots0=L0, log2_slots1=L0 - 3, bucket0=32, bucket1=16,
                   slot_bits0=16, slot_bits1=32, seed=9)
    out = torch.empty(nb, batch, dtype=torch.uint8, device=gpu)
    for b in range(nb):
        t.mixed(keys[b], ops[b], out[b])
    torch.cuda.synchronize()
    print(f"mixed stream: {nb} batches, {n_fresh} distinct keys inserted", flush=True)
    ins = ops == 1
    # batch of each operation, and the first batch inserting each key index
    bat = torch.arange(nb, device=gpu).repeat_interleave(batch).view(nb, batch)
    ji, bi, oi = idx[ins], bat[ins], out[ins]
    assert int(ji.max().item()) < n_fresh
    first = torch.full((n_fresh,), nb, dtype=torch.int64, device=gpu).scatter_reduce(0, ji, bi, reduce="amin")
    assert _count((oi != cpht.PUT) & (oi != cpht.FOUND)) == 0, "an insert answered neither PUT nor FOUND"
    put = oi == cpht.PUT
    assert _count(put) == n_fresh
    puts_per_key = torch.bincount(ji[put], minlength=n_fresh)
    assert _count(puts_per_key != 1) == 0, "a key was not answered PUT exactly once"
    assert _count(first[ji[put]] != bi[put]) == 0, "a PUT came after the first batch inserting its key"
    del ji, bi, oi, put, puts_per_key
    jf, bf, of = idx[~ins], bat[~ins], out[~ins]
    known = jf < n_fresh  # misses are phi(2^33 + j), never inserted
    fb = torch.where(known, first[jf.clamp(max=n_fresh - 1)], torch.full_like(jf, nb))
    before, same = fb < bf, fb == bf
    assert _count(before & (of != 1)) == 0, "a key inserted by an earlier batch was not found"
    assert _count(~before & ~same & (of != 0)) == 0, "a find answered 1 for a key not inserted yet"
    assert _count(same & (of > 1)) == 0
    del jf, bf, of, fb, before, same, bat
    assert t.count()[0] == n_fresh
    for a in range(0, n_fresh, 1 << 26):
        k = synth.distinct_keys(w, 0xC2C2C2C2 + 3, a, min(1 << 26, n_fresh - a), device=gpu)
        missed = _count(t.find(k) != 1)
        assert missed == 0, f"{missed} inserted keys not found"
    miss = synth.distinct_keys(w, 0xC2C2C2C2 + 3, synth.MISS_BASE, 1 << 24, device=gpu)
    assert _count(t.find(miss) != 0) == 0


def test_c5_table_shape_full_size(gpu):
    """The serving table: 2^32 + 2^29 slots (16/32-bit, 40-bit keys), bulk
    filled to load 0.5 in chunks; count and sampled finds are exact."""
    w, L0 = 40, 32
    cap = (1 << L0) + (1 << (L0 - 3))
    t = cpht.Table(scheme=cpht.ICEBERG, key_bits=w, log2_slots0=L0, log2_slots1=L0 - 3, bucket0=32, bucket1=16,
                   slot_bits0=16, slot_bits1=32, seed=80)
    n = int(0.5 * cap)
    chunk = 1 << 28
    puts = 0
    for a in range(0, n, chunk):
        k = synth.distinct_keys(w, SEED, a, min(chunk, n - a), device=gpu)
        puts += int((t.insert(k) == cpht.PUT).sum().item())
        del k
    assert puts == n and t.count() == (n, cap)
    q, truth = _queries(w, n, 1 << 24, 7, gpu)
    bad = _diff(t.find(q), truth)
    assert bad == 0, f"{bad} find answers differ"


def _fop_truth(idx, n_before, dev):
    """Per-position answers of a find-or-put batch: FOUND for stored keys,
    PUT at the first position of each fresh key, FOUND at its later ones."""
    n_ops = idx.numel()
    pos = torch.arange(n_ops, device=dev)
    first = torch.full((int(idx.max().item()) + 1,), n_ops, dtype=torch.int64, device=dev)
    first.scatter_reduce_(0, idx, pos, reduce="amin")
    put = (idx >= n_before) & (first[idx] == pos)
    return torch.where(put, cpht.PUT, cpht.FOUND).to(torch.uint8)


def test_cuckoo_sorted_fop_full_size(gpu):
    """The find-or-put experiment's cuckoo side at full size: 2^27 slots
    filled to 0.5, then one sorted find-or-put of 2^27 keys (stored and fresh
    keys, with repeats) that takes it to exactly 0.9.  Answers are unique
    (the sort is stable), so they are compared per position."""
    w, L = 37, 27
    slots = 1 << L
    n_before, n_after = slots // 2, int(0.9 * slots)
    t = cpht.Table(scheme=cpht.CUCKOO, key_bits=w, log2_slots0=L, bucket0=32, slot_bits0=32, seed=81)
    t.bulk_build(synth.distinct_keys(w, SEED, 0, n_before, device=gpu))
    keys, idx = synth.find_or_put_batch(w, SEED, n_before, n_after - n_before, slots, 17, device=gpu)
    out = t.sorted_fop(keys)
    truth = _fop_truth(idx, n_before, gpu)
    bad = _diff(out, truth)
    assert bad == 0, f"{bad} find-or-put answers differ"
    assert t.count() == (n_after, slots)
    q, hit = _queries(w, n_after, 1 << 24, 8, gpu)
    bad = _diff(t.find(q), hit)
    assert bad == 0, f"{bad} find answers differ"


def test_iceberg_fop_full_size(gpu):
    """The iceberg side of the same experiment: 2^27 + 2^24 slots filled to
    0.5, one find-or-put batch of 2^27 + 2^24 keys taking it to 0.9.  Which
    repeat of a fresh key gets the PUT is timing-dependent, so the check is
    per key: exactly one PUT for each fresh key, FOUND everywhere else."""
    w, L0 = 37, 27
    cap = (1 << L0) + (1 << (L0 - 3))
    n_before, n_after = cap // 2, int(0.9 * cap)
    t = cpht.Table(scheme=cpht.ICEBERG, key_bits=w, log2_slots0=L0, log2_slots1=L0 - 3, bucket0=32, bucket1=16,
                   slot_bits0=16, slot_bits1=32, seed=82)
    t.insert(synth.distinct_keys(w, SEED, 0, n_before, device=gpu))
    keys, idx = synth.find_or_put_batch(w, SEED, n_before, n_after - n_before, cap, 18, device=gpu)
    out = t.insert(keys)
    n_full = _count(out == cpht.FULL)
    assert n_full == 0
    puts = torch.zeros(n_after, dtype=torch.int64, device=gpu)
    puts.scatter_add_(0, idx, (out == cpht.PUT).to(torch.int64))
    wrong_stored = _count(puts[:n_before] != 0)
    wrong_fresh = _count(puts[n_before:] != 1)
    assert wrong_stored == 0 and wrong_fresh == 0
    other = _count((out != cpht.PUT) & (out != cpht.FOUND))
    assert other == 0
    assert t.count() == (n_after, cap)


def test_c4_many_tables_full_size(gpu):
    """The many-table workload at its full size and in the set launch the
    benchmark times: 4096 compact iceberg tables of 2^e + 2^(e-3) slots, e
    uniform in 10..20, 32-bit keys, each filled to 0.85 and queried with twice
    its capacity (50 % hit), eagerly and through a replayed graph.

    A two-level table near its limit may answer FULL (the smallest tables at
    load 0.85 now and then do), so the answers fix the rest: every insert is
    PUT or FULL; a find answers 1 exactly for keys of its own table that were
    PUT (queries are drawn from the table's keys or from keys never inserted);
    each sampled table's count equals its PUTs, its decoded key set is exactly
    its PUT keys, and its FULL keys meet Theorem 1 (e).  Comparisons are
    reduced to counts before asserting (no huge tensors in failure reports)."""
    w, n_tables, load = 32, 4096, 0.85
    e_t = (synth.uniform_below(0xE5, n_tables, 11, gpu) + 10).cpu().tolist()
    cfgs = []
    for i, e in enumerate(e_t):
        c = cpht.default_config(cpht.ICEBERG)
        c.key_bits, c.log2_slots0, c.log2_slots1 = w, e, e - 3
        c.bucket0, c.bucket1, c.slot_bits0, c.slot_bits1, c.subtile = 16, 8, 32, 32, 2
        c.seed = 7000 + i
        cfgs.append(c)
    cap = torch.tensor([(1 << e) + (1 << (e - 3)) for e in e_t], dtype=torch.int64, device=gpu)
    n_t = (cap.double() * load).long()
    q_t = 2 * cap
    ko = torch.zeros(n_tables + 1, dtype=torch.int64, device=gpu)
    ko[1:] = torch.cumsum(n_t, 0)
    qo = torch.zeros(n_tables + 1, dtype=torch.int64, device=gpu)
    qo[1:] = torch.cumsum(q_t, 0)
    total_k, total_q = int(ko[-1]), int(qo[-1])
    keys64 = synth.distinct_keys(w, SEED + 9, 0, total_k, device=gpu)
    tid = torch.repeat_interleave(torch.arange(n_tables, device=gpu), q_t)
    pick = ko[tid] + ((synth.uniform_below(0xAB, total_q, 1 << 30, gpu) * n_t[tid]) >> 30)
    hit = synth.uniform_below(0xCD, total_q, 2, gpu) == 1
    miss = synth.distinct_keys(w, SEED + 9, total_k, total_q, device=gpu)
    queries = synth.to_words(torch.where(hit, keys64[pick], miss), w).contiguous()
    keys = synth.to_words(keys64, w).contiguous()
    del tid, miss
    m = cpht.MultiTable(cfgs, max_keys=max(total_k, total_q))
    out = torch.empty(total_k, dtype=torch.uint8, device=gpu)
    found = torch.empty(total_q, dtype=torch.uint8, device=gpu)

    def check_answers(tag):
        put = out == cpht.PUT
        n_put = int(put.sum().item())
        n_full = int((out == cpht.FULL).sum().item())
        assert n_put + n_full == total_k, f"{tag}: {total_k - n_put - n_full} answers neither PUT nor FULL"
        assert n_full < total_k // 10000, f"{tag}: {n_full} FULL answers"
        expect = (hit & put[pick]).to(torch.uint8)
        n_bad = int((found != expect).sum().item())
        assert n_bad == 0, f"{tag}: {n_bad} of {total_q} find answers differ"
        return put

    m.insert(keys, ko, out)
    m.find(queries, qo, found)
    assert m.error_flags() == 0
    put = check_answers("eager")
    kb = ko.tolist()
    full_tables = [i for i in range(n_tables) if not bool(put[kb[i]:kb[i + 1]].all().item())]
    sample = sorted(set(range(0, n_tables, n_tables // 16)) | set(full_tables[:8]) |
                    {min(range(n_tables), key=lambda i: e_t[i]), max(range(n_tables), key=lambda i: e_t[i])})
    for i in sample:
        v = m.table(i)
        ki = keys64[kb[i]:kb[i + 1]].cpu().numpy().astype(np.uint64)
        pi = put[kb[i]:kb[i + 1]].cpu().numpy()
        assert v.count()[0] == int(pi.sum()), f"table {i}"
        assert np.array_equal(check_table(v), np.sort(ki[pi])), f"table {i}"
        if not pi.all():
            ok, msg = oracle.check_full(oracle_cfg(v), v.export(0), v.export(1), ki[~pi])
            assert ok, f"table {i}: {msg}"
    # the same work captured once and replayed: every replay meets the same rules
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            m.insert(keys, ko, out, stream=s)
            m.find(queries, qo, found, stream=s)
    torch.cuda.synchronize()
    for r in range(2):
        m.clear()
        out.zero_()
        found.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        check_answers(f"replay {r}")


@pytest.mark.parametrize("scheme", ["cuckoo", "iceberg"])
def test_delete_full_size(gpu, scheme):
    """The delete workload at full size: a table at load 0.9 (2^27 slots
    cuckoo, 2^27 + 2^24 iceberg 16/32), one batch of 2^26 deletes, half of
    them distinct stored keys and half never inserted.  Per key: 1 exactly
    for the stored ones; afterwards the deleted keys are not found, every
    other stored key is, and the count dropped by the deleted keys."""
    w, L, nd = 37, 27, 1 << 26
    if scheme == "cuckoo":
        t = cpht.Table(scheme=cpht.CUCKOO, key_bits=w, log2_slots0=L, bucket0=32, slot_bits0=32, seed=83)
    else:
        t = cpht.Table(scheme=cpht.ICEBERG, key_bits=w, log2_slots0=L, log2_slots1=L - 3, bucket0=32, bucket1=16,
                       slot_bits0=16, slot_bits1=32, seed=83)
    cap = t.count()[1]
    n = int(0.9 * cap)
    keys = synth.distinct_keys(w, SEED + 5, 0, n, device=gpu)
    assert _count(t.insert(keys) != cpht.PUT) == 0
    perm = synth.permutation(77, n, device=gpu)
    gone = perm[: nd // 2]
    q = torch.cat([keys[gone], synth.distinct_keys(w, SEED + 5, n, nd // 2, device=gpu)])
    order = synth.permutation(78, nd, device=gpu)
    q = q[order]
    truth = (order < nd // 2).to(torch.uint8)  # position i holds a stored key iff it came from the first half
    bad = _diff(t.delete(q), truth)
    assert bad == 0, f"{bad} delete answers differ"
    assert t.count()[0] == n - nd // 2
    deleted = torch.zeros(n, dtype=torch.bool, device=gpu)
    deleted[gone] = True
    bad = _diff(t.find(keys), (~deleted).to(torch.uint8))
    assert bad == 0, f"{bad} lookups after the deletes differ"


def test_level3_full_size(gpu):
    """The third level at the benchmark's shape: 2^27 + 2^24 slots (16/32),
    2^17 lists and a pool of 2^20 slabs, distinct keys to load 1.0 of the
    bucket levels in one batch.  No FULL; the count equals the keys; every
    key is found and 2^24 never-inserted keys are not; the table checker
    walks every list of the images."""
    w, L = 37, 27
    t = cpht.Table(scheme=cpht.ICEBERG, key_bits=w, log2_slots0=L, log2_slots1=L - 3, bucket0=32, bucket1=16,
                   slot_bits0=16, slot_bits1=32, log2_lists=17, pool_slabs=1 << 20, seed=84)
    cap = t.count()[1]
    keys = synth.distinct_keys(w, SEED + 13, 0, cap, device=gpu)
    out = t.insert(keys)
    n_full = _count(out == cpht.FULL)
    assert n_full == 0
    assert _count(out != cpht.PUT) == 0
    assert t.count()[0] == cap
    used = t.level3_used()
    assert 0 < used < (1 << 20)
    missed = _count(t.find(keys) != 1)
    assert missed == 0
    false_hits = _count(t.find(synth.distinct_keys(w, SEED + 13, 1 << 36, 1 << 24, device=gpu)) != 0)
    assert false_hits == 0
    ok, msg, dec = oracle.check_images(oracle_cfg(t), *[t.export(x) for x in range(t.nimages)])
    assert ok, msg
    assert dec.size == cap


def test_map_full_size(gpu):
    """The map at the benchmark's shape: 2^27 + 2^24 slots (16/32) with 8-byte
    values, distinct keys to load 0.9 with value mix64(key), then 2^26 lookups
    (half hits): found flags exact, every value found is its key's."""
    w, L = 37, 27
    t = cpht.Table(scheme=cpht.ICEBERG, key_bits=w, log2_slots0=L, log2_slots1=L - 3, bucket0=32, bucket1=16,
                   slot_bits0=16, slot_bits1=32, value_bytes=8, seed=85)
    cap = t.count()[1]
    n = int(0.9 * cap)
    keys = synth.distinct_keys(w, SEED, 0, n, device=gpu)  # phi(i < n): the keys _queries draws hits from
    assert _count(t.insert_values(keys, synth.mix64_t(keys)) != cpht.PUT) == 0
    q, truth = _queries(w, n, 1 << 26, 9, gpu)
    found, vals = t.find_values(q)
    bad = _diff(found, truth)
    assert bad == 0, f"{bad} found flags differ"
    hit = truth.bool()
    wrong = _diff(vals[hit], synth.mix64_t(q[hit]))
    assert wrong == 0, f"{wrong} values differ"
