"""Table sets (many tables, one launch per kernel variant) against the
oracle: every table of the set must behave exactly like a table of its own,
also when the batch runs inside a captured graph."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import paper_2406_09255_amd as cpht
import synth
from oracle import sets
from tests.helpers import check_table, host_u64

pytestmark = pytest.mark.gpu


def _configs(n, seed, scheme=cpht.ICEBERG, lo=10, hi=15, w=32):
    r = np.random.default_rng(seed)
    cfgs = []
    for i in range(n):
        e = int(r.integers(lo, hi + 1))
        c = cpht.default_config(scheme)
        c.key_bits = w
        c.seed = 1000 + i
        if scheme == cpht.ICEBERG:
            c.log2_slots0, c.log2_slots1 = e, e - 3
            c.bucket0, c.bucket1 = (32, 16) if i % 3 else (16, 8)
            c.slot_bits0, c.slot_bits1 = 32, 32
            c.subtile = 0 if i % 2 else (4 if c.bucket0 == 32 else 0)
        else:
            c.log2_slots0 = e
            c.bucket0, c.slot_bits0 = (32, 32) if i % 2 else (16, 32)
        cfgs.append(c)
    return cfgs


def _capacity(c):
    return (1 << c.log2_slots0) + ((1 << c.log2_slots1) if c.scheme == cpht.ICEBERG else 0)


def _batches(cfgs, w, load, qfac, seed):
    keys, queries, ko, qo, per_keys = [], [], [0], [0], []
    for i, c in enumerate(cfgs):
        n = int(load * _capacity(c))
        k = synth.distinct_keys(w, seed + i, 0, n)
        q = synth.find_queries(w, seed + i, n, qfac * _capacity(c), 0.5, seed + 7 * i)
        keys.append(k)
        queries.append(q)
        per_keys.append(k)
        ko.append(ko[-1] + n)
        qo.append(qo[-1] + q.numel())
    return (torch.cat(keys), torch.tensor(ko, dtype=torch.int64), torch.cat(queries),
            torch.tensor(qo, dtype=torch.int64), per_keys)


@pytest.mark.parametrize("scheme", [cpht.ICEBERG, cpht.CUCKOO])
def test_table_set_matches_oracle(gpu, scheme):
    w = 32
    cfgs = _configs(48, 5, scheme)
    load = 0.85 if scheme == cpht.ICEBERG else 0.9
    keys, ko, q, qo, per = _batches(cfgs, w, load, 2, 77)
    m = cpht.MultiTable(cfgs, max_keys=max(keys.numel(), q.numel()))
    assert m.info()["groups"] >= 2
    dk, dko = synth.to_words(keys, w).to(gpu), ko.to(gpu)
    out = m.insert(dk, dko).cpu().numpy()
    found = m.find(synth.to_words(q, w).to(gpu), qo.to(gpu)).cpu().numpy()
    assert m.error_flags() == 0
    hq = host_u64(q)
    for i, c in enumerate(cfgs):
        a, b = int(ko[i]), int(ko[i + 1])
        assert (out[a:b] == cpht.PUT).all(), f"table {i}"
        S = np.sort(host_u64(per[i]))
        t = m.table(i)
        assert np.array_equal(check_table(t), S), f"table {i}"
        qa, qb = int(qo[i]), int(qo[i + 1])
        assert np.array_equal(found[qa:qb], sets.find(S, hq[qa:qb])), f"table {i}"


def test_table_set_equals_separate_tables(gpu):
    """The same keys through single-table calls on each view give the same
    answers as the set-wide launch."""
    w = 32
    cfgs = _configs(16, 9)
    keys, ko, q, qo, per = _batches(cfgs, w, 0.8, 2, 91)
    m = cpht.MultiTable(cfgs, max_keys=q.numel())
    m.insert(synth.to_words(keys, w).to(gpu), ko.to(gpu))
    f_set = m.find(synth.to_words(q, w).to(gpu), qo.to(gpu)).cpu().numpy()
    m.clear()
    f_one = np.zeros_like(f_set)
    for i in range(len(cfgs)):
        t = m.table(i)
        t.insert(synth.to_words(keys[int(ko[i]):int(ko[i + 1])], w).to(gpu))
        f_one[int(qo[i]):int(qo[i + 1])] = t.find(synth.to_words(q[int(qo[i]):int(qo[i + 1])], w).to(gpu)).cpu().numpy()
    assert np.array_equal(f_set, f_one)


@pytest.mark.parametrize("scheme", [cpht.ICEBERG, cpht.CUCKOO])
def test_reseeded_view_is_used_by_set_launches(gpu, scheme):
    """cpht_clear with a new seed on one table's view: keys inserted through
    the view (single-table call, new permutations) are found by the set-wide
    find, and keys inserted by the set-wide insert afterwards are found
    through the view; answers as the oracle's table with the new seed."""
    w = 32
    cfgs = _configs(12, 17, scheme)
    keys, ko, q, qo, per = _batches(cfgs, w, 0.6, 2, 55)
    m = cpht.MultiTable(cfgs, max_keys=max(keys.numel(), q.numel()))
    dk, dko = synth.to_words(keys, w).to(gpu), ko.to(gpu)
    dq, dqo = synth.to_words(q, w).to(gpu), qo.to(gpu)
    m.insert(dk, dko)
    i = 5
    v = m.table(i)
    v.clear(0xABCDEF)
    a, b = int(ko[i]), int(ko[i + 1])
    half = a + (b - a) // 2
    assert (v.insert(dk[a:half]) == cpht.PUT).all()
    found = m.find(dq, dqo).cpu().numpy()
    c = v.config
    assert c.seed == 0xABCDEF
    o = oracle.Table(c.scheme, c.key_bits, c.log2_slots0, c.bucket0, c.slot_bits0, log2_slots1=c.log2_slots1,
                     B1=c.bucket1, s1=c.slot_bits1, H=c.n_hash, C=c.max_chain, compact=bool(c.compact), seed=c.seed)
    hk = host_u64(keys)
    assert (o.insert(hk[a:half]) == oracle.PUT).all()
    hq = host_u64(q)
    qa, qb = int(qo[i]), int(qo[i + 1])
    assert np.array_equal(found[qa:qb], o.find(hq[qa:qb]))
    assert np.array_equal(check_table(v), np.sort(hk[a:half]))
    # the other tables kept their seeds and contents
    for j in (0, 11):
        ja, jb = int(qo[j]), int(qo[j + 1])
        S = np.sort(host_u64(per[j]))
        assert np.array_equal(found[ja:jb], sets.find(S, hq[ja:jb]))
    # the set-wide insert places keys by the new permutations as well
    sub_off = torch.zeros(len(cfgs) + 1, dtype=torch.int64)
    sub_off[i + 1:] = b - half
    sub = dk[half:b].contiguous()
    out = m.insert(sub, sub_off.to(gpu)).cpu().numpy()
    assert (out == cpht.PUT).all()
    assert (o.insert(hk[half:b]) == oracle.PUT).all()
    assert (v.find(dk[a:b]) == 1).all()
    ok, msg, dec = o.check()
    assert ok, msg
    assert np.array_equal(check_table(v), dec)


def test_table_set_in_captured_graph(gpu):
    """insert + find of every table captured once and replayed; each replay
    (with an eager clear between replays) must equal the eager run."""
    w = 32
    cfgs = _configs(32, 13)
    keys, ko, q, qo, per = _batches(cfgs, w, 0.85, 2, 31)
    m = cpht.MultiTable(cfgs, max_keys=q.numel())
    dk, dko = synth.to_words(keys, w).to(gpu), ko.to(gpu)
    dq, dqo = synth.to_words(q, w).to(gpu), qo.to(gpu)
    out = torch.empty(dk.numel(), dtype=torch.uint8, device=gpu)
    found = torch.empty(dq.numel(), dtype=torch.uint8, device=gpu)
    m.insert(dk, dko, out)
    m.find(dq, dqo, found)
    torch.cuda.synchronize()
    want_out, want_found = out.cpu().clone(), found.cpu().clone()
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    m.clear()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            m.insert(dk, dko, out, stream=s)
            m.find(dq, dqo, found, stream=s)
    torch.cuda.synchronize()
    for rep in range(3):
        m.clear()
        out.fill_(0)
        found.fill_(9)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out.cpu(), want_out), rep
        assert torch.equal(found.cpu(), want_found), rep
    for i in (0, 7, 31):
        assert np.array_equal(check_table(m.table(i)), np.sort(host_u64(per[i])))


def test_table_set_rejects_oversized_batch(gpu):
    cfgs = _configs(4, 3)
    m = cpht.MultiTable(cfgs, max_keys=1000)
    k = torch.zeros(2000, dtype=torch.int32, device=gpu)
    off = torch.tensor([0, 500, 1000, 1500, 2000], dtype=torch.int64, device=gpu)
    with pytest.raises(cpht.CphtError):
        m.insert(k, off)
    with pytest.raises(ValueError):  # a result buffer shorter than the batch
        m.insert(k[:1000], off.clamp(max=1000), out=torch.empty(999, dtype=torch.uint8, device=gpu))
    view = m.table(1)
    assert cpht.lib().cpht_destroy(view._h) == 7  # views cannot be destroyed on their own
