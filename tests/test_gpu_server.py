"""The serving loop: requests admitted and batched continuously must give
each request the answers it gets alone, apart from finds racing inserts of
other in-flight requests (the dynamic-operation rule of Sec. 3)."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import paper_2406_09255_amd as cpht
import synth
from oracle import sets
from tests.helpers import check_table, host_u64

pytestmark = pytest.mark.gpu

W = 30


def _table(seed=21):
    return cpht.Table(scheme=cpht.ICEBERG, key_bits=W, log2_slots0=20, log2_slots1=17, bucket0=32, bucket1=16,
                      slot_bits0=16, slot_bits1=32, seed=seed)


def _requests(n_req, pre_n, seed, fresh_start, shared=False):
    """Requests of uneven size: 30 % inserts (fresh keys, 30 % repeated inside
    the request), 70 % finds (half keys present before, half never inserted).
    With shared=True the insert keys of neighbouring requests overlap."""
    r = np.random.default_rng(seed)
    sizes = np.clip(np.round(np.exp(r.normal(np.log(600), 1.2, n_req))), 1, 20000).astype(np.int64)
    reqs, fresh = [], fresh_start
    for i, n in enumerate(sizes):
        n_ins = int(round(0.3 * n))
        if shared:
            base = fresh_start + (i // 2) * 400
            ins_idx = base + r.integers(0, 400, n_ins)
        else:
            ins_idx = fresh + np.minimum(np.arange(n_ins), np.maximum(0, (np.arange(n_ins) * 0.7).astype(np.int64)))
            fresh += n_ins
        hit_idx = r.integers(0, pre_n, n - n_ins)
        miss_idx = (1 << 28) + seed * 1000000 + i * 30000 + np.arange(n - n_ins)
        is_hit = r.random(n - n_ins) < 0.5
        find_idx = np.where(is_hit, hit_idx, miss_idx)
        idx = np.concatenate([ins_idx, find_idx])
        ops = np.concatenate([np.ones(n_ins, np.uint8), np.zeros(n - n_ins, np.uint8)])
        p = r.permutation(n)
        keys = synth.feistel(W, 77, torch.from_numpy(idx[p].astype(np.int64)))
        reqs.append((synth.to_words(keys, W).pin_memory(), torch.from_numpy(ops[p]).pin_memory()))
    return reqs


def _prefill(t, gpu, n):
    keys = synth.feistel(W, 77, torch.arange(n, dtype=torch.int64))
    out = t.insert(synth.to_words(keys, W).to(gpu)).cpu().numpy()
    assert (out == cpht.PUT).all()
    return np.sort(host_u64(keys))


def _packed(reqs):
    """The same requests as views of one pinned buffer per field, back to back
    in arrival order (what zero-copy launches coalesce)."""
    keys = torch.cat([k for k, _ in reqs]).pin_memory()
    ops = torch.cat([o for _, o in reqs]).pin_memory()
    cuts = np.cumsum([0] + [k.numel() for k, _ in reqs])
    return [(keys[a:b], ops[a:b]) for a, b in zip(cuts[:-1], cuts[1:])]


def _run(server, reqs, wait_each=False, packed=False):
    if packed:  # packed requests get packed outputs
        buf = torch.zeros(sum(k.numel() for k, _ in reqs), dtype=torch.uint8).pin_memory()
        cuts = np.cumsum([0] + [k.numel() for k, _ in reqs])
        outs = [buf[a:b] for a, b in zip(cuts[:-1], cuts[1:])]
    else:
        outs = [torch.zeros(k.numel(), dtype=torch.uint8).pin_memory() for k, _ in reqs]
    lat = []
    if wait_each:
        for (k, o), out in zip(reqs, outs):
            lat.append(server.wait(server.submit(k, o, out)))
    else:
        tickets = [server.submit(k, o, out) for (k, o), out in zip(reqs, outs)]
        lat = [server.wait(tk) for tk in tickets]
    return [o.numpy().copy() for o in outs], lat


@pytest.mark.parametrize("zero_copy", [0, 1])
def test_server_alone_equals_mix(gpu, zero_copy):
    pre = 50000
    reqs = _requests(120, pre, 1, pre)
    if zero_copy:
        reqs = _packed(reqs)
    t_mix, t_alone = _table(), _table()
    S0 = _prefill(t_mix, gpu, pre)
    _prefill(t_alone, gpu, pre)
    mix = cpht.Server(t_mix, max_inflight=4, coalesce=1, staging_keys=1 << 16, max_batch_keys=1 << 14,
                      zero_copy=zero_copy)
    out_mix, lat = _run(mix, reqs, packed=bool(zero_copy))
    st = mix.stats()
    mix.stop()
    alone = cpht.Server(t_alone, max_inflight=1, coalesce=0, staging_keys=1 << 16, max_batch_keys=1 << 14,
                        zero_copy=zero_copy)
    out_alone, _ = _run(alone, reqs, wait_each=True, packed=bool(zero_copy))
    alone.stop()
    assert st["requests_done"] == len(reqs) and st["launches"] < len(reqs)  # requests were coalesced
    S = S0
    for i, ((k, o), a, b) in enumerate(zip(reqs, out_mix, out_alone)):
        hk, ho = host_u64(k), o.numpy()
        want, S_after, racy = sets.mixed(S, hk, ho)
        f = ho == 0
        assert not racy.any()
        assert np.array_equal(a[f], want[f]) and np.array_equal(b[f], want[f]), f"request {i}"
        for res in (a, b):
            ok, msg = sets.check_insert_outcomes(S, hk[~f], res[~f])
            assert ok, f"request {i}: {msg}"
        S = S_after
    assert np.array_equal(check_table(t_mix), S)
    assert np.array_equal(check_table(t_alone), S)
    assert all(x > 0 for x in lat)


def test_server_overlapping_requests(gpu):
    """Neighbouring requests insert the same keys: over the whole stream each
    key is PUT exactly once; finds of keys present before the stream are 1,
    of keys never inserted 0."""
    pre = 20000
    reqs = _requests(80, pre, 2, pre, shared=True)
    t = _table(22)
    S0 = _prefill(t, gpu, pre)
    srv = cpht.Server(t, max_inflight=6, coalesce=1, staging_keys=1 << 15, max_batch_keys=1 << 12)
    outs, _ = _run(srv, reqs)
    srv.stop()
    all_k = np.concatenate([host_u64(k) for k, _ in reqs])
    all_o = np.concatenate([o.numpy() for _, o in reqs])
    all_r = np.concatenate(outs)
    ins = all_o == 1
    ok, msg = sets.check_insert_outcomes(S0, all_k[ins], all_r[ins])
    assert ok, msg
    S_end = np.union1d(S0, all_k[ins])
    f = ~ins
    fixed = f & (np.isin(all_k, S0) | ~np.isin(all_k, S_end))
    assert np.array_equal(all_r[fixed], np.isin(all_k[fixed], S0).astype(np.uint8))
    assert np.isin(all_r[f & ~fixed], [0, 1]).all()
    assert np.array_equal(check_table(t), S_end)


def test_server_admission_waits_for_staging(gpu):
    """A staging ring far smaller than the stream: requests are admitted only
    as earlier launches free their space, and all complete correctly."""
    pre = 10000
    reqs = _requests(60, pre, 3, pre)
    t = _table(23)
    S = _prefill(t, gpu, pre)
    biggest = max(k.numel() for k, _ in reqs)
    srv = cpht.Server(t, max_inflight=3, coalesce=1, staging_keys=biggest + 64, max_batch_keys=biggest)
    outs, _ = _run(srv, reqs)
    srv.stop()
    for (k, o), res in zip(reqs, outs):
        hk, ho = host_u64(k), o.numpy()
        want, S, _ = sets.mixed(S, hk, ho)
        f = ho == 0
        assert np.array_equal(res[f], want[f])


def test_server_staging_sized_from_free_memory(gpu):
    """staging_keys = 0: the ring (the admission budget) is sized at start
    from the free device memory; requests are served as with a fixed ring."""
    pre = 10000
    reqs = _requests(30, pre, 5, pre)
    t = _table(24)
    S = _prefill(t, gpu, pre)
    srv = cpht.Server(t, max_inflight=2, coalesce=1, staging_keys=0, max_batch_keys=1 << 16)
    outs, _ = _run(srv, reqs)
    srv.stop()
    for (k, o), res in zip(reqs, outs):
        hk, ho = host_u64(k), o.numpy()
        want, S, _ = sets.mixed(S, hk, ho)
        f = ho == 0
        assert np.array_equal(res[f], want[f])
        assert np.isin(res[~f], [cpht.PUT, cpht.FOUND]).all()


@pytest.mark.parametrize("zero_copy", [0, 1])
def test_server_trace_replay(gpu, zero_copy):
    pre = 30000
    reqs = _requests(200, pre, 4, pre)
    t = _table(24)
    S = _prefill(t, gpu, pre)
    keys = torch.cat([k for k, _ in reqs]).pin_memory()
    ops = torch.cat([o for _, o in reqs]).pin_memory()
    out = torch.zeros(keys.numel(), dtype=torch.uint8).pin_memory()
    offsets = np.concatenate([[0], np.cumsum([k.numel() for k, _ in reqs])]).astype(np.uint64)
    arrival = (np.cumsum(np.random.default_rng(5).exponential(20000.0, len(reqs)))).astype(np.uint64)
    srv = cpht.Server(t, zero_copy=zero_copy)
    lat, makespan = srv.replay(arrival, offsets, keys, ops, out)
    srv.stop()
    assert (lat > 0).all() and makespan >= arrival[-1]
    res = out.numpy()
    for i, (k, o) in enumerate(reqs):
        a, b = int(offsets[i]), int(offsets[i + 1])
        hk, ho = host_u64(k), o.numpy()
        want, S, _ = sets.mixed(S, hk, ho)
        f = ho == 0
        assert np.array_equal(res[a:b][f], want[f]), i


def test_server_needs_dynamic_table(gpu):
    c = cpht.Table(scheme=cpht.CUCKOO, key_bits=32, log2_slots0=12, bucket0=32, slot_bits0=32)
    with pytest.raises(cpht.CphtError):
        cpht.Server(c)


def test_server_zero_copy_needs_pinned_buffers(gpu):
    t = _table(25)
    srv = cpht.Server(t, zero_copy=1)
    keys = synth.to_words(synth.feistel(W, 77, torch.arange(100, dtype=torch.int64)), W)
    ops = torch.zeros(100, dtype=torch.uint8)
    out = torch.zeros(100, dtype=torch.uint8)
    with pytest.raises(cpht.CphtError):  # pageable host memory: the device cannot read it in place
        srv.submit(keys, ops, out)
    pk, po, pout = keys.pin_memory(), ops.pin_memory(), out.pin_memory()
    with pytest.raises(cpht.CphtError):  # one pageable buffer is enough to refuse
        srv.submit(pk, po, out)
    srv.wait(srv.submit(pk, po, pout))
    assert (pout.numpy() == 0).all()  # an empty table finds nothing
    srv.stop()


def test_server_replay_rejects_offsets_past_buffers(gpu):
    t = _table(26)
    srv = cpht.Server(t)
    keys = synth.to_words(synth.feistel(W, 77, torch.arange(100, dtype=torch.int64)), W).pin_memory()
    ops = torch.zeros(100, dtype=torch.uint8).pin_memory()
    out = torch.zeros(100, dtype=torch.uint8).pin_memory()
    arrival = np.zeros(2, dtype=np.uint64)
    with pytest.raises(ValueError):  # the second request would read keys 100..149
        srv.replay(arrival, np.array([0, 50, 150], dtype=np.uint64), keys, ops, out)
    with pytest.raises(ValueError):  # one offset short
        srv.replay(arrival, np.array([0, 50], dtype=np.uint64), keys, ops, out)
    lat, _ = srv.replay(arrival, np.array([0, 50, 100], dtype=np.uint64), keys, ops, out)
    srv.stop()
    assert (lat > 0).all() and (out.numpy() == 0).all()
