"""The serving loop's resident mode: one persistent launch takes requests
from a ring in pinned host memory.  Every answer must be the one the request
gets alone (finds of keys that no request inserts are fixed; inserts follow
the put-once rule over the stream), the final key set must be the union, and
the loop must end when idle and start again for the next request."""
from __future__ import annotations

import time

import numpy as np
import pytest
import torch

import paper_2406_09255_amd as cpht
import synth
from oracle import sets
from tests.helpers import check_table, host_u64
from tests.test_gpu_server import W, _packed, _prefill, _requests, _run, _table

pytestmark = pytest.mark.gpu


def _check_stream(reqs, outs, S0):
    """Each request against the set semantics applied in submission order;
    requests do not share insert keys, so only their own repeats race."""
    S = S0
    for i, ((k, o), res) in enumerate(zip(reqs, outs)):
        hk, ho = host_u64(k), o.numpy()
        want, S_after, racy = sets.mixed(S, hk, ho)
        f = ho == 0
        assert not racy.any()
        assert np.array_equal(res[f], want[f]), f"request {i}: finds"
        ok, msg = sets.check_insert_outcomes(S, hk[~f], res[~f])
        assert ok, f"request {i}: {msg}"
        S = S_after
    return S


def test_resident_stream_matches_set_semantics(gpu):
    pre = 50000
    reqs = _packed(_requests(150, pre, 11, pre))
    t = _table(31)
    S0 = _prefill(t, gpu, pre)
    srv = cpht.Server(t, zero_copy=1, resident=1, max_batch_keys=1 << 16)
    outs, lat = _run(srv, reqs, packed=True)
    st = srv.stats()
    srv.stop()
    assert st["requests_done"] == len(reqs) and st["launches"] >= 1
    S = _check_stream(reqs, outs, S0)
    assert np.array_equal(check_table(t), S)
    assert all(x > 0 for x in lat)


def test_resident_equals_launch_per_request(gpu):
    """The same requests through the resident loop and through one launch per
    request (zero-copy, one in flight) give the same answers and tables."""
    pre = 20000
    reqs = _packed(_requests(60, pre, 12, pre))
    t_res, t_one = _table(32), _table(32)
    S0 = _prefill(t_res, gpu, pre)
    _prefill(t_one, gpu, pre)
    res = cpht.Server(t_res, zero_copy=1, resident=1, max_batch_keys=1 << 16)
    out_res, _ = _run(res, reqs, packed=True)
    res.stop()
    one = cpht.Server(t_one, zero_copy=1, max_inflight=1, coalesce=0)
    out_one, _ = _run(one, reqs, wait_each=True, packed=True)
    one.stop()
    for i, ((k, o), a, b) in enumerate(zip(reqs, out_res, out_one)):
        f = o.numpy() == 0
        assert np.array_equal(a[f], b[f]), f"request {i}"
    S = _check_stream(reqs, out_res, S0)
    assert np.array_equal(check_table(t_res), S)
    assert np.array_equal(check_table(t_one), S)


def test_resident_ring_wraps_and_large_requests(gpu):
    """More requests than ring slots in flight at once (the ring wraps while
    the loop runs), mixed with requests of many chunks each."""
    pre = 20000
    r = np.random.default_rng(13)
    sizes = np.where(r.random(2600) < 0.01, r.integers(20000, 60000, 2600), r.integers(1, 300, 2600))
    n = int(sizes.sum())
    n_ins = n // 3
    idx = np.concatenate([pre + np.arange(n_ins), r.integers(0, pre, n - n_ins)])
    ops = np.concatenate([np.ones(n_ins, np.uint8), np.zeros(n - n_ins, np.uint8)])
    p = r.permutation(n)
    keys = synth.to_words(synth.feistel(W, 77, torch.from_numpy(idx[p].astype(np.int64))), W).pin_memory()
    ops_t = torch.from_numpy(ops[p]).pin_memory()
    cuts = np.concatenate([[0], np.cumsum(sizes)])
    reqs = [(keys[a:b], ops_t[a:b]) for a, b in zip(cuts[:-1], cuts[1:])]
    t = _table(33)
    S0 = _prefill(t, gpu, pre)
    srv = cpht.Server(t, zero_copy=1, resident=1, coalesce=0, max_batch_keys=1 << 16)  # one descriptor per request
    t0 = time.perf_counter()
    outs, _ = _run(srv, reqs, packed=True)
    print(f"{len(reqs)} requests, {n} operations in {time.perf_counter() - t0:.3f} s", flush=True)
    srv.stop()
    res = np.concatenate(outs)
    hk, ho = host_u64(keys), ops_t.numpy()
    f = ho == 0
    assert (res[f] == 1).all()  # every find looks for a pre-filled key
    assert (res[~f] == cpht.PUT).all()  # every insert key is fresh and distinct
    assert np.array_equal(check_table(t), np.union1d(S0, hk[~f]))


def test_resident_burst_of_small_requests_64_bit_keys(gpu):
    """20,000 small requests in separate pinned buffers (no two adjacent, so
    one descriptor each) submitted at once on a table of 40-bit keys: the
    leader copies descriptors in bursts; every answer is checked."""
    w = 40
    t = cpht.Table(scheme=cpht.ICEBERG, key_bits=w, log2_slots0=22, log2_slots1=19, bucket0=32, bucket1=16,
                   slot_bits0=32, slot_bits1=32, seed=37)
    pre = 100000
    pk = synth.to_words(synth.feistel(w, 78, torch.arange(pre, dtype=torch.int64)), w).to(gpu)
    assert (t.insert(pk) == cpht.PUT).all()
    r = np.random.default_rng(15)
    n_req, size = 20000, 64
    fresh = pre + np.arange(n_req * size // 2)
    reqs, outs = [], []
    for i in range(n_req):
        idx = np.concatenate([fresh[i * size // 2:(i + 1) * size // 2], r.integers(0, pre, size // 2)])
        ops = np.concatenate([np.ones(size // 2, np.uint8), np.zeros(size // 2, np.uint8)])
        k = synth.to_words(synth.feistel(w, 78, torch.from_numpy(idx.astype(np.int64))), w)
        # separate pinned buffers with a gap: never adjacent
        kb = torch.empty(size + 8, dtype=k.dtype).pin_memory()[:size]
        kb.copy_(k)
        ob = torch.empty(size + 8, dtype=torch.uint8).pin_memory()[:size]
        ob.copy_(torch.from_numpy(ops))
        reqs.append((kb, ob))
        outs.append(torch.zeros(size + 8, dtype=torch.uint8).pin_memory()[:size])
    srv = cpht.Server(t, zero_copy=1, resident=1, max_batch_keys=1 << 16)
    t0 = time.perf_counter()
    tickets = [srv.submit(k, o, out) for (k, o), out in zip(reqs, outs)]
    lat = [srv.wait(tk) for tk in tickets]
    dt = time.perf_counter() - t0
    st = srv.stats()
    srv.stop()
    print(f"{n_req} requests of {size} in {dt:.3f} s, {st['launches']} loop launches", flush=True)
    res = np.stack([o.numpy() for o in outs])
    assert (res[:, : size // 2] == cpht.PUT).all() and (res[:, size // 2:] == 1).all()
    assert t.count()[0] == pre + n_req * size // 2
    assert min(lat) > 0


def test_resident_loop_ends_when_idle_and_restarts(gpu):
    pre = 5000
    reqs = _packed(_requests(6, pre, 14, pre))
    t = _table(34)
    S0 = _prefill(t, gpu, pre)
    srv = cpht.Server(t, zero_copy=1, resident=1, idle_us=300, max_batch_keys=1 << 16)
    outs = []
    for k, o in reqs:
        out = torch.zeros(k.numel(), dtype=torch.uint8).pin_memory()
        srv.wait(srv.submit(k, o, out))
        outs.append(out.numpy().copy())
        time.sleep(0.02)  # far longer than idle_us: the loop has ended before the next request
    st = srv.stats()
    srv.stop()
    assert st["launches"] >= len(reqs)  # started again for every request
    S = _check_stream(reqs, outs, S0)
    assert np.array_equal(check_table(t), S)


def test_resident_configuration_checks(gpu):
    t = _table(35)
    with pytest.raises(cpht.CphtError) as e:  # resident needs zero-copy request buffers
        cpht.Server(t, resident=1)
    assert e.value.code == 1
    with pytest.raises(cpht.CphtError) as e:
        cpht.Server(t, zero_copy=1, resident=1, idle_us=0)
    assert e.value.code == 1
    l3 = cpht.Table(scheme=cpht.ICEBERG, key_bits=20, log2_slots0=16, log2_slots1=13, bucket0=32, bucket1=16,
                    slot_bits0=16, slot_bits1=32, log2_lists=6, pool_slabs=256, seed=36)
    with pytest.raises(cpht.CphtError) as e:  # two-level tables only
        cpht.Server(l3, zero_copy=1, resident=1, max_batch_keys=1 << 16)
    assert e.value.code == 3
    with pytest.raises(cpht.CphtError) as e:  # descriptors beyond the covered size
        cpht.Server(t, zero_copy=1, resident=1, max_batch_keys=1 << 18)
    assert e.value.code == 3
    big = cpht.Table(scheme=cpht.ICEBERG, key_bits=W, log2_slots0=25, log2_slots1=22, bucket0=32, bucket1=16,
                     slot_bits0=16, slot_bits1=32, seed=38)
    with pytest.raises(cpht.CphtError) as e:  # tables beyond the covered size
        cpht.Server(big, zero_copy=1, resident=1, max_batch_keys=1 << 16)
    assert e.value.code == 3


def test_resident_chunk_sizes_follow_the_work_in_flight(gpu):
    """The loop cuts each request into chunks sized from the operations in
    flight: a lone request of 2^17 operations (small chunks, spread over the
    workers), then 64 such requests at once (large chunks), then a lone one
    again.  Per request the first 256 operations insert fresh keys (PUT), the
    rest alternate find-or-put and find of pre-filled keys (FOUND, 1)."""
    pre, size, n_fresh = 300000, 1 << 17, 256
    t = _table(39)
    S0 = _prefill(t, gpu, pre)
    srv = cpht.Server(t, zero_copy=1, resident=1, coalesce=0, max_batch_keys=size)
    j = torch.arange(size, dtype=torch.int64)
    first = j < n_fresh
    ops = torch.where(first | (j % 2 == 0), 1, 0).to(torch.uint8)
    want = torch.where(first, cpht.PUT, torch.where(j % 2 == 0, cpht.FOUND, 1)).to(torch.uint8)
    fresh_next, fresh_all = pre, []
    for phase, n_req in enumerate((1, 64, 1)):
        reqs, outs = [], []
        for i in range(n_req):
            idx = torch.where(first, fresh_next + j, (j * 7 + 13 * (i + 64 * phase)) % pre)
            fresh_all.append(idx[:n_fresh])
            fresh_next += n_fresh
            kb = synth.to_words(synth.feistel(W, 77, idx), W).pin_memory()
            reqs.append((kb, ops.pin_memory()))
            outs.append(torch.zeros(size, dtype=torch.uint8).pin_memory())
        tickets = [srv.submit(k, o, r) for (k, o), r in zip(reqs, outs)]
        for tk in tickets:
            srv.wait(tk)
        for i, r in enumerate(outs):
            bad = torch.nonzero(r != want).flatten()
            assert bad.numel() == 0, f"phase {phase}, request {i}: {bad.numel()} wrong answers, first at {bad[:5]}"
    srv.stop()
    fresh_keys = host_u64(synth.feistel(W, 77, torch.cat(fresh_all)))
    assert np.array_equal(check_table(t), np.union1d(S0, fresh_keys))


def test_resident_many_idle_exits_between_bursts(gpu):
    """Forty bursts of three requests with a pause longer than idle_us after
    each: every burst finds the loop ended, so each launch starts by taking
    back the tickets the previous one gave up; every answer and the final key
    set follow the set semantics."""
    pre = 8000
    reqs = _packed(_requests(120, pre, 16, pre))
    t = _table(40)
    S0 = _prefill(t, gpu, pre)
    srv = cpht.Server(t, zero_copy=1, resident=1, idle_us=100, max_batch_keys=1 << 16)
    outs = []
    for b in range(0, len(reqs), 3):
        burst = reqs[b:b + 3]
        res = [torch.zeros(k.numel(), dtype=torch.uint8).pin_memory() for k, _ in burst]
        tickets = [srv.submit(k, o, r) for (k, o), r in zip(burst, res)]
        for tk in tickets:
            srv.wait(tk)
        outs.extend(r.numpy().copy() for r in res)
        time.sleep(0.003)  # well past idle_us: the loop ends before the next burst
    st = srv.stats()
    srv.stop()
    assert st["requests_done"] == len(reqs)
    assert st["launches"] >= 20  # most bursts started a new launch
    S = _check_stream(reqs, outs, S0)
    assert np.array_equal(check_table(t), S)
