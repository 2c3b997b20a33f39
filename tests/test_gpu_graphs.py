"""Single-table calls captured in a HIP graph (through torch.cuda.graph) and
replayed: every replay, with eager work and synchronisations between the
replays, gives the answers of the eager run.  The captured calls launch
kernels only (the clear is a fill kernel, no memset node)."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import paper_2406_09255_amd as cpht
import synth
from tests.helpers import check_table, host_u64

pytestmark = pytest.mark.gpu


def _capture(fn):
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            fn(s)
    torch.cuda.synchronize()
    return g


def test_cuckoo_clear_build_find_graph(gpu):
    """The benchmark step (clear with a seed, bulk build, finds) as one graph."""
    w = 37
    t = cpht.Table(scheme=cpht.CUCKOO, key_bits=w, log2_slots0=20, bucket0=32, slot_bits0=32, seed=1)
    n = int(0.9 * (1 << 20))
    keys = synth.distinct_keys(w, 0x6A, 0, n, device=gpu)
    q = synth.find_queries(w, 0x6A, n, 1 << 18, 0.5, 5, device=gpu)
    out = torch.empty(n, dtype=torch.uint8, device=gpu)
    found = torch.empty(q.numel(), dtype=torch.uint8, device=gpu)

    def step(s=None):
        t.clear(7, stream=s)
        t.bulk_build(keys, out, stream=s)
        t.find(q, found, stream=s)

    step()
    torch.cuda.synchronize()
    want_out, want_found = out.clone(), found.clone()
    want_set = check_table(t)
    g = _capture(step)
    for rep in range(3):
        # eager work between replays.  The graph holds the permutation of the
        # seed current at capture (kernel arguments are fixed then), so the
        # eager clear keeps that seed for the host view to match the replays.
        t.clear(7)
        t.find(q[:1000])
        out.fill_(0)
        found.fill_(9)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert int((out != want_out).sum()) == 0, rep
        assert int((found != want_found).sum()) == 0, rep
        assert np.array_equal(check_table(t), want_set), rep


def test_iceberg_mixed_graph(gpu):
    """A mixed batch on a pre-filled iceberg table, replayed after restoring
    the table from its image each time."""
    w = 34
    t = cpht.Table(scheme=cpht.ICEBERG, key_bits=w, log2_slots0=20, log2_slots1=17, bucket0=32, bucket1=16,
                   slot_bits0=32, slot_bits1=32, seed=2)
    pre = synth.distinct_keys(w, 0x6B, 0, 400000, device=gpu)
    t.insert(pre)
    torch.cuda.synchronize()
    img = [t.export(x) for x in range(t.nimages)]
    fresh = synth.distinct_keys(w, 0x6B, 400000, 100000, device=gpu)
    kk = torch.cat([pre[:100000], fresh, fresh[:50000]])
    ops = torch.cat([torch.zeros(100000, dtype=torch.uint8), torch.ones(150000, dtype=torch.uint8)]).to(gpu)
    out = torch.empty(kk.numel(), dtype=torch.uint8, device=gpu)
    g = _capture(lambda s: t.mixed(kk, ops, out, stream=s))
    for rep in range(3):
        for x, im in enumerate(img):
            t.import_image(x, im)
        out.fill_(0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        o = out.cpu().numpy()
        assert (o[:100000] == 1).all(), rep                       # finds of stored keys
        first, again = o[100000:200000], o[200000:]
        # each fresh key inserted twice: one PUT and one FOUND, in either order
        pair = np.stack([first[:50000], again], 1)
        assert ((pair == [cpht.PUT, cpht.FOUND]).all(1) | (pair == [cpht.FOUND, cpht.PUT]).all(1)).all(), rep
        assert (first[50000:] == cpht.PUT).all(), rep
        assert np.array_equal(check_table(t), np.sort(np.concatenate([host_u64(pre), host_u64(fresh)]))), rep


def test_sorted_find_or_put_graph(gpu):
    """The sorted cuckoo find-or-put keeps its device-side counts on the
    device, so the whole call is one graph."""
    w = 37
    t = cpht.Table(scheme=cpht.CUCKOO, key_bits=w, log2_slots0=18, bucket0=32, slot_bits0=32, seed=3)
    n_before = 1 << 16
    t.bulk_build(synth.distinct_keys(w, 0x6C, 0, n_before, device=gpu))
    torch.cuda.synchronize()
    img = t.export(0)
    keys, _ = synth.find_or_put_batch(w, 0x6C, n_before, 1 << 16, 1 << 18, 4, device=gpu)
    ws = torch.empty(t.sorted_fop_workspace(keys.numel()), dtype=torch.uint8, device=gpu)
    out = torch.empty(keys.numel(), dtype=torch.uint8, device=gpu)
    t.sorted_fop(keys, out, ws)
    torch.cuda.synchronize()
    want = out.clone()
    want_set = check_table(t)
    g = _capture(lambda s: t.sorted_fop(keys, out, ws, stream=s))
    for rep in range(3):
        t.import_image(0, img)
        out.fill_(0)
        ws.fill_(0xAB)  # scratch contents must not matter
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert int((out != want).sum()) == 0, rep
        assert np.array_equal(check_table(t), want_set), rep
