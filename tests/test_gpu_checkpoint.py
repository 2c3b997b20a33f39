"""Checkpoint / resume through raw images (cpht_export -> cpht_import): a
table rebuilt from its configuration and images answers every lookup as the
original, holds the same key set, and keeps working (the third level's slab
count is restored from the pool image, so new slabs follow the old ones)."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import paper_2406_09255_amd as cpht
import synth
from oracle import sets
from tests.helpers import check_table, host_u64, to_dev

pytestmark = pytest.mark.gpu

KEY_SEED = 0xC4EC


def test_cuckoo_checkpoint_restore(gpu):
    w = 37
    t = cpht.Table(scheme=cpht.CUCKOO, key_bits=w, log2_slots0=16, bucket0=32, slot_bits0=32, seed=3)
    keys = synth.distinct_keys(w, KEY_SEED, 0, 50000, device=gpu)
    assert (t.bulk_build(keys) == cpht.PUT).all()
    r = cpht.Table.restore(t.checkpoint())
    q = synth.find_queries(w, KEY_SEED, 50000, 100000, 0.5, 5, device=gpu)
    assert torch.equal(r.find(q), t.find(q))
    assert np.array_equal(check_table(r), check_table(t))
    assert all(np.array_equal(a, b) for a, b in zip(r.checkpoint()["images"], t.checkpoint()["images"]))


def test_iceberg_map_with_level3_checkpoint_restore(gpu):
    w = 30
    t = cpht.Table(scheme=cpht.ICEBERG, key_bits=w, log2_slots0=12, log2_slots1=9, bucket0=16, bucket1=8,
                   slot_bits0=32, slot_bits1=32, subtile=2, log2_lists=4, pool_slabs=300, value_bytes=8, seed=4)
    cap = t.count()[1]
    kh = host_u64(synth.distinct_keys(w, KEY_SEED + 1, 0, 2 * cap))
    dk = to_dev(torch.from_numpy(kh[:int(1.5 * cap)].astype(np.int64)), w, gpu)
    vals = synth.mix64_t(dk.to(torch.int64))
    assert (t.insert_values(dk, vals) == cpht.PUT).all()
    used = t.level3_used()
    assert used > 0
    r = cpht.Table.restore(t.checkpoint())
    assert r.level3_used() == used
    qall = to_dev(torch.from_numpy(kh.astype(np.int64)), w, gpu)
    f1, v1 = t.find_values(qall)
    f2, v2 = r.find_values(qall)
    assert torch.equal(f1, f2) and torch.equal(v1[f1.bool()], v2[f2.bool()])
    assert np.array_equal(check_table(r), check_table(t))
    # the restored table keeps working: the rest of the keys overflow into new slabs
    rest = to_dev(torch.from_numpy(kh[int(1.5 * cap):].astype(np.int64)), w, gpu)
    S = np.sort(kh[:int(1.5 * cap)])
    out = r.insert_values(rest, synth.mix64_t(rest.to(torch.int64)))
    ok, msg = sets.check_insert_outcomes(S, kh[int(1.5 * cap):], out.cpu().numpy())
    assert ok, msg
    assert np.array_equal(check_table(r), np.sort(kh))
    assert r.level3_used() > used
    f, v = r.find_values(qall)
    assert bool((f == 1).all()) and torch.equal(v, synth.mix64_t(qall.to(torch.int64)))


def test_import_rejects_wrong_size(gpu):
    t = cpht.Table(scheme=cpht.CUCKOO, key_bits=32, log2_slots0=12, bucket0=32, slot_bits0=32)
    img = t.export(0)
    with pytest.raises(cpht.CphtError):
        t.import_image(0, img[:-4])
    with pytest.raises(cpht.CphtError):
        t.import_image(1, img)
