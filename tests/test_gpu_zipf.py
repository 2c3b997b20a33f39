"""Dynamic operation under skew, scaled down: mixed batches of find-or-puts and
finds whose keys are Zipf(1.1) draws (the skewed stream of the dynamic
workload), on an iceberg table of 2^22 + 2^19 slots with the benchmark's
bucket shape (32 x 16-bit primary, 16 x 32-bit secondary; 32-bit keys, the
widest the 16-bit primary slots hold at this size), run until load 0.9.
Every batch is checked against the oracle's set semantics: per distinct key
one PUT (or all FOUND if stored before the batch), finds fixed except where
the batch itself inserts the key; at the end the table checker decodes the
images and the key set must equal the oracle's."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import paper_2406_09255_amd as cpht
import synth
from oracle import sets
from tests.helpers import check_table, host_u64

pytestmark = pytest.mark.gpu


def test_zipf_mixed_stream_to_load_09(gpu):
    w, L0, batch = 32, 22, 1 << 20
    t = cpht.Table(scheme=cpht.ICEBERG, key_bits=w, log2_slots0=L0, log2_slots1=L0 - 3, bucket0=32, bucket1=16,
                   slot_bits0=16, slot_bits1=32, seed=0x21F)
    cap = t.count()[1]
    ops = synth.uniform_below(0x2F, batch, 2, gpu).to(torch.uint8)
    ho = ops.cpu().numpy()
    ins_m = ho == 1
    S = np.zeros(0, np.uint64)
    out = torch.empty(batch, dtype=torch.uint8, device=gpu)
    b, racy_total = 0, 0
    while S.size < 0.9 * cap:
        assert b < 200, "the stream should reach load 0.9 in about 50 batches"
        keys = synth.zipf_keys(w, 0x2F1F, 1.1, batch, 5000 + b, device=gpu)
        t.mixed(synth.to_words(keys, w), ops, out)
        got = out.cpu().numpy()
        hk = host_u64(keys)
        seq, S_after, racy = sets.mixed(S, hk, ho)
        assert not (got == cpht.FULL).any(), f"batch {b}: FULL below load 0.9 (load {S.size / cap:.3f})"
        ok, msg = sets.check_insert_outcomes(S, hk[ins_m], got[ins_m])
        assert ok, f"batch {b}: {msg}"
        fixed = (~ins_m) & ~racy
        bad = np.nonzero(got[fixed] != seq[fixed])[0]
        assert bad.size == 0, f"batch {b}: {bad.size} fixed find answers differ"
        assert np.isin(got[racy], [0, 1]).all()
        racy_total += int(racy.sum())
        S = S_after
        b += 1
    print(f"zipf stream: {b} batches, load {S.size / cap:.4f}, {racy_total} racy finds", flush=True)
    assert t.count()[0] == S.size
    assert np.array_equal(check_table(t), S)
    # the hottest key (rank 1) is stored, and lookups agree with the set
    hot = synth.feistel(w, 0x2F1F, torch.zeros(1, dtype=torch.int64))
    assert int(t.find(synth.to_words(hot, w).to(gpu)).item()) == 1
    probe = synth.zipf_keys(w, 0x2F1F, 1.1, 1 << 18, 99999, device=gpu)
    assert np.array_equal(t.find(synth.to_words(probe, w)).cpu().numpy(), sets.find(S, host_u64(probe)))
