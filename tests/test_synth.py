"""The seeded input generators: distinct keys by construction, the torch
int64 arithmetic agreeing with exact unsigned arithmetic, and the advertised
mixes of hits, misses and duplicates."""
import numpy as np
import pytest
import torch

import synth

M64 = (1 << 64) - 1


def _mix_ref(z: int) -> int:
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def test_mix64_matches_exact_unsigned_arithmetic():
    r = np.random.default_rng(0)
    vals = [int(v) for v in r.integers(-(2**63), 2**63 - 1, size=2000, dtype=np.int64)]
    got = synth.mix64_t(torch.tensor(vals, dtype=torch.int64)).tolist()
    assert [g & M64 for g in got] == [_mix_ref(v & M64) for v in vals]


def test_splitmix_first_output_seed0():
    assert synth.sm64(0, 0) == 0xE220A8397B1DCDAF


@pytest.mark.parametrize("w", [2, 3, 9, 16, 21])
def test_feistel_is_a_bijection(w):
    k = synth.distinct_keys(w, 77, 0, 1 << w)
    assert torch.unique(k).numel() == 1 << w
    assert int(k.min()) >= 0 and int(k.max()) < (1 << w)


@pytest.mark.parametrize("w", [32, 34, 37, 40, 64])
def test_distinct_keys_wide(w):
    k = synth.distinct_keys(w, 3, 1000, 200000)
    assert torch.unique(k).numel() == 200000
    if w < 64:
        assert int(k.min()) >= 0 and int(k.max()) < (1 << w)


def test_queries_hits_and_misses():
    w, n = 34, 5000
    ins = set(synth.distinct_keys(w, 5, 0, n).tolist())
    q = synth.find_queries(w, 5, n, 10000, 0.5, 9).tolist()
    hits = sum(x in ins for x in q)
    assert hits == 5000


def test_duplicate_stream():
    keys, n_fresh = synth.insert_stream_with_duplicates(34, 5, 0, 100000, 0.3, 1)
    u = torch.unique(keys).numel()
    assert u == n_fresh
    assert abs(n_fresh / 100000 - 0.7) < 0.01
    # every duplicate repeats a key issued before it
    seen = set()
    for k in keys.tolist()[:20000]:
        seen.add(k)
    assert len(seen) <= 20000


def test_word_conversion_round_trip():
    k = synth.distinct_keys(32, 1, 0, 100000)
    wds = synth.to_words(k, 32)
    assert wds.dtype == torch.int32
    assert torch.equal(synth.from_words(wds), k)


@pytest.mark.parametrize("s,n", [(1.1, 100), (1.5, 1000), (0.8, 50)])
def test_zipf_matches_exact_pmf(s, n):
    """Chi-square of 400k draws against the exact pmf k^-s / sum_j j^-s."""
    draws = synth.zipf_ranks(s, n, 400000, 17)
    assert int(draws.min()) >= 1 and int(draws.max()) <= n
    counts = torch.bincount(draws, minlength=n + 1)[1:].double().numpy()
    k = np.arange(1, n + 1, dtype=np.float64)
    p = k ** -s / (k ** -s).sum()
    exp = p * draws.numel()
    keep = exp >= 5
    chi2 = (((counts - exp) ** 2) / exp)[keep].sum() + 0.0
    dof = keep.sum() - 1
    assert abs(chi2 - dof) < 6 * np.sqrt(2 * dof), (chi2, dof)


def test_zipf_head_share_large_domain():
    """Over 2^34 ranks with s = 1.1 the top rank holds 1/zeta-like share:
    P(1) = 1 / sum_{k<=2^34} k^-1.1 (about 0.104)."""
    draws = synth.zipf_ranks(1.1, 1 << 34, 200000, 3)
    share = float((draws == 1).double().mean())
    # sum_{k=1}^{N} k^-s ~ zeta(s) - N^(1-s)/(s-1) (Euler-Maclaurin, first terms)
    from scipy.special import zeta

    N = float(1 << 34)
    norm = zeta(1.1) - N ** (-0.1) / 0.1 + 0.5 * N ** -1.1
    assert abs(share - 1.0 / norm) < 0.004, share


def test_find_or_put_batch_structure():
    keys, idx = synth.find_or_put_batch(30, 7, 1000, 500, 4000, 3)
    assert keys.numel() == idx.numel() == 4000
    assert int(idx.min()) >= 0 and int(idx.max()) < 1500
    # every fresh index occurs, and the batch is a shuffle (fresh keys not all in front)
    assert torch.isin(torch.arange(1000, 1500), idx).all()
    assert not bool((idx[:500] >= 1000).all())
    assert torch.equal(keys, synth.feistel(30, 7, idx))
    k2, i2 = synth.find_or_put_batch(30, 7, 1000, 500, 4000, 3)
    assert torch.equal(i2, idx)
