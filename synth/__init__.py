"""Seeded synthetic workloads for the hash-table benchmarks and tests.

This module only draws inputs: key streams, query mixes and operation codes.
It holds none of the hash tables' own arithmetic (no table permutation, no
slot encoding), so the GPU library and the CPU oracle can both be fed from it
without sharing any of the method.

Keys are produced as phi(0), phi(1), ... where phi is a 4-round Feistel
bijection on w-bit strings with a splitmix64 round function (Vigna's
published mixer) and its own seed, so a prefix of the sequence is a set of
distinct keys by construction and phi(i) for i >= n is guaranteed absent from
phi(0..n-1).  Everything is plain torch integer arithmetic on int64 tensors
(two's-complement wrap-around for the 64-bit products, masked shifts for the
logical right shifts), so it runs on the host or on the device.
"""
from __future__ import annotations

import torch

_M64 = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15
_C1 = 0xBF58476D1CE4E5B9
_C2 = 0x94D049BB133111EB


def _s64(v: int) -> int:
    """Two's-complement int64 value of a 64-bit pattern."""
    v &= _M64
    return v - (1 << 64) if v >= (1 << 63) else v


def _lsr(x: torch.Tensor, s: int) -> torch.Tensor:
    """Logical right shift of int64 lanes holding 64-bit patterns."""
    if s == 0:
        return x
    return (x >> s) & ((1 << (64 - s)) - 1)


def _mask(w: int) -> int:
    return _s64((1 << w) - 1) if w < 64 else -1


def mix64_t(z: torch.Tensor) -> torch.Tensor:
    """splitmix64 output function on int64 lanes."""
    z = (z ^ _lsr(z, 30)) * _s64(_C1)
    z = (z ^ _lsr(z, 27)) * _s64(_C2)
    return z ^ _lsr(z, 31)


def sm64(seed: int, i: int) -> int:
    """(i+1)-th output of splitmix64 started at `seed` (host integers)."""
    z = (seed + (i + 1) * _GAMMA) & _M64
    z = ((z ^ (z >> 30)) * _C1) & _M64
    z = ((z ^ (z >> 27)) * _C2) & _M64
    return z ^ (z >> 31)


def feistel(w: int, seed: int, x: torch.Tensor) -> torch.Tensor:
    """phi_seed(x) on w-bit strings (1 <= w <= 64), x an int64 tensor.

    Halves of a = ceil(w/2) and b = floor(w/2) bits; each round maps (L, R) to
    (R, L ^ F(R)), which swaps the half widths, so after four rounds the
    widths are back to (a, b)."""
    if not 2 <= w <= 64:
        raise ValueError("w must be in 2..64")
    a, b = (w + 1) // 2, w // 2
    L = _lsr(x, b) & _mask(a)
    R = x & _mask(b)
    wl, wr = a, b
    for rnd in range(4):
        k = _s64(sm64(seed, rnd))
        F = mix64_t(R + k) & _mask(wl)
        L, R = R, L ^ F
        wl, wr = wr, wl
    out = (L << wr) | R
    return out & _mask(w) if w < 64 else out


def distinct_keys(w: int, seed: int, start: int, count: int, device="cpu") -> torch.Tensor:
    """phi(start), ..., phi(start+count-1): distinct w-bit keys as int64."""
    idx = torch.arange(start, start + count, dtype=torch.int64, device=device)
    return feistel(w, seed, idx)


def _rand_u64(seed: int, start: int, count: int, device) -> torch.Tensor:
    """Counter-based uniform 64-bit draws: mix64(seed' + i*gamma)."""
    idx = torch.arange(start, start + count, dtype=torch.int64, device=device)
    base = _s64(sm64(seed, 0))
    return mix64_t(base + idx * _s64(_GAMMA))


def uniform_below(seed: int, count: int, bound: int, device="cpu") -> torch.Tensor:
    """count draws uniform in [0, bound) (bound < 2^31; bias below 2^-32)."""
    r = _lsr(_rand_u64(seed, 0, count, device), 32)
    return (r * bound) >> 32


def permutation(seed: int, count: int, device="cpu") -> torch.Tensor:
    """A seeded random permutation of 0..count-1 (sort of random 64-bit tags)."""
    tags = _rand_u64(seed ^ 0x5EED, 0, count, device)
    return torch.argsort(tags)


def find_queries(w: int, key_seed: int, n_inserted: int, n_queries: int, hit_frac: float,
                 qseed: int, device="cpu") -> torch.Tensor:
    """Query keys: round(hit_frac*n_queries) hits drawn uniformly (with
    replacement) from phi(0..n_inserted-1), the rest misses phi(n_inserted+j),
    all shuffled."""
    n_hit = int(round(hit_frac * n_queries)) if n_inserted > 0 else 0
    n_miss = n_queries - n_hit
    hit_idx = uniform_below(qseed, n_hit, max(1, n_inserted), device)
    miss_idx = torch.arange(n_inserted, n_inserted + n_miss, dtype=torch.int64, device=device)
    idx = torch.cat([hit_idx, miss_idx])
    idx = idx[permutation(qseed + 1, n_queries, device)]
    return feistel(w, key_seed, idx)


def insert_stream_with_duplicates(w: int, key_seed: int, fresh_start: int, n_ops: int,
                                  dup_frac: float, seed: int, device="cpu", return_index: bool = False):
    """Insert keys where a dup_frac share repeats keys issued earlier.

    Returns (keys, n_fresh): fresh keys are phi(fresh_start + i) in order; each
    duplicate copies a uniformly chosen earlier key of the stream (or of the
    keys issued before it: phi(0..fresh_start-1)).  With return_index, also
    the index of every key (keys = phi(index))."""
    r = _lsr(_rand_u64(seed, 0, n_ops, device), 11)  # 53 random bits
    is_dup = r < int(dup_frac * (1 << 53))
    if fresh_start == 0 and n_ops > 0:
        is_dup[0] = False
    fresh_rank = torch.cumsum((~is_dup).to(torch.int64), 0) - 1  # index of fresh key at or before
    n_fresh = int((~is_dup).sum().item())
    pool = fresh_start + fresh_rank + 1  # keys phi(0..pool-1) exist before op i (for dups)
    pick = (_lsr(_rand_u64(seed + 7, 0, n_ops, device), 32) * pool) >> 32
    idx = torch.where(is_dup, pick, fresh_start + fresh_rank)
    if return_index:
        return feistel(w, key_seed, idx), n_fresh, idx
    return feistel(w, key_seed, idx), n_fresh


MISS_BASE = 1 << 33  # mixed_batches: finds that miss use phi(MISS_BASE + j)


def mixed_batches(w: int, key_seed: int, capacity: int, load: float, batch: int, device="cpu"):
    """The dynamic-operation stream: mixed batches of `batch` operations, half
    find-or-puts and half finds in a seeded random order, run from an empty
    table to `load` * capacity distinct keys.

    Inserts: one stream over all batches in which 70 % of the operations are
    fresh keys phi(0), phi(1), ... in order and 30 % repeat a uniformly chosen
    earlier key of the stream.  Finds of batch b: with probability 1/2 a key
    phi(j) with j uniform below b * (fresh keys per batch expected), else a
    key phi(MISS_BASE + j) that is never inserted (none in batch 0).

    Returns (keys, ops, idx, n_fresh): keys [nb, batch] int64, ops [nb, batch]
    uint8 (1 = find-or-put, 0 = find), idx [nb, batch] int64 with keys =
    phi(idx), and the number of distinct keys inserted."""
    half = batch // 2
    fresh_per_batch = int(0.7 * half)
    nb = int(load * capacity) // fresh_per_batch
    ins, n_fresh, ins_idx = insert_stream_with_duplicates(w, key_seed, 0, nb * half, 0.3, 11, device=device,
                                                          return_index=True)
    g = uniform_below(13, nb * half, 1 << 30, device)
    issued_before = torch.arange(nb, device=device) * fresh_per_batch  # expected fresh keys before batch b
    hit_idx = (g.view(nb, half) * issued_before.clamp(min=1).view(nb, 1)) >> 30
    miss_idx = MISS_BASE + torch.arange(nb * half, dtype=torch.int64, device=device).view(nb, half)
    is_hit = (uniform_below(17, nb * half, 2, device).view(nb, half) == 1) & (issued_before.view(nb, 1) > 0)
    find_idx = torch.where(is_hit, hit_idx, miss_idx)
    del g, hit_idx, miss_idx, is_hit
    idx = torch.cat([ins_idx.view(nb, half), find_idx], dim=1)
    del ins, ins_idx, find_idx
    ops = torch.cat([torch.ones(nb, half, dtype=torch.uint8, device=device),
                     torch.zeros(nb, half, dtype=torch.uint8, device=device)], dim=1)
    perm = torch.stack([permutation(100 + b, batch, device) for b in range(min(nb, 8))])
    order = perm[torch.arange(nb, device=device) % perm.shape[0]]
    idx = torch.gather(idx, 1, order).contiguous()
    ops = torch.gather(ops, 1, order).contiguous()
    del order, perm
    keys = feistel(w, key_seed, idx)
    return keys, ops, idx, n_fresh


def find_or_put_batch(w: int, key_seed: int, n_before: int, n_new: int, n_ops: int, seed: int, device="cpu"):
    """A find-or-put batch over a table holding phi(0 .. n_before-1): every
    fresh key phi(n_before + j), j < n_new, occurs at least once, and the
    other n_ops - n_new operations repeat keys drawn uniformly (with
    replacement) from phi(0 .. n_before + n_new - 1), stored and fresh alike;
    all in a seeded random order.  Returns (keys, idx) with keys = phi(idx)."""
    if n_ops < n_new:
        raise ValueError("n_ops must cover every fresh key")
    fresh = torch.arange(n_before, n_before + n_new, dtype=torch.int64, device=device)
    extra = uniform_below(seed, n_ops - n_new, max(1, n_before + n_new), device)
    idx = torch.cat([fresh, extra])[permutation(seed + 1, n_ops, device)]
    return feistel(w, key_seed, idx), idx


def zipf_ranks(s: float, n: int, count: int, seed: int, device="cpu") -> torch.Tensor:
    """count i.i.d. draws from Zipf(s) on {1, ..., n} (P(k) proportional to
    k^-s, s > 0, s != 1), by rejection-inversion (W. Hormann and G. Derflinger,
    "Rejection-inversion to generate variates from monotone discrete
    distributions", ACM TOMACS 6(3), 1996): invert the integral H of the
    continuous hat x^-s over [k - 1/2, k + 1/2] and accept k unless the draw
    falls in the gap between hat and histogram.  float64 arithmetic; the
    uniform draws are counter-based (splitmix64 of seed and draw index)."""
    if s <= 0 or s == 1.0:
        raise ValueError("s must be positive and != 1")
    f64 = torch.float64
    q = 1.0 - s

    def H(x):  # integral of t^-s from 1 to x
        return torch.expm1(q * torch.log(x)) / q

    def Hinv(y):
        return torch.exp(torch.log1p(q * y) / q)

    def h(x):
        return torch.exp(-s * torch.log(x))

    one = torch.tensor(1.0, dtype=f64, device=device)
    hx1 = float(H(one * 1.5) - 1.0)
    hn = float(H(one * (n + 0.5)))
    sconst = float(2.0 - Hinv(H(one * 2.5) - h(one * 2.0)))
    out = torch.zeros(count, dtype=torch.int64, device=device)
    todo = torch.arange(count, device=device)
    rnd = 0
    while todo.numel():
        u01 = (_lsr(_rand_u64(seed + 0x1000 * rnd, 0, count, device)[todo], 11)).to(f64) * (1.0 / (1 << 53))
        u = hn + u01 * (hx1 - hn)
        x = Hinv(u)
        k = torch.clamp(torch.floor(x + 0.5), 1, n)
        ok = (k - x <= sconst) | (u >= H(k + 0.5) - h(k))
        out[todo[ok]] = k[ok].to(torch.int64)
        todo = todo[~ok]
        rnd += 1
    return out


def zipf_keys(w: int, key_seed: int, s: float, count: int, seed: int, device="cpu") -> torch.Tensor:
    """Zipf(s) draws over ranks 1..2^w mapped to w-bit keys by the Feistel
    bijection: key = phi(rank - 1)."""
    return feistel(w, key_seed, zipf_ranks(s, 1 << w, count, seed, device) - 1)


def to_words(keys: torch.Tensor, w: int) -> torch.Tensor:
    """Key words as stored for the library: int32 lanes (bit pattern of a
    uint32) when w <= 32, int64 lanes otherwise."""
    if w <= 32:
        return (keys & 0xFFFFFFFF).to(torch.int32) if keys.dtype != torch.int32 else keys
    return keys


def from_words(words: torch.Tensor) -> torch.Tensor:
    """Inverse of to_words: int64 lanes holding the unsigned key values."""
    if words.dtype == torch.int32:
        return words.to(torch.int64) & 0xFFFFFFFF
    return words
