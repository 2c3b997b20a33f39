"""Autotuner: pick the kernel variant (sub-tile width, slot width, buckets per
cache line) for a table shape by measuring the compiled candidates.

For a shape (scheme, key bits, slot count, target load) every compiled
variant whose key word size matches and whose stored remainder fits the slot
is built at that shape, filled to the target load with random keys, and
queried with twice its capacity in finds (half of them hits); variants that
answer FULL below the target load are discarded and the fastest of the rest
(insert time + find time, HIP events on the launch stream) wins.  Results are
cached per shape in memory and optionally in a JSON file.
"""
from __future__ import annotations

import json
import os

import torch

from . import CUCKOO, FULL, ICEBERG, Config, Table, check_config, default_config, variants

_CACHE: dict[str, dict] = {}


def _key(scheme, key_bits, log2_slots0, load):
    return f"{scheme}:{key_bits}:{log2_slots0}:{load:.3f}"


def load_cache(path: str) -> None:
    if os.path.exists(path):
        with open(path) as f:
            _CACHE.update(json.load(f))


def save_cache(path: str) -> None:
    with open(path, "w") as f:
        json.dump(_CACHE, f, indent=1, sort_keys=True)


def candidates(scheme: int, key_bits: int, log2_slots0: int, max_bucket_bytes: int = 128) -> list[Config]:
    """Feasible configurations at this shape, one per compiled variant."""
    out = []
    key64 = int(key_bits > 32)
    for v in variants(scheme):
        if v["key64"] != key64:
            continue
        if v["bucket0"] * v["slot_bits0"] // 8 > max_bucket_bytes:
            continue
        c = default_config(scheme)
        c.key_bits = key_bits
        c.log2_slots0 = log2_slots0
        c.bucket0, c.slot_bits0, c.subtile = v["bucket0"], v["slot_bits0"], v["subtile"]
        if scheme == ICEBERG:
            c.log2_slots1 = log2_slots0 - 3
            c.bucket1, c.slot_bits1 = v["bucket1"], v["slot_bits1"]
            if c.slot_bits1 < c.slot_bits0:
                continue
        if (1 << log2_slots0) < c.bucket0 or (scheme == ICEBERG and (1 << c.log2_slots1) < c.bucket1):
            continue
        if check_config(c) is not None:
            out.append(c)
    return out


def _random_keys(n: int, key_bits: int, gen: torch.Generator, device) -> torch.Tensor:
    """n distinct keys of key_bits bits (n <= 2^key_bits) as the library's key
    words, drawn on `device`: a random start and odd stride modulo 2^key_bits
    (a bijection of the index), so a cuckoo build gets the distinct keys its
    contract asks for; the table's own permutation spreads them over buckets."""
    w = min(key_bits, 63)
    mask = (1 << w) - 1
    start = int(torch.randint(0, 1 << 62, (1,), generator=gen, device=gen.device).item()) & mask
    stride = (int(torch.randint(0, 1 << 62, (1,), generator=gen, device=gen.device).item()) & mask) | 1
    i = torch.arange(n, dtype=torch.int64, device=device)
    k = (start + i * stride) & mask  # wraps mod 2^64 before the mask: still i -> k is a bijection mod 2^w
    if key_bits <= 32:
        return (k & 0xFFFFFFFF).to(torch.int32)
    return k


def pick(entries: list[tuple[float | None, float, bool]], tie: float = 0.03) -> int:
    """Index of the winner among (time or None if the candidate failed, bits
    per slot, is the preferred variant): the failed are dropped, candidates
    within `tie` of the fastest count as equally fast, and among those the
    least memory wins, then the preferred one, then the faster."""
    ok = [i for i, (ms, _, _) in enumerate(entries) if ms is not None]
    if not ok:
        raise RuntimeError("no candidate reaches the target load")
    fastest = min(entries[i][0] for i in ok)
    near = [i for i in ok if entries[i][0] <= fastest * (1 + tie)]
    return min(near, key=lambda i: (entries[i][1], not entries[i][2], entries[i][0]))


def _gen(device, seed: int) -> torch.Generator:
    return torch.Generator(device=device).manual_seed(seed)


def measure(c: Config, load: float, device, reps: int = 2, seed: int = 1, headroom: float = 0.05) -> dict | None:
    """Insert + find time of one configuration at `load`.  None if a fill to
    load + headroom (capped at 0.99) answers FULL: a variant must keep a
    margin over the target load, since other key sets fill it differently."""
    t = Table(c)
    cap = (1 << c.log2_slots0) + ((1 << c.log2_slots1) if c.scheme == ICEBERG else 0)
    n = int(load * cap)
    gen = _gen(device, seed)
    probe = _random_keys(int(min(0.99, load + headroom) * cap), c.key_bits, gen, device)
    pout = t.insert(probe)
    if int((pout == FULL).sum().item()):
        t.close()
        return None
    keys = _random_keys(n, c.key_bits, gen, device)
    miss = _random_keys(cap, c.key_bits, gen, device)
    q = torch.cat([keys[torch.randint(0, max(1, n), (cap,), generator=gen, device=gen.device)], miss])
    out = torch.empty(n, dtype=torch.uint8, device=device)
    found = torch.empty(q.numel(), dtype=torch.uint8, device=device)
    ti, tf = [], []
    for r in range(reps + 1):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        t.clear(seed + r)
        e[0].record()
        t.insert(keys, out)
        e[1].record()
        t.find(q, found)
        e[2].record()
        e[2].synchronize()
        if int((out == FULL).sum().item()):
            t.close()
            return None
        if r:
            ti.append(e[0].elapsed_time(e[1]))
            tf.append(e[1].elapsed_time(e[2]))
    t.close()
    return {"insert_ms": min(ti), "find_ms": min(tf), "total_ms": min(ti) + min(tf)}


def _bits_per_slot(c: Config) -> float:
    if c.scheme == ICEBERG:
        n0, n1 = 1 << c.log2_slots0, 1 << c.log2_slots1
        return (n0 * c.slot_bits0 + n1 * c.slot_bits1) / (n0 + n1)
    return float(c.slot_bits0)


def tune(scheme: int, key_bits: int, log2_slots0: int, load: float, device="cuda", reps: int = 3,
         tie: float = 0.03, prefer: Config | None = None) -> Config:
    """Best configuration for the shape (cached).  Candidates within `tie` of
    the fastest count as equally fast; among them the one using the least
    memory wins, then the one equal to `prefer` (so neighbouring size classes
    share a kernel variant and a table set needs fewer launches)."""
    k = _key(scheme, key_bits, log2_slots0, load)
    if k not in _CACHE:
        cands, entries, tried = candidates(scheme, key_bits, log2_slots0), [], []

        def same(c):
            return prefer is not None and all(
                getattr(c, f) == getattr(prefer, f) for f in ("bucket0", "slot_bits0", "slot_bits1", "subtile"))

        for c in cands:
            m = measure(c, load, device, reps)
            ms = None if m is None else m["total_ms"]
            tried.append({"bucket0": c.bucket0, "slot_bits0": c.slot_bits0, "slot_bits1": c.slot_bits1,
                          "subtile": c.subtile, "ms": None if ms is None else round(ms, 4)})
            entries.append((ms, _bits_per_slot(c), same(c)))
        try:
            w = pick(entries, tie)
        except RuntimeError:
            raise RuntimeError(f"no configuration reaches load {load} at 2^{log2_slots0} slots") from None
        _CACHE[k] = {"config": cands[w].as_dict(), "ms": entries[w][0], "tried": tried}
    c = Config()
    for name, v in _CACHE[k]["config"].items():
        setattr(c, name, v)
    return c


def tune_set(scheme: int, key_bits: int, log2_sizes: list[int], load: float, device="cuda", reps: int = 2,
             tie: float = 0.03, full_tol: float = 1e-6, seed: int = 3) -> tuple[dict, list[dict]]:
    """Pick one kernel variant for a whole table set by timing the set itself.

    Every table i gets 2^log2_sizes[i] primary slots (plus 1/8 secondary for
    iceberg).  Each candidate variant feasible at the smallest size (hence at
    all sizes: the remainder only shrinks as tables grow) is applied to every
    table; the set is filled to `load` and queried with twice its capacity
    (half hits) in one table-set launch each, as it will run.  Candidates whose
    FULL answers exceed full_tol of the inserts are discarded; the fastest wins,
    results within `tie` going to the smaller memory footprint.  Returns the
    chosen variant fields and the per-candidate timings."""
    from . import MultiTable

    smallest = min(log2_sizes)
    cands = candidates(scheme, key_bits, smallest)
    gen = _gen(device, seed)
    caps = [(1 << e) + ((1 << (e - 3)) if scheme == ICEBERG else 0) for e in log2_sizes]
    n_t = [int(load * c) for c in caps]
    keys = _random_keys(sum(n_t), key_bits, gen, device)
    ko = torch.tensor([0] + list(torch.tensor(n_t).cumsum(0).tolist()), dtype=torch.int64, device=device)
    q_t = [2 * c for c in caps]
    qo = torch.tensor([0] + list(torch.tensor(q_t).cumsum(0).tolist()), dtype=torch.int64, device=device)
    tid = torch.repeat_interleave(torch.arange(len(caps)), torch.tensor(q_t)).to(device)
    ntd = torch.tensor(n_t, dtype=torch.int64, device=device)
    hit_at = ko[:-1][tid] + (torch.rand(tid.numel(), generator=gen, device=gen.device) * ntd[tid]).long()
    hits = torch.rand(tid.numel(), generator=gen, device=gen.device) < 0.5
    queries = torch.where(hits, keys[hit_at.clamp(max=keys.numel() - 1)],
                          _random_keys(tid.numel(), key_bits, gen, device))
    out = torch.empty(keys.numel(), dtype=torch.uint8, device=device)
    found = torch.empty(queries.numel(), dtype=torch.uint8, device=device)
    rows = []
    for c in cands:
        cfgs = []
        for i, e in enumerate(log2_sizes):
            ci = Config()
            ctypes_copy(ci, c)
            ci.log2_slots0 = e
            if scheme == ICEBERG:
                ci.log2_slots1 = e - 3
            ci.seed = 100 + i
            cfgs.append(ci)
        m = MultiTable(cfgs, max_keys=max(keys.numel(), queries.numel()))
        times = []
        nfull = 0
        for r in range(reps + 1):
            m.clear()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            m.insert(keys, ko, out)
            m.find(queries, qo, found)
            b.record()
            b.synchronize()
            nfull = int((out == FULL).sum().item())
            if r:
                times.append(a.elapsed_time(b))
        m.close()
        ok = nfull <= full_tol * keys.numel()
        rows.append({"bucket0": c.bucket0, "slot_bits0": c.slot_bits0, "slot_bits1": c.slot_bits1,
                     "subtile": c.subtile, "ms": round(min(times), 3), "full": nfull, "ok": ok,
                     "bits_per_slot": _bits_per_slot(c)})
    try:
        w = pick([(r["ms"] if r["ok"] else None, r["bits_per_slot"], False) for r in rows], tie)
    except RuntimeError:
        raise RuntimeError("no variant reaches the target load for the set") from None
    best = rows[w]
    return {k: best[k] for k in ("bucket0", "slot_bits0", "slot_bits1", "subtile")}, rows


def ctypes_copy(dst: Config, src: Config) -> None:
    for name, _ in Config._fields_:
        setattr(dst, name, getattr(src, name))


def report(scheme: int, key_bits: int, log2_slots0: int, load: float) -> dict | None:
    return _CACHE.get(_key(scheme, key_bits, log2_slots0, load))


__all__ = ["candidates", "measure", "pick", "tune", "tune_set", "report", "load_cache", "save_cache", "CUCKOO", "ICEBERG"]
