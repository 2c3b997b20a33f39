"""Benchmark: static bulk build then finds on a compact cuckoo table at GPU scale.

Workload (one GPU): compact bucketed cuckoo hashing, H = 2 hash functions,
2^27 slots in 2^22 buckets of 32 x 32-bit slots (128-byte buckets), 37-bit
keys held in uint64 words.  One step = empty the table with a new permutation
seed, bulk-insert 0.9 * 2^27 distinct keys (load 0.9), then 2^26 finds with
50 % hits and 50 % misses.  The same step is also timed on the non-compact
("plain") table: the same kernels with 64-bit slots that store all 37 bits of
pi_j(k) (256-byte buckets).  Keys are synthetic, seeded, and already resident
in device memory when the timed region starts.

Prints one JSON line.  Extra fields: per-kernel Mops/s and p50/p99 batch
latency for insert and find, compact vs plain, a load sweep, the roofline of
the dominant kernel, and the sequential CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mops/s insert & find at load 0.9, compact vs plain; p50/p99 batch latency"
W_KEY = 37
LOG2_SLOTS = 27
BUCKET = 32
LOAD = 0.9
N_FIND = 1 << 26
KEY_SEED = 0xC2C2C2C2
Q_SEED = 0x51515151
HBM_PEAK_GBS = 8000.0
LINE = 128

# Bucket reads per operation counted by the sequential oracle model
# (oracle/lines_per_op.py at 2^22 slots, buckets of 32 slots, 50 % hit finds):
# cuckoo put rounds (one bucket read and one bucket write each) and find probes.
ROUNDS_PER_PUT = {0.5: 1.00002, 0.7: 1.00252, 0.8: 1.01291, 0.9: 1.05175, 0.95: 1.11011}
PROBES_PER_FIND = {0.5: 1.00014, 0.7: 1.01809, 0.8: 1.07518, 0.9: 1.22454, 0.95: 1.36303}
# Iceberg at load 0.9 (B0 = 32, B1 = 16; sequential oracle at 2^22 primary
# slots, 50 % hit finds): an insert reads its primary bucket and, with
# probability ICE_L2["put"], both secondary buckets; a find likewise with
# probability ICE_L2["find"] (put / find bucket reads 1.15165 / 1.62852).
ICE_L2 = {"put": 0.075824, "find": 0.314262}
KEY_BYTES = 8
RESULT_BYTES = 1
CAS_BYTES = 4  # the atomic of a put round moves one 32-bit slot (8 bytes for 64-bit slots)
SECTOR = 64  # write-back unit of a modified slot (measured: 67.0 B written per put at 1.05 rounds)

# HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE (scaled by the
# copy-kernel calibration factors 2.0 / 1.0), profiles/cuckoo_c2_hbm_bytes.md.
# Valid only for the kernel sources they were taken with (hash of KERNEL_SOURCES below).
TRAFFIC = {"csrc_sha": "d690d9abc3ada6cc", "cuckoo_put": 25332912320, "cuckoo_find": 11035491456}


# The sources the profiled cuckoo kernels are compiled from.
KERNEL_SOURCES = ("cpht_device.hpp", "cpht_cuckoo.hpp", "cpht_registry.hpp", "inst_cuckoo_u64.hip")

# Measured HBM bytes per operation (read + written, same calibration) of the
# iceberg kernels at the iceberg_static shape, profiles/iceberg_hbm_bytes.md;
# valid for the iceberg sources they were taken with.
ICE_TRAFFIC = {"src_sha": "e487985929bbc784", "insert_16_32": 222.9, "find_16_32": 214.3,
               "insert_64_64": 352.6, "find_64_64": 344.0}
ICE_SOURCES = ("cpht_device.hpp", "cpht_iceberg.hpp", "cpht_registry.hpp", "inst_iceberg_u64.hip")


def csrc_sha(sources=KERNEL_SOURCES) -> str:
    import hashlib

    h = hashlib.sha256()
    for name in sources:
        h.update(name.encode())
        with open(os.path.join(ROOT, "paper_2406_09255_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def put_bytes(load: float, bucket_lines: int, cas_bytes: int = CAS_BYTES) -> float:
    """Algorithmic bytes of one put: each round reads its bucket's 128-byte
    lines and performs one atomic on one slot; plus the key word read and the
    result byte written."""
    return ROUNDS_PER_PUT[load] * (bucket_lines * LINE + cas_bytes) + KEY_BYTES + RESULT_BYTES


def put_bytes_sector(load: float, bucket_lines: int) -> float:
    """The same put charged with what the memory system moves for its atomic:
    the 64-byte sector holding the claimed or swapped slot is written back."""
    return ROUNDS_PER_PUT[load] * (bucket_lines * LINE + SECTOR) + KEY_BYTES + RESULT_BYTES


def find_bytes(load: float, bucket_lines: int) -> float:
    return PROBES_PER_FIND[load] * bucket_lines * LINE + KEY_BYTES + RESULT_BYTES


def pct(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = min(len(xs) - 1, max(0, int(round(q / 100.0 * (len(xs) - 1)))))
    return xs[k]


class Runner:
    """Times build + find steps on one table with events on the launch stream."""

    def __init__(self, torch, cpht, table, keys, queries, n_ins):
        self.torch, self.cpht, self.t = torch, cpht, table
        self.keys, self.queries, self.n_ins = keys, queries, n_ins
        self.out = torch.empty(keys.numel(), dtype=torch.uint8, device=keys.device)
        self.found = torch.empty(queries.numel(), dtype=torch.uint8, device=keys.device)
        self.ev = []

    def step(self, seed: int, n_ins: int | None = None, record: bool = True):
        torch = self.torch
        n = self.n_ins if n_ins is None else n_ins
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        self.t.clear(seed)
        e[0].record()
        self.t.bulk_build(self.keys[:n], self.out)
        e[1].record()
        self.t.find(self.queries, self.found)
        e[2].record()
        if record:
            self.ev.append(e)

    def times_ms(self):
        self.torch.cuda.synchronize()
        ins = [a.elapsed_time(b) for a, b, _ in self.ev]
        fnd = [b.elapsed_time(c) for _, b, c in self.ev]
        self.ev = []
        return ins, fnd


# Optional sections of the JSON line (each has a --no-<name> switch or is
# picked with --only).
SECTIONS = ("plain", "equal", "cachefree", "window", "sweep", "servingsmall", "small", "iceberg", "fop", "delete", "level3", "map", "many",
            "serving", "ceilings", "cpu")
# Sections run only when named in --only (minutes of host time).
OPT_IN = ("cpu_full",)

# Fill factors of the paper's Put / Find benchmarks (Sec. 5.1).
SWEEP_LOADS = (0.5, 0.6, 0.7, 0.75, 0.8, 0.85, 0.9, 0.95)

# (slot bits, compact, slots per bucket) of the load sweep: compact 32-bit and
# plain 64-bit slots at 8, 16 and 32 slots per bucket.
SWEEP_SHAPES = ((32, 1, 32), (64, 0, 32), (32, 1, 16), (64, 0, 16), (32, 1, 8), (64, 0, 8))


def equal_memory(torch, cpht, keys, queries, n_ins, reps=5):
    """Equal memory, equal key count: the compact table gets 2^28 32-bit slots
    (1 GiB, the plain table's footprint) and the same 0.9 * 2^27 keys, so it
    runs at load 0.45 while the plain 2^27 x 64-bit table runs at 0.9."""
    L = LOG2_SLOTS + 1
    t = cpht.Table(scheme=cpht.CUCKOO, key_bits=W_KEY, log2_slots0=L, bucket0=BUCKET, slot_bits0=32,
                   n_hash=2, max_chain=256, compact=1, seed=1)
    r = Runner(torch, cpht, t, keys, queries, n_ins)
    for rep in range(reps + 1):
        r.step(seed=300 + rep, record=rep > 0)
    ins, fnd = r.times_ms()
    ok = int((r.out[:n_ins] == cpht.PUT).sum().item()) == n_ins
    res = {"config": (f"compact cuckoo 2^{L} slots x 32-bit ({t.level_bytes(0)} bytes) holding the same {n_ins} keys "
                      f"(load {n_ins / (1 << L):.3f}), 2^26 finds 50% hit"),
           "check": "ok" if ok else "FAILED", "table_bytes": t.level_bytes(0),
           "insert_mops": round(n_ins / (sum(ins) / len(ins) / 1000.0) / 1e6, 1),
           "find_mops": round(N_FIND / (sum(fnd) / len(fnd) / 1000.0) / 1e6, 1)}
    del t, r
    return res


def cache_free(torch, cpht, synth, dev, reps=3):
    """The headline step on tables far larger than the 256 MB Infinity Cache,
    so that bucket reads come from HBM: compact 2^30 x 32-bit slots and plain
    2^29 x 64-bit slots (4 GiB each), plus compact 2^29 (the plain table's
    slot count, 2 GiB), each built to load 0.9 with a new permutation seed
    per repetition, then 2^26 finds at 50 % hit."""
    rows = []
    for label, log2_slots, slot_bits, cmp_ in (("compact_4GiB", 30, 32, 1), ("plain_4GiB", 29, 64, 0),
                                               ("compact_2GiB", 29, 32, 1)):
        n = int(LOAD * (1 << log2_slots))
        keys = synth.distinct_keys(W_KEY, KEY_SEED, 0, n, device=dev)
        queries = synth.find_queries(W_KEY, KEY_SEED, n, N_FIND, 0.5, Q_SEED, device=dev)
        t = cpht.Table(scheme=cpht.CUCKOO, key_bits=W_KEY, log2_slots0=log2_slots, bucket0=BUCKET,
                       slot_bits0=slot_bits, n_hash=2, max_chain=256, compact=cmp_, seed=1)
        r = Runner(torch, cpht, t, keys, queries, n)
        for rep in range(reps + 1):
            r.step(seed=700 + rep, record=rep > 0)
        ins, fnd = r.times_ms()
        n_put = int((r.out == cpht.PUT).sum().item())
        hit = float(r.found.float().mean().item())
        occ, _ = t.count()
        ok = n_put == n and occ == n and abs(hit - 0.5) < 0.01
        ims, fms = sum(ins) / len(ins), sum(fnd) / len(fnd)
        lines = 1 if slot_bits == 32 else 2
        put_gbs = n * put_bytes(LOAD, lines, 4 if slot_bits == 32 else 8) / (ims / 1000.0) / 1e9
        find_gbs = N_FIND * find_bytes(LOAD, lines) / (fms / 1000.0) / 1e9
        rows.append({"table": label, "slots": 1 << log2_slots, "slot_bits": slot_bits, "compact": bool(cmp_),
                     "table_bytes": t.level_bytes(0), "inserts": n, "check": "ok" if ok else "FAILED",
                     "insert_mops": round(n / (ims / 1000.0) / 1e6, 1),
                     "find_mops": round(N_FIND / (fms / 1000.0) / 1e6, 1),
                     "insert_ms": round(ims, 3), "find_ms": round(fms, 3),
                     "put_hbm_frac": round(put_gbs / HBM_PEAK_GBS, 4),
                     "find_hbm_frac": round(find_gbs / HBM_PEAK_GBS, 4),
                     "find_line_reads_G_per_s": round(N_FIND * PROBES_PER_FIND[LOAD] * lines / (fms / 1000.0) / 1e9,
                                                      2)})
        del t, r, keys, queries
        torch.cuda.empty_cache()
    by = {r["table"]: r for r in rows}
    c, p = by["compact_4GiB"], by["plain_4GiB"]
    return {"rows": rows,
            "compact_vs_plain_equal_memory": {"insert": round(c["insert_mops"] / p["insert_mops"], 3),
                                              "find": round(c["find_mops"] / p["find_mops"], 3)},
            "compact_vs_plain_equal_slots": {
                "insert": round(by["compact_2GiB"]["insert_mops"] / p["insert_mops"], 3),
                "find": round(by["compact_2GiB"]["find_mops"] / p["find_mops"], 3)}}


def marginal_window(torch, cpht, keys, n_ins, lo=0.85, reps=5):
    """Insert throughput of the last window of the build: fill the compact
    table to load `lo` (untimed), then time inserting the keys that take it
    from `lo` to 0.9."""
    n_lo = int(lo * (1 << LOG2_SLOTS))
    t = cpht.Table(scheme=cpht.CUCKOO, key_bits=W_KEY, log2_slots0=LOG2_SLOTS, bucket0=BUCKET, slot_bits0=32,
                   n_hash=2, max_chain=256, compact=1, seed=1)
    out = torch.empty(n_ins - n_lo, dtype=torch.uint8, device=keys.device)
    times, ok = [], True
    for rep in range(reps + 1):
        t.clear(500 + rep)
        t.insert(keys[:n_lo])
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        t.insert(keys[n_lo:n_ins], out)
        b.record()
        b.synchronize()
        ok = ok and int((out == cpht.PUT).sum().item()) == out.numel()
        if rep:
            times.append(a.elapsed_time(b))
    del t
    return {"window": [lo, LOAD], "keys": n_ins - n_lo, "check": "ok" if ok else "FAILED",
            "insert_mops": round((n_ins - n_lo) / (sum(times) / len(times) / 1000.0) / 1e6, 1),
            "ms": round(sum(times) / len(times), 4)}


def find_or_put(torch, cpht, synth, dev, reps=3):
    """The find-or-put experiment: a table filled to a `before` load gets one
    find-or-put batch with as many keys as it has slots -- stored keys, fresh
    keys and repeats of both -- that fills it to exactly the `after` load.
    Iceberg (2^27 + 2^24 slots) runs its own find-or-put; cuckoo (2^27 slots)
    runs the sorted find-or-put (sort the batch, look each distinct key up
    once, put the missing ones).  37-bit keys; the timed region is the one
    call, keys resident; the table is rebuilt to `before` (untimed) each rep."""
    w, L = 37, 27
    shapes = [
        ("iceberg_16_32", dict(scheme=cpht.ICEBERG, key_bits=w, log2_slots0=L, log2_slots1=L - 3, bucket0=32,
                               bucket1=16, slot_bits0=16, slot_bits1=32, seed=5), ((0.0, 0.5), (0.5, 0.9), (0.8, 0.9))),
        ("iceberg_64_64", dict(scheme=cpht.ICEBERG, key_bits=w, log2_slots0=L, log2_slots1=L - 3, bucket0=32,
                               bucket1=16, slot_bits0=64, slot_bits1=64, compact=0, seed=5),
         ((0.0, 0.5), (0.5, 0.9))),
    ]
    # the smaller primary buckets of the paper's benchmark (they answer FULL
    # before load 0.9, so their batches end at 0.5 and 0.6)
    for b0 in (8, 16):
        for s0, s1 in ((16, 32), (64, 64)):
            shapes.append((f"iceberg_{s0}_{s1}_b{b0}",
                           dict(scheme=cpht.ICEBERG, key_bits=w, log2_slots0=L, log2_slots1=L - 3, bucket0=b0,
                                bucket1=b0 // 2, slot_bits0=s0, slot_bits1=s1, compact=int(s0 < 64), seed=5),
                           ((0.0, 0.5), (0.4, 0.6))))
    shapes += [
        ("cuckoo_32", dict(scheme=cpht.CUCKOO, key_bits=w, log2_slots0=L, bucket0=32, slot_bits0=32, seed=5),
         ((0.0, 0.5), (0.5, 0.9), (0.8, 0.9))),
        ("cuckoo_64", dict(scheme=cpht.CUCKOO, key_bits=w, log2_slots0=L, bucket0=32, slot_bits0=64, compact=0,
                           seed=5), ((0.5, 0.9),)),
    ]
    res = {"config": "find-or-put batch of #slots keys (stored + fresh, with repeats) taking the table from the "
                     "`before` to the `after` load; iceberg 2^27 + 2^24 slots, cuckoo 2^27 slots (sorted "
                     "find-or-put), 37-bit keys"}
    for name, kw, combos in shapes:
        t = cpht.Table(**kw)
        cap = t.count()[1]
        ws = None
        if kw["scheme"] == cpht.CUCKOO:
            ws = torch.empty(t.sorted_fop_workspace(cap), dtype=torch.uint8, device=dev)
        rows = []
        for before, after in combos:
            n_b, n_a = int(before * cap), int(after * cap)
            pre = synth.distinct_keys(w, KEY_SEED + 3, 0, n_b, device=dev)
            keys, idx = synth.find_or_put_batch(w, KEY_SEED + 3, n_b, n_a - n_b, cap, 41, device=dev)
            del idx
            out = torch.empty(cap, dtype=torch.uint8, device=dev)
            times, ok = [], True
            for rep in range(reps + 1):
                t.clear(60 + rep)
                if n_b:
                    t.insert(pre)
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                if ws is not None:
                    t.sorted_fop(keys, out, ws)
                else:
                    t.insert(keys, out)
                b.record()
                b.synchronize()
                ok = ok and int((out == cpht.PUT).sum().item()) == n_a - n_b and t.count()[0] == n_a
                if rep:
                    times.append(a.elapsed_time(b))
            ms = sum(times) / len(times)
            rows.append({"before": before, "after": after, "ops": cap, "ms": round(ms, 3),
                         "mops": round(cap / (ms / 1000.0) / 1e6, 1), "check": "ok" if ok else "FAILED"})
            del pre, keys, out
        res[name] = rows
        del t, ws
    m = {r["before"]: r["mops"] for r in res["iceberg_16_32"]}
    c = {r["before"]: r["mops"] for r in res["cuckoo_32"]}
    res["iceberg_vs_sorted_cuckoo"] = {str(k): round(m[k] / c[k], 2) for k in m if k in c}
    # 16/32-bit against 64/64-bit iceberg per primary bucket size, batch 0 -> 0.5
    def at(name, before):
        return next(r["mops"] for r in res[name] if r["before"] == before)
    res["iceberg_16_32_vs_64_64_load_0_to_0.5"] = {
        str(b0): round(at(f"iceberg_16_32{sfx}", 0.0) / at(f"iceberg_64_64{sfx}", 0.0), 3)
        for b0, sfx in ((8, "_b8"), (16, "_b16"), (32, ""))}
    return res


def deletes(torch, cpht, synth, dev, reps=3):
    """Delete by tombstone on the compact cuckoo (2^27 slots) and compact
    iceberg (2^27 + 2^24 slots, 16/32-bit) tables at load 0.9: one batch of
    2^26 deletes, half of them stored keys and half absent keys; the table is
    rebuilt (untimed) before each rep."""
    w, L, nd = 37, 27, 1 << 26
    res = {"config": "2^26 deletes (50% stored keys, 50% absent) on a table at load 0.9, 37-bit keys"}
    for name, kw in (("cuckoo_32", dict(scheme=cpht.CUCKOO, key_bits=w, log2_slots0=L, bucket0=32, slot_bits0=32,
                                        seed=9)),
                     ("iceberg_16_32", dict(scheme=cpht.ICEBERG, key_bits=w, log2_slots0=L, log2_slots1=L - 3,
                                            bucket0=32, bucket1=16, slot_bits0=16, slot_bits1=32, seed=9))):
        t = cpht.Table(**kw)
        cap = t.count()[1]
        n = int(0.9 * cap)
        keys = synth.distinct_keys(w, KEY_SEED + 5, 0, n, device=dev)
        # the hits must be distinct for an exact check: draw them as a prefix of a permutation
        hit_idx = synth.permutation(77, n, device=dev)[: nd // 2]
        q = torch.cat([keys[hit_idx], synth.distinct_keys(w, KEY_SEED + 5, n, nd // 2, device=dev)])
        q = q[synth.permutation(78, nd, device=dev)]
        out = torch.empty(nd, dtype=torch.uint8, device=dev)
        times, ok = [], True
        for rep in range(reps + 1):
            t.clear(90 + rep)
            t.insert(keys)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            t.delete(q, out)
            b.record()
            b.synchronize()
            ok = ok and int(out.sum().item()) == nd // 2 and t.count()[0] == n - nd // 2
            if rep:
                times.append(a.elapsed_time(b))
        ms = sum(times) / len(times)
        res[name] = {"ms": round(ms, 3), "mops": round(nd / (ms / 1000.0) / 1e6, 1), "check": "ok" if ok else "FAILED"}
        del t, keys, q, out
    return res


def level3(torch, cpht, synth, dev, reps=3):
    """Third iceberg level: compact 2^27 + 2^24 slots (16/32-bit), 37-bit keys,
    filled in one batch to load 1.0 of the bucket levels -- past the point
    where two levels answer FULL -- with and without a pool of 2^20 slabs
    (128 MiB) in 2^17 lists (one list per 32 primary buckets, so a list
    holds about one slab of overflow); then 2^26 finds (50 % hit).  Reports FULL answers,
    keys that went to the lists, and insert / find rates."""
    w, L = 37, 27
    res = {"config": "iceberg 2^27 + 2^24 slots (16/32-bit), 37-bit keys, one insert batch to load 1.0 of the "
                     "bucket levels, then 2^26 finds 50% hit; third level: 2^17 lists, pool of 2^20 slabs"}
    for name, extra in (("two_levels", {}), ("three_levels", dict(log2_lists=17, pool_slabs=1 << 20))):
        t = cpht.Table(scheme=cpht.ICEBERG, key_bits=w, log2_slots0=L, log2_slots1=L - 3, bucket0=32, bucket1=16,
                       slot_bits0=16, slot_bits1=32, seed=11, **extra)
        cap = t.count()[1]
        n = cap
        keys = synth.distinct_keys(w, KEY_SEED + 13, 0, n, device=dev)
        q = synth.find_queries(w, KEY_SEED + 13, n, N_FIND, 0.5, Q_SEED + 13, device=dev)
        out = torch.empty(n, dtype=torch.uint8, device=dev)
        found = torch.empty(N_FIND, dtype=torch.uint8, device=dev)
        ti, tf = [], []
        for rep in range(reps + 1):
            t.clear(70 + rep)
            e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            e[0].record()
            t.insert(keys, out)
            e[1].record()
            t.find(q, found)
            e[2].record()
            e[2].synchronize()
            if rep:
                ti.append(e[0].elapsed_time(e[1]))
                tf.append(e[1].elapsed_time(e[2]))
        nfull = int((out == cpht.FULL).sum().item())
        occ = t.count()[0]
        row = {"full": nfull, "stored": occ, "fill_of_bucket_levels": round(occ / cap, 4),
               "insert_mops": round(n / (sum(ti) / len(ti) / 1000.0) / 1e6, 1),
               "find_mops": round(N_FIND / (sum(tf) / len(tf) / 1000.0) / 1e6, 1),
               "hit_fraction": round(float(found.float().mean().item()), 4)}
        if extra:
            used = t.level3_used()
            row["slabs_used"] = used
            row["pool_bytes"] = t.level_bytes(2)
        res[name] = row
        del t, keys, q, out, found
    return res


def kv_map(torch, cpht, synth, dev, reps=3):
    """Key-value map on the iceberg table (values at the slot index of their
    key, 8 bytes each): 2^27 + 2^24 slots, 37-bit keys, insert to load 0.9
    in one batch then 2^26 lookups (50 % hit), compact 16/32-bit against
    plain 64/64-bit slots, beside the same workload as a set."""
    w, L = 37, 27
    res = {"config": "iceberg 2^27 + 2^24 slots, 37-bit keys, 8-byte values; insert to load 0.9 then 2^26 lookups "
                     "50% hit"}
    shapes = (("map_16_32", dict(slot_bits0=16, slot_bits1=32, value_bytes=8)),
              ("map_64_64", dict(slot_bits0=64, slot_bits1=64, compact=0, value_bytes=8)),
              ("set_16_32", dict(slot_bits0=16, slot_bits1=32)))
    for name, kw in shapes:
        t = cpht.Table(scheme=cpht.ICEBERG, key_bits=w, log2_slots0=L, log2_slots1=L - 3, bucket0=32, bucket1=16,
                       seed=12, **kw)
        cap = t.count()[1]
        n = int(0.9 * cap)
        keys = synth.distinct_keys(w, KEY_SEED + 17, 0, n, device=dev)
        vals = synth.mix64_t(keys)
        q = synth.find_queries(w, KEY_SEED + 17, n, N_FIND, 0.5, Q_SEED + 17, device=dev)
        out = torch.empty(n, dtype=torch.uint8, device=dev)
        found = torch.empty(N_FIND, dtype=torch.uint8, device=dev)
        vout = torch.zeros(N_FIND, dtype=torch.int64, device=dev)
        ti, tf = [], []
        for rep in range(reps + 1):
            t.clear(80 + rep)
            e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            e[0].record()
            if "value_bytes" in kw:
                t.insert_values(keys, vals, out)
            else:
                t.insert(keys, out)
            e[1].record()
            if "value_bytes" in kw:
                t.find_values(q, found, vout)
            else:
                t.find(q, found)
            e[2].record()
            e[2].synchronize()
            if rep:
                ti.append(e[0].elapsed_time(e[1]))
                tf.append(e[1].elapsed_time(e[2]))
        ok = int((out == cpht.PUT).sum().item()) == n and abs(float(found.float().mean().item()) - 0.5) < 0.01
        if "value_bytes" in kw:  # every value returned is the one inserted with its key
            hit = found.bool()
            ok = ok and torch.equal(vout[hit], synth.mix64_t(q[hit]))
        bytes_ = sum(t.level_bytes(x) for x in range(2))
        if "value_bytes" in kw:
            bytes_ += cap * 8
        res[name] = {"insert_mops": round(n / (sum(ti) / len(ti) / 1000.0) / 1e6, 1),
                     "find_mops": round(N_FIND / (sum(tf) / len(tf) / 1000.0) / 1e6, 1),
                     "bytes": bytes_, "check": "ok" if ok else "FAILED"}
        del t, keys, vals, q, out, found, vout
    res["compact_vs_plain_map"] = {
        "insert": round(res["map_16_32"]["insert_mops"] / res["map_64_64"]["insert_mops"], 3),
        "find": round(res["map_16_32"]["find_mops"] / res["map_64_64"]["find_mops"], 3),
        "memory": round(res["map_16_32"]["bytes"] / res["map_64_64"]["bytes"], 3)}
    return res


def _host_cpu() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(log2_slots: int = 26):
    """The sequential oracle on the host: same bucket shape, load and find mix,
    at 2^log2_slots slots (a bounded sample of the workload)."""
    import numpy as np
    import torch

    import oracle
    import synth

    n = int(LOAD * (1 << log2_slots))
    nq = 1 << (log2_slots - 1)
    keys = synth.distinct_keys(W_KEY, KEY_SEED, 0, n).numpy().astype(np.uint64)
    q = synth.find_queries(W_KEY, KEY_SEED, n, nq, 0.5, Q_SEED).numpy().astype(np.uint64)
    t = oracle.Table(oracle.CUCKOO, W_KEY, log2_slots, BUCKET, 32, seed=1)
    t0 = time.perf_counter()
    out = t.insert(keys)
    t1 = time.perf_counter()
    f = t.find(q)
    t2 = time.perf_counter()
    assert (out == oracle.PUT).all()
    del torch
    # context beside the sample: the small cuckoo shape whole, and a 1/16 sample
    # of the iceberg shape (compact 16/32, load 0.9, finds at 50 % hit)
    ks = synth.distinct_keys(32, KEY_SEED + 21, 0, 104857).numpy().astype(np.uint64)
    qs = synth.find_queries(32, KEY_SEED + 21, 104857, 100000, 0.5, Q_SEED + 21).numpy().astype(np.uint64)
    ts = oracle.Table(oracle.CUCKOO, 32, 17, 32, 32, seed=1)
    a = time.perf_counter()
    ts.insert(ks)
    b = time.perf_counter()
    ts.find(qs)
    c = time.perf_counter()
    small = {"insert_us": round((b - a) * 1e6, 1), "find_us": round((c - b) * 1e6, 1),
             "shape": "cuckoo 2^17 slots, 32 x 32-bit buckets, 32-bit keys: 104857 inserts, 10^5 finds"}
    ni, nqi = int(LOAD * ((1 << 23) + (1 << 20))), 1 << 22
    ki = synth.distinct_keys(33, KEY_SEED + 22, 0, ni).numpy().astype(np.uint64)
    qi = synth.find_queries(33, KEY_SEED + 22, ni, nqi, 0.5, Q_SEED + 22).numpy().astype(np.uint64)
    ti = oracle.Table(oracle.ICEBERG, 33, 23, 32, 16, log2_slots1=20, B1=16, s1=32, seed=5)
    a = time.perf_counter()
    ti.insert(ki)
    b = time.perf_counter()
    ti.find(qi)
    c = time.perf_counter()
    ice = {"insert_mops": round(ni / (b - a) / 1e6, 3), "find_mops": round(nqi / (c - b) / 1e6, 3),
           "shape": f"iceberg 2^23 + 2^20 slots (16/32-bit, 33-bit keys: at 1/16 of the iceberg benchmark's slots a "
                    f"16-bit primary slot holds 33-bit keys' remainders), "
                    f"{ni} inserts to load {LOAD}, {nqi} finds at 50% hit"}
    return {
        "value": round((n + nq) / (t2 - t0) / 1e6, 3),
        "unit": "Mops/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"sequential oracle, compact cuckoo 2^{log2_slots} slots (1/{1 << (LOG2_SLOTS - log2_slots)} "
                   f"of the workload's slots, same 32 x 32-bit buckets), build to load {LOAD} ({n} keys) "
                   f"then {nq} finds at 50% hit, one host thread"),
        "insert_mops": round(n / (t1 - t0) / 1e6, 3),
        "find_mops": round(nq / (t2 - t1) / 1e6, 3),
        "seconds": round(t2 - t0, 2),
        "hit_fraction": round(float(f.mean()), 4),
        "host_threads_available": os.cpu_count(),
        "host_cpu": _host_cpu(),
        "small_cuckoo": small,
        "iceberg_sample": ice,
    }


def cpu_full(torch, synth, dev, sweep=(0.5, 0.7, 0.8, 0.9, 0.95), batch=1 << 20):
    """The sequential oracle at full scale, timed once on one host thread
    (minutes of host time, so only on request):
      - the compact cuckoo benchmark table (2^27 slots, 32 x 32-bit buckets,
        37-bit keys) built from empty through every load of the sweep, the
        time to each load being the build's time up to it (the oracle is
        sequential, so this equals a separate build to that load), with 2^26
        finds at 50 % hit timed at each load;
      - the uniform dynamic-operation stream of the iceberg benchmark (2^28 +
        2^25 slots, 16/32-bit, 34-bit keys; the same batches as the GPU run)
        from load 0 to 0.9, batch by batch through the oracle's mixed call.
    Keys are generated on the device and copied to host memory outside the
    timed calls."""
    import numpy as np

    import oracle

    t_all = time.perf_counter()
    ck = oracle.Table(oracle.CUCKOO, W_KEY, LOG2_SLOTS, BUCKET, 32, seed=1)
    n_max = int(max(sweep) * (1 << LOG2_SLOTS))
    keys = synth.distinct_keys(W_KEY, KEY_SEED, 0, n_max, device=dev).cpu().numpy().astype(np.uint64)
    built, build_s, rows = 0, 0.0, {}
    for L in sweep:
        n = int(L * (1 << LOG2_SLOTS))
        a = time.perf_counter()
        out = ck.insert(keys[built:n])
        build_s += time.perf_counter() - a
        assert (out == oracle.PUT).all(), f"oracle cuckoo build failed below load {L}"
        built = n
        q = synth.find_queries(W_KEY, KEY_SEED, n, N_FIND, 0.5, Q_SEED, device=dev).cpu().numpy().astype(np.uint64)
        a = time.perf_counter()
        f = ck.find(q)
        fs = time.perf_counter() - a
        rows[str(L)] = {"inserts": n, "insert_s": round(build_s, 2), "insert_mops": round(n / build_s / 1e6, 3),
                        "finds": int(q.size), "find_s": round(fs, 2), "find_mops": round(q.size / fs / 1e6, 3),
                        "hit_fraction": round(float(f.mean()), 4)}
        print(f"[bench] cpu_full cuckoo load {L}: {rows[str(L)]}", file=sys.stderr, flush=True)
    del ck, keys
    w = 34
    L0, L1 = LOG2_SLOTS + 1, LOG2_SLOTS - 2
    cap = (1 << L0) + (1 << L1)
    mk, mo, _, n_fresh = synth.mixed_batches(w, KEY_SEED + 3, cap, LOAD, batch, device=dev)
    nb = mk.shape[0]
    ice = oracle.Table(oracle.ICEBERG, w, L0, 32, 16, log2_slots1=L1, B1=16, s1=32, seed=9)
    ms, nops, nfull = 0.0, 0, 0
    for b in range(nb):
        hk = mk[b].cpu().numpy().astype(np.uint64)
        ho = mo[b].cpu().numpy()
        a = time.perf_counter()
        out = ice.mixed(hk, ho)
        ms += (time.perf_counter() - a) * 1e3
        nops += hk.size
        nfull += int((out[ho == 1] == oracle.FULL).sum())
        if b % 100 == 99:
            print(f"[bench] cpu_full iceberg batch {b + 1}/{nb}: {nops / ms / 1e3:.2f} Mops/s", file=sys.stderr,
                  flush=True)
    occ, capo = ice.occupied(), ice.capacity()
    del mk, mo, ice
    many = _cpu_many_tables_sample(torch, synth, dev)
    print(f"[bench] cpu_full many tables: {many}", file=sys.stderr, flush=True)
    srv = _cpu_serving_sample(torch, synth, dev)
    print(f"[bench] cpu_full serving: {srv}", file=sys.stderr, flush=True)
    return {
        "kind": "oracle", "cores": 1, "host_threads_available": os.cpu_count(), "host_cpu": _host_cpu(),
        "cuckoo_load_sweep": rows,
        "cuckoo_shape": (f"compact cuckoo 2^{LOG2_SLOTS} slots, 32 x 32-bit buckets, {W_KEY}-bit keys; one build "
                         f"from empty, timed to each load; {N_FIND} finds (50% hit) at each load"),
        "iceberg_uniform_stream": {"ops": nops, "batches": nb, "ms": round(ms, 1),
                                   "mops": round(nops / ms / 1e3, 3), "full": nfull,
                                   "fill_factor": round(occ / capo, 4), "distinct_inserted": n_fresh,
                                   "count_matches": occ == n_fresh},
        "iceberg_shape": (f"iceberg 2^{L0} + 2^{L1} slots, B0=32 x 16-bit, B1=16 x 32-bit, {w}-bit keys; "
                          f"{nb} mixed batches of {batch} ops (the GPU run's batches), load 0 -> {LOAD}"),
        "many_tables_sample": many,
        "serving_sample": srv,
        "seconds": round(time.perf_counter() - t_all, 1),
    }


def _cpu_many_tables_sample(torch, synth, dev, n_tables=4096, n_sample=256, lo=10, hi=20, load=0.85):
    """The sequential oracle on the first n_sample tables of the many-table
    workload (the same size draw, 2^e + 2^(e-3) slots, 32-bit keys; buckets
    of 32 x 32-bit primary and 16 x 32-bit secondary slots): each filled to
    the load with distinct keys, then queried with twice its capacity in finds
    (half hits on its own keys, half misses)."""
    import numpy as np

    import oracle

    w = 32
    e_t = (synth.uniform_below(0xE5, n_tables, hi - lo + 1, dev) + lo).cpu().tolist()[:n_sample]
    rng = np.random.default_rng(0xAB)
    base, ins_s, find_s, n_ins, n_find, hits = 0, 0.0, 0.0, 0, 0, 0
    for i, e in enumerate(e_t):
        cap = (1 << e) + (1 << (e - 3))
        n, nq = int(cap * load), 2 * cap
        keys = synth.distinct_keys(w, KEY_SEED + 9, base, n).numpy().astype(np.uint64)
        miss = synth.distinct_keys(w, KEY_SEED + 9, (1 << 31) + base, nq).numpy().astype(np.uint64)
        base += n
        hit = rng.random(nq) < 0.5
        q = np.where(hit, keys[rng.integers(0, n, nq)], miss)
        tab = oracle.Table(oracle.ICEBERG, w, e, 32, 32, log2_slots1=e - 3, B1=16, s1=32, seed=7000 + i)
        a = time.perf_counter()
        out = tab.insert(keys)
        b = time.perf_counter()
        f = tab.find(q)
        c = time.perf_counter()
        assert (out == oracle.PUT).all() and np.array_equal(f.astype(bool), hit), f"oracle table {i}"
        ins_s, find_s = ins_s + (b - a), find_s + (c - b)
        n_ins, n_find, hits = n_ins + n, n_find + nq, hits + int(hit.sum())
        del tab
    return {"tables": n_sample, "of": n_tables, "inserts": n_ins, "finds": n_find,
            "insert_mops": round(n_ins / ins_s / 1e6, 3), "find_mops": round(n_find / find_s / 1e6, 3),
            "ops_mops": round((n_ins + n_find) / (ins_s + find_s) / 1e6, 3), "seconds": round(ins_s + find_s, 1)}


def _cpu_serving_sample(torch, synth, dev, log2_slots0=28, prefill=0.5, ops_max=1 << 25, seed=3):
    """The sequential oracle on the serving workload at 1/16 of the table
    (2^28 + 2^25 slots, 16/32-bit; the GPU table has 2^32 + 2^29 with 40-bit
    keys, and the key width shrinks with the table, to 36 bits, so that the
    stored remainders keep their width and fit the 16-bit slots):
    pre-filled to load 0.5, then the first requests of the same trace
    (lognormal sizes, 70 % finds at half hits, 30 % inserts of fresh keys)
    up to ops_max operations, applied in arrival order.  Every answer is
    checked."""
    import numpy as np

    import oracle

    L0, L1 = log2_slots0, log2_slots0 - 3
    w = 40 - (32 - L0)
    cap = (1 << L0) + (1 << L1)
    n_pre = int(prefill * cap)
    tab = oracle.Table(oracle.ICEBERG, w, L0, 32, 16, log2_slots1=L1, B1=16, s1=32, seed=23)
    pre_s = 0.0
    for a in range(0, n_pre, 1 << 24):
        k = synth.distinct_keys(w, KEY_SEED + 7, a, min(1 << 24, n_pre - a), device=dev).cpu().numpy()
        t0 = time.perf_counter()
        out = tab.insert(k.astype(np.uint64))
        pre_s += time.perf_counter() - t0
        assert (out == oracle.PUT).all()
    r = np.random.default_rng(seed)
    sizes = np.clip(np.round(np.exp(r.normal(np.log(4096), 2.0, 100000))), 1, 1 << 22).astype(np.int64)
    n_req = int(np.searchsorted(np.cumsum(sizes), ops_max, side="right"))
    total = int(sizes[:n_req].sum())
    is_ins = synth.uniform_below(0x31, total, 10, dev) < 3
    is_hit = synth.uniform_below(0x32, total, 2, dev) == 1
    fresh_idx = n_pre + torch.cumsum(is_ins.to(torch.int64), 0)
    hit_idx = synth.uniform_below(0x33, total, 1 << 30, dev) * n_pre >> 30
    miss_idx = (1 << (w - 1)) + torch.arange(total, device=dev)
    idx = torch.where(is_ins, fresh_idx, torch.where(is_hit, hit_idx, miss_idx))
    keys = synth.feistel(w, KEY_SEED + 7, idx).cpu().numpy().astype(np.uint64)
    ops = is_ins.to(torch.uint8).cpu().numpy()
    want = np.where(ops == 1, oracle.PUT, is_hit.cpu().numpy().astype(np.uint8)).astype(np.uint8)
    del is_ins, is_hit, fresh_idx, hit_idx, miss_idx, idx
    t0 = time.perf_counter()
    got = tab.mixed(keys, ops)
    run_s = time.perf_counter() - t0
    assert np.array_equal(got, want), "oracle serving sample"
    return {"table": f"2^{L0} + 2^{L1} slots (16/32-bit), {w}-bit keys, pre-filled to load {prefill}",
            "prefill_inserts": n_pre, "prefill_mops": round(n_pre / pre_s / 1e6, 3), "requests": n_req,
            "operations": total, "mops": round(total / run_s / 1e6, 3), "seconds": round(pre_s + run_s, 1)}


def small_cuckoo(torch, cpht, synth, dev, reps=20):
    """The small cuckoo shape: 2^17 slots in 2^12 buckets of 32 x 32-bit
    slots, 32-bit keys split into a 12-bit bucket and a 20-bit remainder plus
    the hash-index bit; bulk insert 104,857 keys (load 0.8), then 10^5 finds
    with 50 % hits.  The table (512 KiB) lives in cache, so this measures the
    latency of one small batch (launch included), not bandwidth."""
    w, L, n, nq = 32, 17, 104857, 100000
    t = cpht.Table(scheme=cpht.CUCKOO, key_bits=w, log2_slots0=L, bucket0=32, slot_bits0=32, seed=1)
    keys = synth.to_words(synth.distinct_keys(w, KEY_SEED + 11, 0, n, device=dev), w)
    q = synth.to_words(synth.find_queries(w, KEY_SEED + 11, n, nq, 0.5, Q_SEED, device=dev), w)
    out = torch.empty(n, dtype=torch.uint8, device=dev)
    found = torch.empty(nq, dtype=torch.uint8, device=dev)
    ins, fnd = [], []
    for r in range(reps + 2):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        t.clear(100 + r)
        e[0].record()
        t.bulk_build(keys, out)
        e[1].record()
        t.find(q, found)
        e[2].record()
        e[2].synchronize()
        if r >= 2:
            ins.append(e[0].elapsed_time(e[1]) * 1000)
            fnd.append(e[1].elapsed_time(e[2]) * 1000)
    ok = int((out == cpht.PUT).sum().item()) == n and abs(float(found.float().mean().item()) - 0.5) < 0.01
    return {"config": "cuckoo H=2, 2^17 slots in 2^12 buckets of 32 x 32-bit slots, 32-bit keys; insert 104857 "
                      "(load 0.8) then 10^5 finds 50% hit",
            "check": "ok" if ok else "FAILED",
            "insert_us": {"p50": round(pct(ins, 50), 2), "p99": round(pct(ins, 99), 2)},
            "find_us": {"p50": round(pct(fnd, 50), 2), "p99": round(pct(fnd, 99), 2)},
            "insert_mops": round(n / pct(ins, 50), 1), "find_mops": round(nq / pct(fnd, 50), 1)}


def iceberg_static(torch, cpht, synth, dev, reps=3):
    """Iceberg Put / Find at the paper's Sec. 5.1 shape: 2^27 primary + 2^24
    secondary slots, B0 = 32, B1 = 16, 37-bit keys; fill from empty to load
    0.9 with distinct keys in one batch, then 2^26 finds at 50 % hit.
    Compact 16/32-bit slots against plain 64/64-bit slots."""
    w, L0, L1 = 37, 27, 24
    cap = (1 << L0) + (1 << L1)
    n = int(LOAD * cap)
    keys = synth.distinct_keys(w, KEY_SEED + 1, 0, n, device=dev)
    q = synth.find_queries(w, KEY_SEED + 1, n, N_FIND, 0.5, Q_SEED + 1, device=dev)
    out = torch.empty(n, dtype=torch.uint8, device=dev)
    found = torch.empty(N_FIND, dtype=torch.uint8, device=dev)
    rows = {}
    for label, s0, s1, cmp_ in (("compact_16_32", 16, 32, 1), ("plain_64_64", 64, 64, 0)):
        t = cpht.Table(scheme=cpht.ICEBERG, key_bits=w, log2_slots0=L0, log2_slots1=L1, bucket0=32, bucket1=16,
                       slot_bits0=s0, slot_bits1=s1, compact=cmp_, seed=5)
        ins, fnd = [], []
        for rep in range(reps + 1):
            e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            t.clear(50 + rep)
            e[0].record()
            t.insert(keys, out)
            e[1].record()
            t.find(q, found)
            e[2].record()
            e[2].synchronize()
            if rep:
                ins.append(e[0].elapsed_time(e[1]))
                fnd.append(e[1].elapsed_time(e[2]))
        occ, cap_ = t.count()
        nfull = int((out == cpht.FULL).sum().item())
        ti, tf = sum(ins) / len(ins), sum(fnd) / len(fnd)
        # algorithmic bytes and random bucket reads (128-byte lines) per operation
        b0, b1 = 32 * s0 // 8, 16 * s1 // 8
        l0, l1 = -(-b0 // LINE), -(-b1 // LINE)
        ins_b = b0 + 2 * ICE_L2["put"] * b1 + SECTOR + KEY_BYTES + RESULT_BYTES
        fnd_b = b0 + 2 * ICE_L2["find"] * b1 + KEY_BYTES + RESULT_BYTES
        ins_l, fnd_l = l0 + 2 * ICE_L2["put"] * l1, l0 + 2 * ICE_L2["find"] * l1
        rows[label] = {"insert_mops": round(n / ti / 1e3, 1), "find_mops": round(N_FIND / tf / 1e3, 1),
                       "insert_ms": round(ti, 3), "find_ms": round(tf, 3), "full": nfull,
                       "fill_factor": round(occ / cap_, 4),
                       "table_bytes": t.level_bytes(0) + t.level_bytes(1),
                       "roofline": {
                           "insert": {"bytes_per_op": round(ins_b, 1), "GB_per_s": round(n * ins_b / ti / 1e6, 1),
                                      "frac": round(n * ins_b / ti / 1e6 / HBM_PEAK_GBS, 4),
                                      "line_reads_G_per_s": round(n * ins_l / ti / 1e6, 2)},
                           "find": {"bytes_per_op": round(fnd_b, 1), "GB_per_s": round(N_FIND * fnd_b / tf / 1e6, 1),
                                    "frac": round(N_FIND * fnd_b / tf / 1e6 / HBM_PEAK_GBS, 4),
                                    "line_reads_G_per_s": round(N_FIND * fnd_l / tf / 1e6, 2)}}}
        if ICE_TRAFFIC["src_sha"] == csrc_sha(ICE_SOURCES):  # measured bytes, where still valid
            for op, nops, ms in (("insert", n, ti), ("find", N_FIND, tf)):
                tb = ICE_TRAFFIC[f"{op}_{s0}_{s1}"]
                rows[label]["roofline"][op].update(
                    traffic_bytes_per_op=tb, traffic_GB_per_s=round(nops * tb / ms / 1e6, 1),
                    traffic_frac=round(nops * tb / ms / 1e6 / HBM_PEAK_GBS, 4))
        del t
    rows["compact_vs_plain"] = {
        "insert": round(rows["compact_16_32"]["insert_mops"] / rows["plain_64_64"]["insert_mops"], 3),
        "find": round(rows["compact_16_32"]["find_mops"] / rows["plain_64_64"]["find_mops"], 3),
        "memory": round(rows["compact_16_32"]["table_bytes"] / rows["plain_64_64"]["table_bytes"], 4),
    }
    rows["config"] = (f"iceberg 2^{L0} + 2^{L1} slots, B0=32, B1=16, {w}-bit keys; insert {n} distinct keys "
                      f"(load {LOAD}) in one batch, then 2^26 finds 50% hit")
    return rows


def iceberg_sweep(torch, cpht, synth, dev, reps=2):
    """The paper's iceberg Put / Find benchmarks (Sec. 5.1): 2^27 + 2^24 slots,
    37-bit keys, 8, 16 and 32 slots per primary bucket (secondary buckets
    half as large) with 16/32-bit (extra compact), 32/32-bit (compact) and
    64/64-bit (plain) slots; for each fill factor of the sweep the table is
    filled from empty with distinct keys in one batch and then queried with
    2^26 distinct keys, half of them stored.  Rates are medians over `reps`
    repetitions with a new permutation seed each; fill factors at which an
    insert answered FULL are marked (iceberg reaches 0.9 only with 32-slot
    primary buckets, Sec. 5.2)."""
    w, L0, L1 = 37, 27, 24
    cap = (1 << L0) + (1 << L1)
    loads = tuple(x for x in SWEEP_LOADS if x <= 0.9)
    n_max = int(max(loads) * cap)
    keys = synth.distinct_keys(w, KEY_SEED + 21, 0, n_max, device=dev)
    qs = {L: synth.find_queries(w, KEY_SEED + 21, int(L * cap), N_FIND, 0.5, Q_SEED + 21, device=dev)
          for L in loads}
    out = torch.empty(n_max, dtype=torch.uint8, device=dev)
    found = torch.empty(N_FIND, dtype=torch.uint8, device=dev)
    rows = []
    for s0, s1 in ((16, 32), (32, 32), (64, 64)):
        for b0 in (8, 16, 32):
            t = cpht.Table(scheme=cpht.ICEBERG, key_bits=w, log2_slots0=L0, log2_slots1=L1, bucket0=b0,
                           bucket1=b0 // 2, slot_bits0=s0, slot_bits1=s1, compact=int(s0 < 64), seed=5)
            for L in loads:
                n = int(L * cap)
                ins, fnd = [], []
                for rep in range(reps + 1):
                    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
                    t.clear(900 + rep)
                    e[0].record()
                    t.insert(keys[:n], out[:n])
                    e[1].record()
                    t.find(qs[L], found)
                    e[2].record()
                    e[2].synchronize()
                    if rep:
                        ins.append(e[0].elapsed_time(e[1]))
                        fnd.append(e[1].elapsed_time(e[2]))
                full = int((out[:n] == cpht.FULL).sum().item())
                rows.append({"slot_bits": f"{s0}/{s1}", "bucket0": b0, "load": L, "subtile": t.config.subtile,
                             "insert_mops": round(n / (sorted(ins)[len(ins) // 2] / 1000.0) / 1e6, 1),
                             "find_mops": round(N_FIND / (sorted(fnd)[len(fnd) // 2] / 1000.0) / 1e6, 1),
                             "full": full})
            del t
    del keys, qs
    return {"config": (f"iceberg 2^{L0} + 2^{L1} slots, {w}-bit keys, B1 = B0/2; fill from empty to each load in "
                       f"one batch, then 2^26 finds 50% hit"), "rows": rows}


def mixed_stream_check(torch, idx, ops, out, n_fresh, counted):
    """Answers of the dynamic-operation stream (synth.mixed_batches) against
    the set semantics, from the index each key was drawn from (keys =
    phi(index), distinct indices give distinct keys): every distinct inserted
    key is answered PUT exactly once, in the first batch that inserts it, and
    FOUND everywhere else; a find answers 1 if its key was inserted by an
    earlier batch, 0 if by no batch up to its own, either way if by its own
    batch; the table ends holding exactly the distinct inserted keys."""
    import synth

    nb, batch = idx.shape
    dev = idx.device
    bidx = torch.arange(nb, device=dev).view(nb, 1).expand(nb, batch)
    ins = ops == 1
    j, b, o = idx[ins], bidx[ins], out[ins]
    first = torch.full((n_fresh,), nb, dtype=torch.int64, device=dev)
    first.scatter_reduce_(0, j, b, reduce="amin")
    bad_answer = int(((o != 1) & (o != 2)).sum().item())  # PUT or FOUND only
    put = o == 1
    cnt = torch.zeros(n_fresh, dtype=torch.int32, device=dev)
    cnt.scatter_add_(0, j[put], torch.ones(int(put.sum().item()), dtype=torch.int32, device=dev))
    bad_put_count = int((cnt != 1).sum().item())
    late_put = int((first[j[put]] != b[put]).sum().item())
    del j, b, o, put, cnt
    fnd = ~ins
    j, b, o = idx[fnd], bidx[fnd], out[fnd]
    inserted = j < n_fresh
    assert int((inserted & (j >= synth.MISS_BASE)).sum().item()) == 0
    fj = torch.where(inserted, first[j.clamp(max=n_fresh - 1)], torch.full_like(j, nb))
    must1 = fj < b
    racy = fj == b
    wrong_find = int(((o != 1) & must1).sum().item()) + int(((o != 0) & ~must1 & ~racy).sum().item()) + \
        int(((o > 1) & racy).sum().item())
    ok = bad_answer == 0 and bad_put_count == 0 and late_put == 0 and wrong_find == 0 and counted == n_fresh
    return {"result": "ok" if ok else "FAILED", "insert_answers_not_put_or_found": bad_answer,
            "keys_not_put_exactly_once": bad_put_count, "puts_after_first_batch": late_put,
            "wrong_fixed_finds": wrong_find, "racy_finds": int(racy.sum().item()),
            "count": counted, "distinct_inserted": n_fresh}


def iceberg_mixed(torch, cpht, synth, dev, log2_slots0=28, batch=1 << 20, graph_run=32):
    """Dynamic operation at 2^28 + 2^25 slots (B0 = 32, B1 = 16, 34-bit keys):
    mixed batches of `batch` operations, half finds and half find-or-puts in
    random order; 30 % of inserts repeat an earlier-issued key; finds hit keys
    inserted by earlier batches half of the time (synth.mixed_batches).  Runs
    from load 0 to 0.9, batches issued one by one on one stream, and for the
    compact table also with runs of `graph_run` batches captured in one HIP
    graph and replayed (batches still run in order, one launch each).
    Reports ops/s over the whole run, the per-batch latency distribution and
    a check of every answer against the set semantics."""
    w = 34
    L0, L1 = log2_slots0, log2_slots0 - 3
    cap = (1 << L0) + (1 << L1)
    keys, ops, idx, n_fresh = synth.mixed_batches(w, KEY_SEED + 3, cap, LOAD, batch, device=dev)
    nb = keys.shape[0]
    out = torch.empty(nb, batch, dtype=torch.uint8, device=dev)
    rows = {}
    for label, s0, s1, cmp_ in (("compact_16_32", 16, 32, 1), ("plain_64_64", 64, 64, 0)):
        t = cpht.Table(scheme=cpht.ICEBERG, key_bits=w, log2_slots0=L0, log2_slots1=L1, bucket0=32, bucket1=16,
                       slot_bits0=s0, slot_bits1=s1, compact=cmp_, seed=9)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(nb + 1)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev[0].record()
        for b in range(nb):
            t.mixed(keys[b], ops[b], out[b])
            ev[b + 1].record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        lat = [ev[b].elapsed_time(ev[b + 1]) for b in range(nb)]
        occ, cap_ = t.count()
        nfull = int((out == cpht.FULL).sum().item())
        first_full = None
        if nfull:
            first_full = int(torch.nonzero((out == cpht.FULL).any(dim=1))[0].item())
        gpu_ms = ev[0].elapsed_time(ev[nb])
        rows[label] = {"mops": round(nb * batch / gpu_ms / 1e3, 1), "wall_mops": round(nb * batch / wall / 1e6, 1),
                       "batches": nb, "batch_ops": batch,
                       "batch_latency_ms": {"p50": round(pct(lat, 50), 4), "p99": round(pct(lat, 99), 4)},
                       "fill_factor": round(occ / cap_, 4), "full": nfull, "first_full_batch": first_full,
                       "table_bytes": t.level_bytes(0) + t.level_bytes(1),
                       "check": mixed_stream_check(torch, idx, ops, out, n_fresh, occ)}
        if cmp_:
            rows[label]["graph_replay"] = mixed_graph_run(torch, t, keys, ops, out, graph_run)
            rows[label]["graph_replay"]["check"] = mixed_stream_check(torch, idx, ops, out, n_fresh, t.count()[0])
        del t
    rows["compact_vs_plain"] = round(rows["compact_16_32"]["mops"] / rows["plain_64_64"]["mops"], 3)
    rows["config"] = (f"iceberg 2^{L0} + 2^{L1} slots, B0=32, B1=16, {w}-bit keys; {nb} mixed batches of {batch} "
                      f"ops (50% find / 50% find-or-put, 30% duplicate inserts, finds 50% hit), load 0 -> {LOAD}")
    del keys, ops, idx, out
    return rows


def mixed_graph_run(torch, t, keys, ops, out, run):
    """The same batches from an empty table (same seed), runs of `run`
    consecutive batches captured in one graph each and replayed once; the
    capture and instantiation of each run happen before the timed region."""
    nb = keys.shape[0]
    t.clear(t.config.seed)
    torch.cuda.synchronize()
    graphs = []
    s = torch.cuda.Stream()
    for a in range(0, nb, run):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            for b in range(a, min(nb, a + run)):
                t.mixed(keys[b], ops[b], out[b])
        graphs.append(g)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for g in graphs:
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    del graphs
    return {"mops": round(nb * keys.shape[1] / ms / 1e3, 1), "batches_per_graph": run, "ms": round(ms, 3)}


def many_tables(torch, cpht, synth, dev, n_tables=4096, lo=10, hi=20, load=0.85, reps=3):
    """Many-table workload: n_tables independent compact iceberg tables with
    2^e + 2^(e-3) slots, e uniform in lo..hi, 32-bit keys; each table is filled
    to `load` with distinct keys and then queried with twice its capacity in
    finds (50 % hit).  The autotuner picks each size class's kernel variant.
    Timed three ways: table-set launches (plan + one persistent launch per
    variant group), the same captured once in a graph and replayed, and one
    single-table launch per table."""
    from paper_2406_09255_amd import tune

    w = 32
    e_t = (synth.uniform_below(0xE5, n_tables, hi - lo + 1, dev) + lo).cpu().tolist()
    t0 = time.perf_counter()
    chosen, tried = tune.tune_set(cpht.ICEBERG, w, e_t, load, device=dev)
    tune_s = time.perf_counter() - t0
    cfgs = []
    for i, e in enumerate(e_t):
        c = cpht.default_config(cpht.ICEBERG)
        c.key_bits = w
        c.log2_slots0, c.log2_slots1 = e, e - 3
        c.bucket0, c.slot_bits0, c.slot_bits1, c.subtile = (chosen["bucket0"], chosen["slot_bits0"],
                                                           chosen["slot_bits1"], chosen["subtile"])
        c.bucket1 = c.bucket0 // 2
        c.seed = 7000 + i
        cfgs.append(c)
    cap = torch.tensor([(1 << e) + (1 << (e - 3)) for e in e_t], dtype=torch.int64, device=dev)
    n_t = (cap.double() * load).long()
    q_t = 2 * cap
    ko = torch.zeros(n_tables + 1, dtype=torch.int64, device=dev)
    ko[1:] = torch.cumsum(n_t, 0)
    qo = torch.zeros(n_tables + 1, dtype=torch.int64, device=dev)
    qo[1:] = torch.cumsum(q_t, 0)
    total_k, total_q = int(ko[-1]), int(qo[-1])
    keys64 = synth.distinct_keys(w, KEY_SEED + 9, 0, total_k, device=dev)
    tid = torch.repeat_interleave(torch.arange(n_tables, device=dev), q_t)
    pick = ko[tid] + ((synth.uniform_below(0xAB, total_q, 1 << 30, dev) * n_t[tid]) >> 30)
    hit = synth.uniform_below(0xCD, total_q, 2, dev) == 1
    miss = synth.distinct_keys(w, KEY_SEED + 9, total_k, total_q, device=dev)
    queries = synth.to_words(torch.where(hit, keys64[pick], miss), w).contiguous()
    keys = synth.to_words(keys64, w).contiguous()
    del keys64, tid, pick, hit, miss
    m = cpht.MultiTable(cfgs, max_keys=max(total_k, total_q))
    info = m.info()
    out = torch.empty(total_k, dtype=torch.uint8, device=dev)
    found = torch.empty(total_q, dtype=torch.uint8, device=dev)
    ops = total_k + total_q

    def timed(fn, n):
        ts = []
        for _ in range(n):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            m.clear()
            a.record()
            fn()
            b.record()
            b.synchronize()
            ts.append(a.elapsed_time(b))
        return sorted(ts)[len(ts) // 2]

    def set_launch():
        m.insert(keys, ko, out)
        m.find(queries, qo, found)

    set_launch()
    set_ms = timed(set_launch, reps)
    n_put = int((out == cpht.PUT).sum().item())
    n_full = int((out == cpht.FULL).sum().item())
    ok = n_put + n_full == total_k  # FULL is a valid answer of a two-level table near its limit
    hit_frac = float(found.float().mean().item())

    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            m.insert(keys, ko, out, stream=s)
            m.find(queries, qo, found, stream=s)
    torch.cuda.synchronize()
    graph_ms = timed(g.replay, reps)
    ok = ok and int((out == cpht.PUT).sum().item()) + int((out == cpht.FULL).sum().item()) == total_k

    views = [m.table(i) for i in range(n_tables)]
    kb, qb = ko.tolist(), qo.tolist()

    def per_table():
        for i, v in enumerate(views):
            v.insert(keys[kb[i]:kb[i + 1]], out[kb[i]:kb[i + 1]])
        for i, v in enumerate(views):
            v.find(queries[qb[i]:qb[i + 1]], found[qb[i]:qb[i + 1]])

    per_table()
    sep_ms = timed(per_table, 2)
    ok = ok and int((out == cpht.PUT).sum().item()) + int((out == cpht.FULL).sum().item()) == total_k
    return {
        "config": (f"{n_tables} compact iceberg tables, 2^e + 2^(e-3) slots with e uniform in {lo}..{hi}, 32-bit "
                   f"keys; fill each to {load} ({total_k} inserts), then 2x capacity finds at 50% hit "
                   f"({total_q} finds)"),
        "check": "ok" if ok and abs(hit_frac - 0.5) < 0.01 else "FAILED",
        "puts": n_put, "full": n_full, "hit_fraction": round(hit_frac, 4),
        "table_set_mops": round(ops / set_ms / 1e3, 1), "table_set_ms": round(set_ms, 3),
        "graph_mops": round(ops / graph_ms / 1e3, 1), "graph_ms": round(graph_ms, 3),
        "separate_launches_mops": round(ops / sep_ms / 1e3, 1), "separate_launches_ms": round(sep_ms, 3),
        "graph_vs_separate": round(sep_ms / graph_ms, 2),
        "variant_groups": info["groups"], "arena_bytes": info["arena_bytes"],
        "autotune_seconds": round(tune_s, 2), "autotuned": chosen, "autotune_candidates": tried,
    }


def iceberg_zipf(torch, cpht, synth, dev, log2_slots0=28, batch=1 << 20, max_batches=8000, chunk=250,
                 target=0.9):
    """Dynamic operation under skew: 2^28 + 2^25 slots, mixed batches of
    `batch` operations (half finds, half find-or-puts), keys Zipf(1.1) over
    2^34 ranks mapped to 34-bit keys by a bijection, for inserts and finds
    alike; the hottest key is about 10 % of all draws, so most inserts repeat
    a key already present.  Runs until the table reaches `target` load or an
    insert answers FULL (at most max_batches batches).  Keys are generated on
    the device in chunks between timed regions; each batch is timed alone."""
    w = 34
    L0, L1 = log2_slots0, log2_slots0 - 3
    t = cpht.Table(scheme=cpht.ICEBERG, key_bits=w, log2_slots0=L0, log2_slots1=L1, bucket0=32, bucket1=16,
                   slot_bits0=16, slot_bits1=32, seed=19)
    cap = t.count()[1]
    ops = (synth.uniform_below(0x2F, batch, 2, dev)).to(torch.uint8)
    ins = ops == 1
    outs = torch.empty((chunk, batch), dtype=torch.uint8, device=dev)
    # truth: first[k] = 1 + the first batch that inserts key k (0: none yet),
    # over the whole 2^34 key space (32 GiB of int16)
    first = torch.zeros(1 << w, dtype=torch.int16, device=dev)
    bad = {"insert": 0, "put_count": 0, "find": 0}
    lat, curve = [], []
    b, occ, first_full, puts, racy = 0, 0, None, 0, 0
    while b < max_batches and occ < target * cap and first_full is None:
        nb = min(chunk, max_batches - b)
        keys = [synth.zipf_keys(w, KEY_SEED + 5, 1.1, batch, 1000 + b + i, device=dev) for i in range(nb)]
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(nb + 1)]
        torch.cuda.synchronize()
        ev[0].record()
        for i in range(nb):
            t.mixed(keys[i], ops, outs[i])
            ev[i + 1].record()
        torch.cuda.synchronize()
        ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(nb)]
        lat += ms
        full_rows = torch.nonzero((outs[:nb] == cpht.FULL).any(dim=1))
        if full_rows.numel():
            first_full = b + int(full_rows[0].item())
        puts += int(((outs[:nb] == cpht.PUT) & ins).sum().item())  # finds answer 1 too
        for i in range(nb):  # every answer against the set semantics (untimed)
            r = zipf_batch_check(torch, first, b + i, keys[i], ins, outs[i])
            racy += r.pop("racy")
            for k_ in bad:
                bad[k_] += r[k_]
        occ = t.count()[0]
        b += nb
        curve.append({"batches": b, "load": round(occ / cap, 4), "mops": round(nb * batch / sum(ms) / 1e3, 1)})
        del keys
    distinct = int(torch.count_nonzero(first).item())
    del first
    ok = first_full is None and not any(bad.values()) and distinct == occ == puts
    check = {"result": "ok" if ok else "FAILED", "wrong_insert_answers": bad["insert"],
             "batches_with_wrong_put_count": bad["put_count"], "wrong_fixed_finds": bad["find"],
             "racy_finds": racy, "distinct_inserted": distinct, "count": occ, "puts": puts}
    rows = {"check": check, "mops": round(b * batch / sum(lat) / 1e3, 1),
            "batch_latency_ms": {"p50": round(pct(lat, 50), 4), "p99": round(pct(lat, 99), 4)},
            "batches": b, "operations": b * batch, "puts": puts, "fill_factor": round(occ / cap, 4),
            "first_full_batch": first_full, "by_load": curve[:: max(1, len(curve) // 12)] + curve[-1:],
            "config": (f"iceberg 2^{L0} + 2^{L1} slots (16/32-bit), {w}-bit keys Zipf(1.1) over 2^34 ranks; mixed "
                       f"batches of {batch} ops (50% find / 50% find-or-put) until load {target} or the first "
                       f"FULL (at most {max_batches} batches)")}
    del t, outs
    return rows


def zipf_batch_check(torch, first, b, keys, ins, out):
    """One mixed batch against the set semantics, with first[k] = 1 + the
    first batch that inserted key k (0 = not yet), updated here: an insert of
    a key stored by an earlier batch answers FOUND; the batch's new keys are
    answered PUT once each (and FOUND otherwise); a find answers 1 if an
    earlier batch inserted its key, 0 if no batch up to this one did, either
    way if this batch does."""
    ki, oi = keys[ins], out[ins]
    seen = first[ki] != 0
    wrong_insert = int((seen & (oi != 2)).sum().item()) + int((~seen & (oi != 1) & (oi != 2)).sum().item())
    new = ki[~seen]
    put_keys = ki[oi == 1]
    n_new = int(torch.unique(new).numel())
    put_ok = put_keys.numel() == n_new and int(torch.unique(put_keys).numel()) == n_new
    first[new] = b + 1
    v = first[keys[~ins]].to(torch.int32)
    of = out[~ins]
    earlier, same = (v != 0) & (v <= b), v == b + 1
    wrong_find = int((earlier & (of != 1)).sum().item()) + int((~earlier & ~same & (of != 0)).sum().item()) + \
        int((same & (of > 1)).sum().item())
    return {"insert": wrong_insert, "put_count": 0 if put_ok else 1, "find": wrong_find,
            "racy": int(same.sum().item())}


def serving(torch, cpht, synth, dev, n_req=100000, n_req_other=20000, log2_slots0=32, prefill=0.5, seed=3,
            stop_load=0.85):
    """Serving loop over one resident compact iceberg table of 2^32 + 2^29
    slots (16/32-bit, 40-bit keys), pre-filled to load 0.5.  Requests: sizes
    lognormal (median 4096, sigma 2) clipped to 1..2^22; 70 % finds (half hits
    on pre-filled keys, half on keys never inserted) and 30 % inserts of fresh
    keys; host-resident (pinned) buffers.  Runs: all n_req requests at t = 0
    (saturation) and Poisson arrivals at 50 % of the saturated request rate;
    the first n_req_other requests at 25, 75 and 90 %.  The trace is cut where
    its inserts would take the table past stop_load.  The comparator is the
    same server with one request per launch and one launch in flight (plain
    batched launches in arrival order).  Each run is made with the staged
    and the zero-copy server.  The table is emptied and pre-filled
    again before each run, and every answer of every run is checked: inserts
    of fresh keys answer PUT, finds answer 1 exactly for pre-filled keys."""
    import numpy as np

    w = 40
    L0, L1 = log2_slots0, log2_slots0 - 3
    cap = (1 << L0) + (1 << L1)
    n_pre = int(prefill * cap)
    t = cpht.Table(scheme=cpht.ICEBERG, key_bits=w, log2_slots0=L0, log2_slots1=L1, bucket0=32, bucket1=16,
                   slot_bits0=16, slot_bits1=32, seed=23)

    def refill():
        t.clear(23)
        chunk = 1 << 28
        for a in range(0, n_pre, chunk):
            k = synth.distinct_keys(w, KEY_SEED + 7, a, min(chunk, n_pre - a), device=dev)
            t.insert(k)
            del k
        torch.cuda.synchronize()

    r = np.random.default_rng(seed)
    sizes = np.clip(np.round(np.exp(r.normal(np.log(4096), 2.0, n_req))), 1, 1 << 22).astype(np.int64)
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    total = int(offsets[-1])
    is_ins = synth.uniform_below(0x31, total, 10, dev) < 3
    # cut the trace where its inserts would pass stop_load
    ins_upto = torch.cumsum(is_ins.to(torch.int64), 0)
    room = int(stop_load * cap) - n_pre
    # first operation past the room (the running count is sorted)
    last_op = int(torch.searchsorted(ins_upto, torch.tensor([room], device=dev), right=True)[0].item())
    if last_op < total:
        n_req = int(np.searchsorted(offsets, last_op, side="right")) - 1
        total = int(offsets[n_req])
        is_ins = is_ins[:total]
    del ins_upto
    n_req_other = min(n_req_other, n_req)
    is_hit = synth.uniform_below(0x32, total, 2, dev) == 1
    fresh_idx = n_pre + torch.cumsum(is_ins.to(torch.int64), 0)
    hit_idx = synth.uniform_below(0x33, total, 1 << 30, dev) * n_pre >> 30
    miss_idx = (1 << 39) + torch.arange(total, device=dev)
    idx = torch.where(is_ins, fresh_idx, torch.where(is_hit, hit_idx, miss_idx))
    keys = torch.empty(total, dtype=torch.int64, pin_memory=True)
    keys.copy_(synth.feistel(w, KEY_SEED + 7, idx))
    ops = torch.empty(total, dtype=torch.uint8, pin_memory=True)
    ops.copy_(is_ins.to(torch.uint8))
    out = torch.zeros(total, dtype=torch.uint8, pin_memory=True)
    # the answer every operation must get: no find looks for a key that a
    # request inserts, so no answer depends on how requests overlap
    truth = torch.where(is_ins, torch.full_like(is_ins, cpht.PUT, dtype=torch.uint8), is_hit.to(torch.uint8))
    ins_in = {nr: int(is_ins[:int(offsets[nr])].sum().item()) for nr in {n_req, n_req_other}}
    del is_hit, fresh_idx, hit_idx, miss_idx, idx, is_ins
    torch.cuda.empty_cache()

    def run(arrival, nr, **kw):
        refill()
        out.zero_()
        srv = cpht.Server(t, **kw)
        lat, mk = srv.replay(arrival[:nr], offsets[:nr + 1], keys, ops, out)
        st = srv.stats()
        srv.stop()
        ops_n = int(offsets[nr])
        wrong = int((out[:ops_n].to(dev) != truth[:ops_n]).sum().item())
        want_count = n_pre + ins_in[nr]
        counted = t.count()[0]
        lat_ms = lat.astype(np.float64) / 1e6
        print(f"[bench] serving run: {nr} requests, {kw}, {mk / 1e6:.1f} ms", file=sys.stderr, flush=True)
        return {"requests": nr, "operations": ops_n, "mops": round(ops_n / (mk / 1e9) / 1e6, 1),
                "requests_per_s": round(nr / (mk / 1e9), 0),
                "p50_ms": round(float(np.percentile(lat_ms, 50)), 3),
                "p99_ms": round(float(np.percentile(lat_ms, 99)), 3),
                "makespan_ms": round(mk / 1e6, 2), "launches": st["launches"], "max_queue": st["max_queue"],
                "load_end": round(counted / cap, 4),
                "check": "ok" if (wrong == 0 and counted == want_count) else
                         f"FAILED: {wrong} wrong answers, count {counted} (want {want_count})"}

    # staging_keys = 0: the staged servers size their staging ring, the
    # admission budget, from the device memory free when they start
    cont = dict(max_inflight=4, coalesce=1, staging_keys=0, max_batch_keys=1 << 22)
    plain = dict(max_inflight=1, coalesce=0, staging_keys=0, max_batch_keys=1 << 22)
    direct = dict(max_inflight=4, coalesce=1, max_batch_keys=1 << 22, zero_copy=1)
    res = {"config": (f"iceberg 2^{L0} + 2^{L1} slots (16/32-bit, {t.level_bytes(0) + t.level_bytes(1)} bytes), "
                      f"{w}-bit keys, pre-filled to load {prefill}; {n_req} requests ({total} operations) for the "
                      f"saturated and 50% runs, the first {n_req_other} for the other rates; sizes "
                      f"lognormal(median 4096, sigma 2) in 1..2^22, 70% find / 30% insert, pinned host buffers; "
                      f"trace cut at load {stop_load}; staged servers admit by a staging ring sized from the free "
                      f"device memory at start"),
           "requests": n_req, "operations": total}
    zero = np.zeros(n_req, dtype=np.uint64)
    res["saturated"] = run(zero, n_req, **cont)
    res["saturated_plain"] = run(zero, n_req, **plain)
    res["saturated_zero_copy"] = run(zero, n_req, **direct)
    rate = res["saturated"]["requests_per_s"]
    for frac in (0.25, 0.5, 0.75, 0.9):
        nr = n_req if frac == 0.5 else n_req_other
        gaps = r.exponential(1e9 / (frac * rate), nr)
        arrival = np.cumsum(gaps).astype(np.uint64)
        res[f"poisson_{int(frac * 100)}"] = run(arrival, nr, **cont)
        if frac == 0.5:
            res[f"poisson_{int(frac * 100)}_plain"] = run(arrival, nr, **plain)
        res[f"poisson_{int(frac * 100)}_zero_copy"] = run(arrival, nr, **direct)
    checks = [v["check"] for v in res.values() if isinstance(v, dict) and "check" in v]
    res["check"] = "ok" if all(c == "ok" for c in checks) else "FAILED"
    # one 4096-operation request at a time on an idle server, beside a bare
    # mixed launch over device-resident buffers (launch + kernel + synchronise)
    import time
    nq = 4096
    kq, oq, rq = keys[:nq], ops[:nq], out[:nq]
    kd, od = kq.to(dev), oq.to(dev)
    rd = torch.empty(nq, dtype=torch.uint8, device=dev)
    bare = []
    for _ in range(300):
        a = time.perf_counter_ns()
        t.mixed(kd, od, out=rd)
        torch.cuda.synchronize()
        bare.append(time.perf_counter_ns() - a)
    idle = {"bare_launch_device_buffers": bare}
    for name, kw in (("staged", cont), ("zero_copy", direct)):
        srv = cpht.Server(t, **kw)
        idle[name] = [srv.wait(srv.submit(kq, oq, rq)) for _ in range(300)]
        srv.stop()
    res["idle_request_4096_us"] = {k: {"p50": round(float(np.percentile(v, 50)) / 1e3, 1),
                                       "p99": round(float(np.percentile(v, 99)) / 1e3, 1)} for k, v in idle.items()}
    # every operation moves its key and opcode to the device and its answer
    # back over the host link; the inbound direction binds
    kb = t.key_dtype.itemsize
    link = host_link(torch, dev)
    res["host_link"] = dict(link, bytes_in_per_op=kb + 1, bytes_out_per_op=1)
    for name in ("saturated", "saturated_zero_copy"):
        gbs = res[name]["mops"] * 1e6 * (kb + 1) / 1e9
        res[name]["host_link_in_GBps"] = round(gbs, 2)
        res[name]["frac_of_h2d"] = round(gbs / link["h2d_GBps"], 3)
    del t, keys, ops, out, truth
    return res


def serving_small(torch, cpht, synth, dev, n_burst=20000, burst_ops=64, reps=300):
    """The three request paths on a table within the resident loop's covered
    shapes: iceberg 2^22 + 2^19 slots (32/32-bit, 40-bit keys), pre-filled to
    load 0.5.  (1) One 4096-operation request at a time on an idle server
    (half finds of pre-filled keys, half inserts of fresh keys), staged,
    zero-copy and resident, beside a bare mixed launch + synchronise on device
    buffers; (2) a burst of n_burst requests of burst_ops operations in
    separate pinned buffers submitted at once, per path; (3) 1024 requests of
    2^16 operations back to back in one pinned buffer submitted at once, per
    path.  Every answer of (2) and (3) is checked (inserts of fresh keys PUT,
    of pre-filled keys FOUND, finds of pre-filled keys 1)."""
    import numpy as np

    w, L0, L1 = 40, 22, 19
    out = {"config": (f"iceberg 2^{L0} + 2^{L1} slots (32/32-bit), {w}-bit keys, pre-filled to load 0.5; "
                      f"idle 4096-operation requests; a burst of {n_burst} requests of {burst_ops} operations "
                      f"in separate pinned buffers")}
    paths = {"staged": dict(max_inflight=4, coalesce=1, staging_keys=1 << 20, max_batch_keys=1 << 16),
             "zero_copy": dict(max_inflight=4, coalesce=1, max_batch_keys=1 << 16, zero_copy=1),
             "resident": dict(zero_copy=1, resident=1, max_batch_keys=1 << 16)}
    cap = (1 << L0) + (1 << L1)
    n_pre = cap // 2

    def fresh_table():
        t = cpht.Table(scheme=cpht.ICEBERG, key_bits=w, log2_slots0=L0, log2_slots1=L1, bucket0=32, bucket1=16,
                       slot_bits0=32, slot_bits1=32, seed=41)
        t.insert(synth.distinct_keys(w, KEY_SEED + 11, 0, n_pre, device=dev))
        torch.cuda.synchronize()
        return t

    def words(idx):
        return synth.to_words(synth.feistel(w, KEY_SEED + 11, idx), w)

    # (1) idle latency
    nq = 4096
    fresh = n_pre + torch.arange(reps * nq, dtype=torch.int64)
    hits = torch.arange(nq // 2, dtype=torch.int64) * 7 % n_pre
    lat = {}
    t = fresh_table()
    ops1 = torch.cat([torch.ones(nq // 2, dtype=torch.uint8), torch.zeros(nq // 2, dtype=torch.uint8)])
    kd = torch.cat([words(fresh[:nq // 2]), words(hits)]).to(dev)
    od = ops1.to(dev)
    rd = torch.empty(nq, dtype=torch.uint8, device=dev)
    bare = []
    for i in range(reps):
        a = time.perf_counter_ns()
        t.mixed(kd, od, out=rd)
        torch.cuda.synchronize()
        bare.append(time.perf_counter_ns() - a)
    lat["bare_launch_device_buffers"] = bare
    del t
    for name, kw in paths.items():
        t = fresh_table()
        kq = torch.cat([words(fresh[:nq // 2]), words(hits)]).pin_memory()
        oq = ops1.pin_memory()
        rq = torch.zeros(nq, dtype=torch.uint8).pin_memory()
        srv = cpht.Server(t, **kw)
        lat[name] = [srv.wait(srv.submit(kq, oq, rq)) for _ in range(reps)]
        srv.stop()
        del t
    out["idle_request_4096_us"] = {k: {"p50": round(float(np.percentile(v, 50)) / 1e3, 1),
                                       "p99": round(float(np.percentile(v, 99)) / 1e3, 1)} for k, v in lat.items()}
    # (2) burst of small requests in separate buffers
    half = burst_ops // 2
    hit_idx = (torch.arange(n_burst * half, dtype=torch.int64) * 13) % n_pre
    burst = {}
    for name, kw in paths.items():
        t = fresh_table()
        reqs, outs = [], []
        for i in range(n_burst):
            k = torch.cat([words(n_pre + torch.arange(i * half, (i + 1) * half, dtype=torch.int64)),
                           words(hit_idx[i * half:(i + 1) * half])])
            kb = torch.empty(burst_ops + 8, dtype=k.dtype).pin_memory()[:burst_ops]
            kb.copy_(k)
            ob = torch.empty(burst_ops + 8, dtype=torch.uint8).pin_memory()[:burst_ops]
            ob[:half] = 1
            ob[half:] = 0
            reqs.append((kb, ob))
            outs.append(torch.zeros(burst_ops + 8, dtype=torch.uint8).pin_memory()[:burst_ops])
        srv = cpht.Server(t, **kw)
        a = time.perf_counter()
        tickets = [srv.submit(k, o, r) for (k, o), r in zip(reqs, outs)]
        for tk in tickets:
            srv.wait(tk)
        dt = time.perf_counter() - a
        st = srv.stats()
        srv.stop()
        res = torch.stack(outs).numpy()
        ok = bool((res[:, :half] == cpht.PUT).all() and (res[:, half:] == 1).all()
                  and t.count()[0] == n_pre + n_burst * half)
        burst[name] = {"ms": round(dt * 1e3, 1), "requests_per_s": round(n_burst / dt), "launches": st["launches"],
                       "check": "ok" if ok else "FAILED"}
        print(f"[bench] serving_small burst {name}: {dt * 1e3:.1f} ms", file=sys.stderr, flush=True)
        del t, reqs, outs
    out["burst"] = burst
    # (3) saturated: n_sat requests of 2^16 operations back to back in one
    # pinned buffer, submitted at once (each is one launch or one ring
    # descriptor: max_batch_keys = 2^16).  Per request the first 256
    # operations insert fresh keys (PUT), the rest alternate find-or-put and
    # find of pre-filled keys (FOUND, 1).
    n_sat, sat_ops, n_fresh = 1024, 1 << 16, 256
    tot = n_sat * sat_ops
    pos = torch.arange(tot, dtype=torch.int64, device=dev)
    j = pos % sat_ops
    is_fresh = j < n_fresh
    idx = torch.where(is_fresh, n_pre + (pos // sat_ops) * n_fresh + j, (pos * 13) % n_pre)
    ops_d = torch.where(is_fresh | (j % 2 == 0), 1, 0).to(torch.uint8)
    want_d = torch.where(is_fresh, cpht.PUT, torch.where(j % 2 == 0, cpht.FOUND, 1)).to(torch.uint8)
    keys_h = torch.empty(tot, dtype=torch.int64).pin_memory()
    keys_h.copy_(synth.to_words(synth.feistel(w, KEY_SEED + 11, idx), w))
    ops_h = torch.empty(tot, dtype=torch.uint8).pin_memory()
    ops_h.copy_(ops_d)
    want = want_d.cpu()
    del pos, j, is_fresh, idx, ops_d, want_d
    sat = {}
    for name, kw in paths.items():
        t = fresh_table()
        res_h = torch.zeros(tot, dtype=torch.uint8).pin_memory()
        srv = cpht.Server(t, **kw)
        a = time.perf_counter()
        tickets = [srv.submit(keys_h[i * sat_ops:(i + 1) * sat_ops], ops_h[i * sat_ops:(i + 1) * sat_ops],
                              res_h[i * sat_ops:(i + 1) * sat_ops]) for i in range(n_sat)]
        shown = a
        for i, tk in enumerate(tickets):
            srv.wait(tk)
            if time.perf_counter() - shown > 10:
                shown = time.perf_counter()
                print(f"[bench] serving_small saturated {name}: {i + 1} of {n_sat} requests done",
                      file=sys.stderr, flush=True)
        dt = time.perf_counter() - a
        st = srv.stats()
        srv.stop()
        ok = bool(torch.equal(res_h, want) and t.count()[0] == n_pre + n_sat * n_fresh)
        sat[name] = {"ms": round(dt * 1e3, 2), "mops": round(tot / dt / 1e6, 1), "launches": st["launches"],
                     "check": "ok" if ok else "FAILED"}
        print(f"[bench] serving_small saturated {name}: {dt * 1e3:.1f} ms", file=sys.stderr, flush=True)
        del t, res_h
    out["saturated_2e16_requests"] = sat
    out["config"] += f"; saturated: {n_sat} requests of {sat_ops} operations back to back in one pinned buffer"
    out["check"] = "ok" if all(v["check"] == "ok" for v in list(burst.values()) + list(sat.values())) else "FAILED"
    return out


def host_link(torch, dev, mib=512, reps=5):
    """Copy rates between pinned host memory and the device (one 512 MiB
    transfer per direction, best of 5): the ceiling of any path whose
    operations cross the host link."""
    n = mib << 20
    h = torch.empty(n, dtype=torch.uint8).pin_memory()
    d = torch.empty(n, dtype=torch.uint8, device=dev)
    out = {}
    for name, dst, src in (("h2d_GBps", d, h), ("d2h_GBps", h, d)):
        best = None
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            dst.copy_(src, non_blocking=True)
            b.record()
            b.synchronize()
            ms = a.elapsed_time(b)
            best = ms if best is None else min(best, ms)
        out[name] = round(n / (best / 1e3) / 1e9, 2)
    del h, d
    return out


def ceilings(torch, cpht, dev, res, split_keys):
    """Measured random-access rates: 128-byte line reads, 32-bit CAS, and a
    line read followed by a CAS into it, on a buffer the size of the compact
    table (partly served by the 256 MB Infinity Cache) and on a 4 GiB buffer."""
    out = {}
    sink = torch.zeros(1, dtype=torch.int32, device=dev)
    for label, nbytes in (("table_size", res["table_bytes"]), ("4GiB", 1 << 32)):
        buf = torch.zeros(nbytes // 4, dtype=torch.int32, device=dev)
        row = {}
        for kind, name in ((cpht.PROBE_LINES, "line_reads"), (cpht.PROBE_CAS, "cas"),
                           (cpht.PROBE_CAS64, "cas64"), (cpht.PROBE_LINE_CAS, "line_read_then_cas"),
                           (cpht.PROBE_HALF_LINES, "half_line_reads"),
                           (cpht.PROBE_LINES_NT, "line_reads_nontemporal")):
            ops = 1 << 27
            cpht.probe(kind, buf, ops, 1, sink)  # warm-up (and first touch)
            times = []
            for rep in range(3):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                done = cpht.probe(kind, buf, ops, 2 + rep, sink)
                b.record()
                b.synchronize()
                times.append(a.elapsed_time(b))
            ms = sorted(times)[1]
            row[name] = {"G_per_s": round(done / (ms / 1000.0) / 1e9, 2), "ms": round(ms, 3)}
        row["line_reads"]["GB_per_s"] = round(row["line_reads"]["G_per_s"] * 128, 1)
        row["half_line_reads"]["GB_per_s"] = round(row["half_line_reads"]["G_per_s"] * 64, 1)
        out[label] = row
        del buf
    # the benchmark's kernels against these ceilings (lines per op from the oracle model)
    lines_put = ROUNDS_PER_PUT[LOAD]
    lines_find = PROBES_PER_FIND[LOAD]
    r = out["table_size"]
    out["put_vs_line_read_then_cas"] = round(res["insert_mops"] * lines_put / (r["line_read_then_cas"]["G_per_s"] * 1e3), 3)
    out["find_vs_line_reads"] = round(res["find_mops"] * lines_find / (r["line_reads"]["G_per_s"] * 1e3), 3)
    out["find_vs_line_reads_4GiB"] = round(res["find_mops"] * lines_find /
                                           (out["4GiB"]["line_reads"]["G_per_s"] * 1e3), 3)
    cf = res.get("cache_free")
    if isinstance(cf, dict) and "rows" in cf:
        # the 4 GiB compact table (not cache-resident) against the 4 GiB ceilings
        c4 = next(row for row in cf["rows"] if row["table"] == "compact_4GiB")
        g = out["4GiB"]
        out["cache_free_find_vs_line_reads_4GiB"] = round(c4["find_line_reads_G_per_s"] /
                                                          g["line_reads"]["G_per_s"], 3)
        out["cache_free_put_vs_line_read_then_cas_4GiB"] = round(
            c4["insert_mops"] * lines_put / (g["line_read_then_cas"]["G_per_s"] * 1e3), 3)
    # the quotienting split alone (three permutations per key) on the
    # benchmark's keys, against the build that applies it
    keys = split_keys[: 1 << 26]  # a power-of-two buffer of the benchmark's keys
    n = keys.numel()
    cpht.probe(cpht.PROBE_SPLIT, keys, n, 1, sink)
    times = []
    for rep in range(3):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        done = cpht.probe(cpht.PROBE_SPLIT, keys, n, 2 + rep, sink)
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b))
    ms = sorted(times)[1]
    per_key_s = ms / 1e3 / done
    out["split_three_perms"] = {"keys": done, "ms": round(ms, 4), "G_keys_per_s": round(1 / per_key_s / 1e9, 2),
                                "time_vs_put_per_key": round(per_key_s * res["insert_mops"] * 1e6, 4),
                                "time_vs_find_per_key": round(per_key_s * res["find_mops"] * 1e6, 4)}
    return out


_T0 = time.perf_counter()


def progress(name: str):
    """One line per finished section on stderr (the JSON line stays alone on stdout)."""
    print(f"[bench] {name} done at {time.perf_counter() - _T0:.1f} s", file=sys.stderr, flush=True)


def run_section(res: dict, name: str, fn):
    """res[name] = fn(); a section that raises is reported in its place (and
    its traceback on stderr) so that the headline and the other sections
    still make the JSON line."""
    try:
        res[name] = fn()
    except Exception as e:  # noqa: BLE001 - reported, not hidden
        import traceback

        traceback.print_exc()
        res[name] = {"error": f"{type(e).__name__}: {e}"}
    progress(name)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-plain", action="store_true", help="skip the non-compact comparator")
    ap.add_argument("--no-sweep", action="store_true", help="skip the load sweep")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-ceilings", action="store_true", help="skip the random-access ceiling probes")
    ap.add_argument("--no-iceberg", action="store_true", help="skip the iceberg sections")
    ap.add_argument("--no-many", action="store_true", help="skip the many-table section")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving-loop section")
    ap.add_argument("--only", default="",
                    help="comma list of extra sections to run beside the headline step, all others skipped "
                         "('headline' for none): " + ",".join(SECTIONS + OPT_IN) +
                         "; the OPT_IN sections (" + ",".join(OPT_IN) + ") run only when named here")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (reference kernel for HBM byte counters)")
    args = ap.parse_args()
    if args.only:
        want = set(args.only.split(",")) - {"headline"}  # "headline": the headline step alone
        unknown = want - set(SECTIONS) - set(OPT_IN)
        if unknown:
            ap.error(f"unknown sections {sorted(unknown)}")
        for sec in SECTIONS + OPT_IN:
            setattr(args, "no_" + sec, sec not in want)
    else:
        for sec in SECTIONS:
            if not hasattr(args, "no_" + sec):
                setattr(args, "no_" + sec, False)
        for sec in OPT_IN:
            setattr(args, "no_" + sec, True)

    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (this path has no multi-GPU "
              "sharding: every configuration is one GPU's share)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2406_09255_amd as cpht
    import synth

    dev = torch.device("cuda:0")
    cpht.lib()  # the HIP library must be present: no fallback

    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.int32, device=dev).fill_(1)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": a.numel() * 4, "bytes_written": b.numel() * 4,
                          "launches": 3}))
        return

    n_ins = int(LOAD * (1 << LOG2_SLOTS))
    n_max = int(0.95 * (1 << LOG2_SLOTS))
    keys64 = synth.distinct_keys(W_KEY, KEY_SEED, 0, n_max, device=dev)
    queries64 = synth.find_queries(W_KEY, KEY_SEED, n_ins, N_FIND, 0.5, Q_SEED, device=dev)
    keys = keys64.contiguous()
    queries = queries64.contiguous()
    torch.cuda.synchronize()

    compact = cpht.Table(scheme=cpht.CUCKOO, key_bits=W_KEY, log2_slots0=LOG2_SLOTS, bucket0=BUCKET,
                         slot_bits0=32, n_hash=2, max_chain=256, compact=1, seed=1)
    run = Runner(torch, cpht, compact, keys, queries, n_ins)

    for i in range(args.warmup):
        run.step(seed=1000 + i, record=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        run.step(seed=1 + i)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ins_ms, fnd_ms = run.times_ms()
    wall = t1 - t0

    # correctness guard on the last timed step (full check lives in the tests)
    outs = run.out[:n_ins]
    n_put = int((outs == cpht.PUT).sum().item())
    hit = float(run.found.float().mean().item())
    occ, cap = compact.count()
    check = "ok" if (n_put == n_ins and occ == n_ins and abs(hit - 0.5) < 0.01) else "FAILED"

    ms_step = wall * 1000.0 / args.steps
    ops = n_ins + N_FIND
    value = ops / (ms_step / 1000.0) / 1e6
    ins_avg, fnd_avg = sum(ins_ms) / len(ins_ms), sum(fnd_ms) / len(fnd_ms)
    res = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "Mops/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {
            "workload": (f"compact cuckoo H=2, 2^{LOG2_SLOTS} slots in 2^{LOG2_SLOTS - 5} buckets of 32 x 32-bit "
                         f"slots, {W_KEY}-bit keys in u64 words; per step: clear with a new seed, bulk build to "
                         f"load {LOAD} ({n_ins} keys), then 2^26 finds (50% hit / 50% miss)"),
            "slots": 1 << LOG2_SLOTS, "bucket": BUCKET, "slot_bits": 32, "key_bits": W_KEY, "load": LOAD,
            "inserts": n_ins, "finds": N_FIND, "subtile": compact.config.subtile,
        },
        "check": check,
        "insert_mops": round(n_ins / (ins_avg / 1000.0) / 1e6, 1),
        "find_mops": round(N_FIND / (fnd_avg / 1000.0) / 1e6, 1),
        "latency_ms": {
            "insert": {"p50": round(pct(ins_ms, 50), 3), "p99": round(pct(ins_ms, 99), 3)},
            "find": {"p50": round(pct(fnd_ms, 50), 3), "p99": round(pct(fnd_ms, 99), 3)},
        },
        "fill_factor": round(occ / cap, 4),
        "table_bytes": compact.level_bytes(0),
    }

    # roofline of the dominant kernel (algorithmic bytes / average launch time)
    kern = {
        "cuckoo_put": (ins_avg, n_ins * put_bytes(LOAD, 1)),
        "cuckoo_find": (fnd_avg, N_FIND * find_bytes(LOAD, 1)),
    }
    dom = max(kern, key=lambda k: kern[k][0])
    fresh = TRAFFIC["csrc_sha"] == csrc_sha()
    rl = {}
    for name, (ms, nbytes) in kern.items():
        gbs = nbytes / (ms / 1000.0) / 1e9
        rl[name] = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": TRAFFIC[name] if fresh else None,
                    "avg_ms": round(ms, 4), "algorithmic_bytes": int(nbytes),
                    "bytes_per_op": round(nbytes / (n_ins if name == "cuckoo_put" else N_FIND), 2)}
    # the put also charged with the 64-byte sector its atomic writes back
    rl["cuckoo_put"]["frac_sector_model"] = round(
        n_ins * put_bytes_sector(LOAD, 1) / (ins_avg / 1000.0) / 1e9 / HBM_PEAK_GBS, 4)
    res["roofline"] = dict(rl[dom], kernel=dom)
    res["roofline_other"] = {k: v for k, v in rl.items() if k != dom}
    del compact
    progress("headline")

    if not args.no_plain:
        plain = cpht.Table(scheme=cpht.CUCKOO, key_bits=W_KEY, log2_slots0=LOG2_SLOTS, bucket0=BUCKET,
                           slot_bits0=64, n_hash=2, max_chain=256, compact=0, seed=1)
        prun = Runner(torch, cpht, plain, keys, queries, n_ins)
        prun.step(seed=999, record=False)
        torch.cuda.synchronize()
        p0 = time.perf_counter()
        for i in range(args.steps):
            prun.step(seed=1 + i)
        torch.cuda.synchronize()
        p1 = time.perf_counter()
        pins, pfnd = prun.times_ms()
        pms = (p1 - p0) * 1000.0 / args.steps
        pi, pf = sum(pins) / len(pins), sum(pfnd) / len(pfnd)
        res["plain"] = {
            "value": round(ops / (pms / 1000.0) / 1e6, 2), "ms_per_step": round(pms, 3),
            "insert_mops": round(n_ins / (pi / 1000.0) / 1e6, 1), "find_mops": round(N_FIND / (pf / 1000.0) / 1e6, 1),
            "latency_ms": {"insert": {"p50": round(pct(pins, 50), 3), "p99": round(pct(pins, 99), 3)},
                           "find": {"p50": round(pct(pfnd, 50), 3), "p99": round(pct(pfnd, 99), 3)}},
            "slot_bits": 64, "table_bytes": plain.level_bytes(0),
        }
        res["compact_vs_plain"] = {
            "step": round(res["value"] / res["plain"]["value"], 3),
            "insert": round(res["insert_mops"] / res["plain"]["insert_mops"], 3),
            "find": round(res["find_mops"] / res["plain"]["find_mops"], 3),
            "memory": round(res["table_bytes"] / res["plain"]["table_bytes"], 3),
        }
        del plain, prun
        progress("plain")

    if not args.no_plain and not args.no_equal:
        run_section(res, "equal_memory", lambda: equal_memory(torch, cpht, keys, queries, n_ins))

    if not args.no_cachefree:
        run_section(res, "cache_free", lambda: cache_free(torch, cpht, synth, dev))

    if not args.no_window:
        run_section(res, "marginal_window", lambda: marginal_window(torch, cpht, keys, n_ins))

    if not args.no_sweep:
        loads = SWEEP_LOADS
        qs = {load: synth.find_queries(W_KEY, KEY_SEED, int(load * (1 << LOG2_SLOTS)), N_FIND, 0.5, Q_SEED + 7,
                                       device=dev) for load in loads}
        sweep = []
        for slot_bits, cmp_, bucket in SWEEP_SHAPES:
            if cmp_ == 0 and args.no_plain:
                continue
            t = cpht.Table(scheme=cpht.CUCKOO, key_bits=W_KEY, log2_slots0=LOG2_SLOTS, bucket0=bucket,
                           slot_bits0=slot_bits, n_hash=2, max_chain=256, compact=cmp_, seed=1)
            r = Runner(torch, cpht, t, keys, queries, 0)
            r.found = torch.empty(N_FIND, dtype=torch.uint8, device=dev)
            for load in loads:
                n = int(load * (1 << LOG2_SLOTS))
                r.queries = qs[load]
                for rep in range(3):
                    r.step(seed=77 + rep, n_ins=n, record=rep > 0)
                ins, fnd = r.times_ms()
                full = int((r.out[:n] == cpht.FULL).sum().item())
                sweep.append({"slot_bits": slot_bits, "compact": bool(cmp_), "bucket": bucket,
                              "bucket_bytes": bucket * slot_bits // 8, "load": load,
                              "insert_mops": round(n / (sum(ins) / len(ins) / 1000.0) / 1e6, 1),
                              "find_mops": round(N_FIND / (sum(fnd) / len(fnd) / 1000.0) / 1e6, 1),
                              "full": full})
            del t, r
        del qs
        res["sweep"] = sweep
        progress("sweep")

    if not args.no_small:
        run_section(res, "small_cuckoo", lambda: small_cuckoo(torch, cpht, synth, dev))

    if not args.no_iceberg:
        run_section(res, "iceberg_static", lambda: iceberg_static(torch, cpht, synth, dev))
        run_section(res, "iceberg_sweep", lambda: iceberg_sweep(torch, cpht, synth, dev))
        run_section(res, "iceberg_mixed", lambda: iceberg_mixed(torch, cpht, synth, dev))
        run_section(res, "iceberg_zipf", lambda: iceberg_zipf(torch, cpht, synth, dev))

    if not args.no_fop:
        run_section(res, "find_or_put", lambda: find_or_put(torch, cpht, synth, dev))

    if not args.no_delete:
        run_section(res, "delete", lambda: deletes(torch, cpht, synth, dev))

    if not args.no_level3:
        run_section(res, "level3", lambda: level3(torch, cpht, synth, dev))

    if not args.no_map:
        run_section(res, "map", lambda: kv_map(torch, cpht, synth, dev))

    if not args.no_many:
        run_section(res, "many_tables", lambda: many_tables(torch, cpht, synth, dev))

    if not args.no_serving:
        run_section(res, "serving", lambda: serving(torch, cpht, synth, dev))

    if not args.no_servingsmall:
        run_section(res, "serving_small", lambda: serving_small(torch, cpht, synth, dev))

    if not args.no_ceilings:
        run_section(res, "ceilings", lambda: ceilings(torch, cpht, dev, res, keys))
        c = res["ceilings"].get("table_size")
        if c is not None and res["roofline"]["kernel"] == "cuckoo_put":
            # one CAS per put round: the device's random line-read-then-CAS rate bounds the kernel
            res["roofline"]["atomic_ceiling"] = {
                "what": "measured random 128-B line read + 32-bit CAS into it, table-sized buffer",
                "G_per_s": c["line_read_then_cas"]["G_per_s"],
                "achieved_G_per_s": round(res["insert_mops"] * ROUNDS_PER_PUT[LOAD] / 1e3, 2),
                "frac": res["ceilings"]["put_vs_line_read_then_cas"]}

    if not args.no_cpu:
        run_section(res, "cpu_baseline", cpu_baseline)
    if not args.no_cpu_full:
        run_section(res, "cpu_full", lambda: cpu_full(torch, synth, dev))
    print(json.dumps(res))


if __name__ == "__main__":
    main()
