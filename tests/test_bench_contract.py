"""bench.py on the host: the multi-GPU request is refused with a message, and
the pieces of the roofline arithmetic behave as documented."""
import subprocess
import sys
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_algorithmic_bytes_model():
    """A put round reads its bucket's 128-byte lines and performs one 4-byte
    CAS (8 bytes for 64-bit slots); plus an 8-byte key word and a result byte.
    At load 0.9 (1.05175 rounds per put, one-line compact buckets) that is
    147.83 bytes per put; a find reads its probed buckets, key and result."""
    assert abs(bench.put_bytes(0.9, 1) - (1.05175 * (128 + 4) + 9)) < 1e-9
    assert abs(bench.put_bytes(0.9, 1) - 147.831) < 1e-3
    assert abs(bench.put_bytes(0.9, 2, 8) - (1.05175 * (256 + 8) + 9)) < 1e-9
    assert abs(bench.find_bytes(0.9, 2) - (1.22454 * 256 + 9)) < 1e-9
    # the sector model charges the 64-byte write-back instead of the 4-byte atomic
    assert abs(bench.put_bytes_sector(0.5, 1) - (1.00002 * 192 + 9)) < 1e-9


def test_roofline_fraction_reproduces_from_the_profile():
    """frac = algorithmic bytes of the put launch / its average duration / 8 TB/s.
    With the rocprofv3 average of the put kernel at the headline shape
    (profiles/cuckoo_c2_kernel_stats.md: 5.4415 ms for 120,795,955 keys)
    that is 0.41."""
    n = int(0.9 * (1 << 27))
    assert n == 120795955
    gbs = n * bench.put_bytes(0.9, 1) / 5.4415e-3 / 1e9
    assert abs(gbs / bench.HBM_PEAK_GBS - 0.41) < 0.005


def test_traffic_is_tied_to_kernel_sources():
    sha = bench.csrc_sha()
    assert len(sha) == 16 and all(c in "0123456789abcdef" for c in sha)


def test_percentiles():
    xs = list(range(1, 101))
    assert bench.pct(xs, 50) in (50, 51)
    assert bench.pct(xs, 99) == 99


def test_iceberg_overflow_rates_match_the_oracle():
    """ICE_L2 (share of inserts / finds that read both secondary buckets at
    load 0.9) comes from the sequential oracle; recount it at a smaller shape
    with the same buckets and load."""
    import numpy as np

    import oracle
    import synth

    L0, w = 16, 26  # 2^11 primary buckets, 15-bit remainders in 16-bit slots
    t = oracle.Table(oracle.ICEBERG, w, L0, 32, 16, log2_slots1=L0 - 3, B1=16, s1=32, seed=11)
    cap = (1 << L0) + (1 << (L0 - 3))
    n = int(0.9 * cap)
    keys = synth.distinct_keys(w, 0x5EED, 0, n).numpy().astype(np.uint64)
    _, lput = t.insert(keys, lines=True)
    q = synth.find_queries(w, 0x5EED, n, 1 << 15, 0.5, 3).numpy().astype(np.uint64)
    _, lfind = t.find(q, lines=True)
    assert abs((lput.mean() - 1) / 2 - bench.ICE_L2["put"]) < 0.01
    assert abs((lfind.mean() - 1) / 2 - bench.ICE_L2["find"]) < 0.02


def test_a_failing_section_is_reported_not_fatal(capsys):
    res = {}
    bench.run_section(res, "good", lambda: {"x": 1})

    def bad():
        raise RuntimeError("boom")

    bench.run_section(res, "bad", bad)
    assert res["good"] == {"x": 1}
    assert res["bad"] == {"error": "RuntimeError: boom"}
    err = capsys.readouterr().err
    assert "boom" in err and "[bench] bad done" in err


def test_iceberg_traffic_is_tied_to_iceberg_sources():
    assert bench.csrc_sha(bench.ICE_SOURCES) != bench.csrc_sha()
    assert set(bench.ICE_TRAFFIC) == {"src_sha", "insert_16_32", "find_16_32", "insert_64_64", "find_64_64"}
