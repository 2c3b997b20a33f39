"""The roofline probes (cpht_probe) and raw level access: the measurement
kernels touch only their buffer and issue the operations they report, and a
level's device address reads back as its exported image."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest
import torch

import paper_2406_09255_amd as cpht
import synth

pytestmark = pytest.mark.gpu


def test_probe_cas_writes_only_claimed_words(gpu):
    buf = torch.zeros(1 << 20, dtype=torch.int32, device=gpu)  # 4 MiB
    sink = torch.zeros(1, dtype=torch.int32, device=gpu)
    done = cpht.probe(cpht.PROBE_CAS, buf, 1 << 16, 7, sink)
    torch.cuda.synchronize()
    assert done == 1 << 16
    nz = buf[buf != 0]
    assert 0 < nz.numel() <= done
    assert bool(((nz & 1) == 1).all())  # every claimed word holds an odd lane tag
    before = buf.clone()
    cpht.probe(cpht.PROBE_LINES, buf, 1 << 16, 8, sink)  # reads leave the buffer alone
    torch.cuda.synchronize()
    assert torch.equal(buf, before)
    cpht.probe(cpht.PROBE_LINE_CAS, buf, 1 << 16, 9, sink)
    torch.cuda.synchronize()
    assert int((buf != 0).sum()) >= nz.numel()


def test_probe_cas64_and_split(gpu):
    """64-bit CAS claims 8-byte words with odd tags and nothing else; the
    split probe reads its keys and leaves them alone."""
    buf = torch.zeros(1 << 19, dtype=torch.int64, device=gpu)  # 4 MiB
    sink = torch.zeros(1, dtype=torch.int32, device=gpu)
    done = cpht.probe(cpht.PROBE_CAS64, buf, 1 << 16, 11, sink)
    torch.cuda.synchronize()
    assert done == 1 << 16
    nz = buf[buf != 0]
    assert 0 < nz.numel() <= done
    assert bool(((nz & 1) == 1).all())
    keys = synth.distinct_keys(37, 5, 0, 1 << 18, device=gpu).contiguous()
    before = keys.clone()
    done = cpht.probe(cpht.PROBE_SPLIT, keys, 1 << 20, 3, sink)
    torch.cuda.synchronize()
    assert done == 1 << 20
    assert torch.equal(keys, before)


def test_probe_half_line_and_nontemporal_reads_leave_the_buffer(gpu):
    buf = torch.arange(1 << 20, dtype=torch.int32, device=gpu)  # 4 MiB
    sink = torch.zeros(1, dtype=torch.int32, device=gpu)
    before = buf.clone()
    for kind in (cpht.PROBE_HALF_LINES, cpht.PROBE_LINES_NT):
        done = cpht.probe(kind, buf, 1 << 16, 13, sink)
        torch.cuda.synchronize()
        assert done == 1 << 16
    assert torch.equal(buf, before)


def test_probe_rejects_bad_buffers(gpu):
    sink = torch.zeros(1, dtype=torch.int32, device=gpu)
    with pytest.raises(cpht.CphtError):  # not a power of two
        cpht.probe(cpht.PROBE_LINES, torch.zeros(3000, dtype=torch.int32, device=gpu), 1024, 1, sink)
    with pytest.raises(cpht.CphtError):  # no operations
        cpht.probe(cpht.PROBE_LINES, torch.zeros(4096, dtype=torch.int32, device=gpu), 0, 1, sink)
    with pytest.raises(cpht.CphtError):  # no such probe
        cpht.probe(7, torch.zeros(4096, dtype=torch.int32, device=gpu), 1024, 1, sink)


def test_level_ptr_reads_back_the_image(gpu):
    w = 30
    t = cpht.Table(scheme=cpht.ICEBERG, key_bits=w, log2_slots0=14, log2_slots1=11, bucket0=32, bucket1=16,
                   slot_bits0=32, slot_bits1=32, seed=4)
    t.insert(synth.to_words(synth.distinct_keys(w, 3, 0, 10000, device=gpu), w))
    torch.cuda.synchronize()
    ptrs = [t.level_ptr(x) for x in range(t.nimages)]
    assert all(ptrs) and len(set(ptrs)) == len(ptrs)
    hip = ctypes.CDLL("libamdhip64.so")  # the runtime the library and torch share
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    device_to_device = 3
    for x, p in enumerate(ptrs):
        nbytes = t.level_bytes(x)
        dev = torch.empty(nbytes, dtype=torch.uint8, device=gpu)
        assert hip.hipMemcpy(dev.data_ptr(), p, nbytes, device_to_device) == 0
        assert np.array_equal(dev.cpu().numpy(), t.export(x))
    with pytest.raises(cpht.CphtError):
        t.level_ptr(t.nimages)
