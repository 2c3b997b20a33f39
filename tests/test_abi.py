"""The C ABI library without a GPU: it loads, exports every function the
public header declares, and validates arguments before touching the device."""
import ctypes
import os
import re

import pytest

import paper_2406_09255_amd as cpht

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "cpht.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cpht_[a-z_0-9]+)\s*\(", src)))


def test_header_symbols_exported():
    L = cpht.lib()
    names = declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n


def test_binding_covers_header():
    assert sorted(cpht._SIGNATURES) == declared()


def test_status_strings_and_defaults():
    assert cpht.lib().cpht_status_str(0) == b"ok"
    assert cpht.lib().cpht_status_str(3) == b"unsupported configuration"
    c = cpht.default_config(cpht.ICEBERG)
    assert (c.bucket0, c.bucket1, c.slot_bits0, c.slot_bits1) == (32, 16, 16, 32)
    c = cpht.default_config(cpht.CUCKOO)
    assert (c.bucket0, c.slot_bits0, c.n_hash, c.max_chain) == (32, 32, 2, 256)


def test_variant_table():
    ice = cpht.variants(cpht.ICEBERG)
    ck = cpht.variants(cpht.CUCKOO)
    assert any(v["bucket0"] == 32 and v["slot_bits0"] == 16 and v["slot_bits1"] == 32 for v in ice)
    assert any(v["bucket0"] == 32 and v["slot_bits0"] == 32 and v["key64"] == 1 for v in ck)
    for v in ice:
        assert v["bucket1"] * 2 == v["bucket0"]
        assert v["bucket0"] * v["slot_bits0"] % (32 * v["subtile"]) == 0


@pytest.mark.parametrize("fields", [
    dict(scheme=cpht.CUCKOO, key_bits=40, log2_slots0=12, bucket0=32, slot_bits0=32),  # remainder too wide
    dict(scheme=cpht.CUCKOO, key_bits=32, log2_slots0=12, bucket0=32, slot_bits0=16),  # no 16-bit cuckoo
    dict(scheme=cpht.ICEBERG, key_bits=34, log2_slots0=10, log2_slots1=7, bucket0=32, bucket1=16,
         slot_bits0=16, slot_bits1=32),
    dict(scheme=cpht.ICEBERG, key_bits=20, log2_slots0=12, log2_slots1=9, bucket0=32, bucket1=8,
         slot_bits0=32, slot_bits1=32),  # bucket1 must be bucket0 / 2
    dict(scheme=cpht.CUCKOO, key_bits=32, log2_slots0=12, bucket0=24, slot_bits0=32),  # not a power of two
])
def test_unsupported_configurations_rejected_before_device_use(fields):
    with pytest.raises(cpht.CphtError) as e:
        cpht.Table(**fields)
    assert e.value.code == 3


def test_null_arguments():
    L = cpht.lib()
    assert L.cpht_create(None, None) == 1
    assert L.cpht_destroy(None) == 1
    assert L.cpht_find(None, None, 0, None, None) == 1


def test_every_entry_point_rejects_null_arguments():
    """Every call returning a status answers CPHT_E_ARG to null handles and
    pointers (zero sizes), before touching any device."""
    L = cpht.lib()
    ints = (ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int)
    checked = 0
    for name, (res, args) in sorted(cpht._SIGNATURES.items()):
        if res is not cpht._I32 or name == "cpht_variant_info":  # variant_info returns a count
            continue
        vals = [0 if a in ints else None for a in args]
        assert getattr(L, name)(*vals) == 1, name
        checked += 1
    assert checked >= 40
