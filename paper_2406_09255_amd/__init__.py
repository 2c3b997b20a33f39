"""Compact parallel hash tables on AMD MI355X (gfx950): Python binding.

A thin ctypes layer over ``libcpht.so`` (the C-ABI declared in
``include/cpht.h``).  It only marshals arguments: torch tensors supply device
buffers and the current HIP stream; every step of insert, find, count and the
key split runs in the library's own HIP kernels.  There is no fallback: if the
library is missing or a call fails, an exception is raised.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcpht.so")

CUCKOO, ICEBERG = 0, 1
PUT, FOUND, FULL = 1, 2, 3
OP_FIND, OP_INSERT = 0, 1

_STATUS = {
    0: "ok", 1: "invalid argument", 2: "out of device memory", 3: "unsupported configuration",
    4: "key out of range", 5: "device error", 6: "busy", 7: "operation not valid for this table",
}


class CphtError(RuntimeError):
    def __init__(self, code: int, call: str):
        super().__init__(f"{call}: {_STATUS.get(code, code)} (status {code})")
        self.code = code


class Config(ctypes.Structure):
    """Mirror of cpht_config_t."""

    _fields_ = [
        ("scheme", ctypes.c_uint32),
        ("key_bits", ctypes.c_uint32),
        ("log2_slots0", ctypes.c_uint32),
        ("log2_slots1", ctypes.c_uint32),
        ("bucket0", ctypes.c_uint32),
        ("bucket1", ctypes.c_uint32),
        ("slot_bits0", ctypes.c_uint32),
        ("slot_bits1", ctypes.c_uint32),
        ("n_hash", ctypes.c_uint32),
        ("max_chain", ctypes.c_uint32),
        ("subtile", ctypes.c_uint32),
        ("compact", ctypes.c_uint32),
        ("log2_lists", ctypes.c_uint32),
        ("pool_slabs", ctypes.c_uint32),
        ("value_bytes", ctypes.c_uint32),
        ("pad", ctypes.c_uint32),
        ("seed", ctypes.c_uint64),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None

# Every symbol include/cpht.h declares, with (restype, argtypes).
_VP, _U32, _U64, _I32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
_SIGNATURES = {
    "cpht_config_default": (None, [_U32, ctypes.POINTER(Config)]),
    "cpht_config_check": (_I32, [ctypes.POINTER(Config), ctypes.POINTER(Config)]),
    "cpht_create": (_I32, [ctypes.POINTER(Config), ctypes.POINTER(_VP)]),
    "cpht_destroy": (_I32, [_VP]),
    "cpht_get_config": (_I32, [_VP, ctypes.POINTER(Config)]),
    "cpht_clear": (_I32, [_VP, _U64, _VP]),
    "cpht_insert": (_I32, [_VP, _VP, _U64, _VP, _VP]),
    "cpht_bulk_build": (_I32, [_VP, _VP, _U64, _VP, _VP]),
    "cpht_find": (_I32, [_VP, _VP, _U64, _VP, _VP]),
    "cpht_mixed": (_I32, [_VP, _VP, _VP, _U64, _VP, _VP]),
    "cpht_delete": (_I32, [_VP, _VP, _U64, _VP, _VP]),
    "cpht_insert_values": (_I32, [_VP, _VP, _VP, _U64, _VP, _VP]),
    "cpht_find_values": (_I32, [_VP, _VP, _U64, _VP, _VP, _VP]),
    "cpht_values_bytes": (_I32, [_VP, _U32, ctypes.POINTER(_U64)]),
    "cpht_export_values": (_I32, [_VP, _U32, _VP, _U64]),
    "cpht_import_values": (_I32, [_VP, _U32, _VP, _U64]),
    "cpht_import": (_I32, [_VP, _U32, _VP, _U64]),
    "cpht_sorted_fop": (_I32, [_VP, _VP, _U64, _VP, _VP, _U64, _VP]),
    "cpht_sorted_fop_workspace": (_I32, [_VP, _U64, ctypes.POINTER(_U64)]),
    "cpht_sorted_fop_noalloc": (_I32, [_VP, _VP, _U64, _VP, _VP]),
    "cpht_count": (_I32, [_VP, ctypes.POINTER(_U64), ctypes.POINTER(_U64), _VP]),
    "cpht_level_bytes": (_I32, [_VP, _U32, ctypes.POINTER(_U64)]),
    "cpht_level3_used": (_I32, [_VP, ctypes.POINTER(_U32)]),
    "cpht_level_ptr": (_I32, [_VP, _U32, ctypes.POINTER(_VP)]),
    "cpht_export": (_I32, [_VP, _U32, _VP, _U64]),
    "cpht_split": (_I32, [_VP, _U32, _VP, _U64, _VP, _VP, _VP]),
    "cpht_variant_info": (_I32, [_U32, _I32, ctypes.POINTER(_U32)]),
    "cpht_probe": (_I32, [_U32, _VP, _U64, _U64, _U64, _VP, ctypes.POINTER(_U64), _VP]),
    "cpht_server_config_default": (None, [_VP]),
    "cpht_server_start": (_I32, [_VP, _VP, ctypes.POINTER(_VP)]),
    "cpht_server_submit": (_I32, [_VP, _VP, _VP, _U64, _VP, ctypes.POINTER(_U64)]),
    "cpht_server_poll": (_I32, [_VP, _U64, ctypes.POINTER(_I32), ctypes.POINTER(_U64)]),
    "cpht_server_wait": (_I32, [_VP, _U64, ctypes.POINTER(_U64)]),
    "cpht_server_stats": (_I32, [_VP, ctypes.POINTER(_U64), ctypes.POINTER(_U64), ctypes.POINTER(_U64),
                                 ctypes.POINTER(_U64)]),
    "cpht_server_stop": (_I32, [_VP]),
    "cpht_server_replay": (_I32, [_VP, _U64, _VP, _VP, _VP, _VP, _VP, _VP, ctypes.POINTER(_U64)]),
    "cpht_multi_create": (_I32, [_U32, _VP, _U64, ctypes.POINTER(_VP)]),
    "cpht_multi_destroy": (_I32, [_VP]),
    "cpht_multi_table": (_I32, [_VP, _U32, ctypes.POINTER(_VP)]),
    "cpht_multi_clear": (_I32, [_VP, _VP]),
    "cpht_multi_insert": (_I32, [_VP, _VP, _VP, _U64, _VP, _VP]),
    "cpht_multi_find": (_I32, [_VP, _VP, _VP, _U64, _VP, _VP]),
    "cpht_multi_info": (_I32, [_VP, ctypes.POINTER(_U64), ctypes.POINTER(_U32), ctypes.POINTER(_U64)]),
    "cpht_multi_error": (_I32, [_VP, ctypes.POINTER(_U32)]),
    "cpht_status_str": (ctypes.c_char_p, [_I32]),
}


def lib():
    """Load libcpht.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2406_09255_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(code: int, call: str):
    if code != 0:
        raise CphtError(code, call)


def _stream(stream) -> int | None:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else stream


def _dev_ptr(t: torch.Tensor, name: str) -> int:
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t.data_ptr()


def default_config(scheme: int) -> Config:
    c = Config()
    lib().cpht_config_default(scheme, ctypes.byref(c))
    return c


def check_config(cfg: Config) -> Config | None:
    """The resolved configuration if the library accepts `cfg`, else None
    (no device memory is touched)."""
    out = Config()
    return out if lib().cpht_config_check(ctypes.byref(cfg), ctypes.byref(out)) == 0 else None


def variants(scheme: int) -> list[dict]:
    """Compiled kernel variants of a scheme."""
    n = lib().cpht_variant_info(scheme, -1, None)
    out = []
    buf = (_U32 * 6)()
    for i in range(n):
        lib().cpht_variant_info(scheme, i, buf)
        out.append(dict(zip(("key64", "slot_bits0", "slot_bits1", "bucket0", "bucket1", "subtile"), list(buf))))
    return out


PROBE_LINES, PROBE_CAS, PROBE_LINE_CAS, PROBE_CAS64, PROBE_SPLIT, PROBE_HALF_LINES, PROBE_LINES_NT = range(7)


def probe(kind: int, buf: torch.Tensor, ops: int, seed: int, sink: torch.Tensor, stream=None) -> int:
    """Launch a random-access roofline probe on `buf`; returns operations issued."""
    done = _U64(0)
    _check(lib().cpht_probe(kind, _dev_ptr(buf, "buf"), buf.numel() * buf.element_size(), ops, seed,
                            _dev_ptr(sink, "sink"), ctypes.byref(done), _stream(stream)), "cpht_probe")
    return done.value


class Table:
    """One compact hash table resident in device memory (cpht_table_t)."""

    @classmethod
    def _view(cls, handle, owner) -> "Table":
        t = cls.__new__(cls)
        t._h = handle
        t._owner = owner  # keeps the table set alive; views are never destroyed
        t.config = Config()
        _check(lib().cpht_get_config(t._h, ctypes.byref(t.config)), "cpht_get_config")
        return t

    def __init__(self, config: Config | None = None, **fields):
        scheme = fields.get("scheme", config.scheme if config is not None else CUCKOO)
        cfg = Config()
        if config is not None:
            ctypes.memmove(ctypes.byref(cfg), ctypes.byref(config), ctypes.sizeof(Config))
        else:
            lib().cpht_config_default(scheme, ctypes.byref(cfg))
        for k, v in fields.items():
            setattr(cfg, k, int(v))
        h = _VP()
        _check(lib().cpht_create(ctypes.byref(cfg), ctypes.byref(h)), "cpht_create")
        self._h = h
        self.config = Config()
        _check(lib().cpht_get_config(self._h, ctypes.byref(self.config)), "cpht_get_config")

    # -- lifetime -----------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) and getattr(self, "_owner", None) is None:
            lib().cpht_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- properties ---------------------------------------------------------
    @property
    def key_dtype(self) -> torch.dtype:
        return torch.int32 if self.config.key_bits <= 32 else torch.int64

    @property
    def nlevels(self) -> int:
        return 2 if self.config.scheme == ICEBERG else 1

    @property
    def nimages(self) -> int:
        """Exported images: the bucket levels, then (third level) pool and heads."""
        return self.nlevels + (2 if self.config.pool_slabs else 0)

    def level3_used(self) -> int:
        """Slabs taken from the third level's pool so far."""
        v = _U32(0)
        _check(lib().cpht_level3_used(self._h, ctypes.byref(v)), "cpht_level3_used")
        return v.value

    def _keys(self, keys: torch.Tensor) -> int:
        if keys.dtype != self.key_dtype:
            raise ValueError(f"keys must be {self.key_dtype} words for key_bits={self.config.key_bits}")
        return _dev_ptr(keys, "keys")

    def _out(self, out: torch.Tensor | None, n: int, like: torch.Tensor) -> torch.Tensor:
        if out is None:
            out = torch.empty(n, dtype=torch.uint8, device=like.device)
        if out.dtype != torch.uint8 or out.numel() < n:
            raise ValueError("out must be a uint8 device tensor with one byte per key")
        return out

    # -- batch operations (asynchronous on the stream) ----------------------
    def clear(self, seed: int | None = None, stream=None):
        s = self.config.seed if seed is None else seed
        _check(lib().cpht_clear(self._h, s & (2**64 - 1), _stream(stream)), "cpht_clear")
        self.config.seed = s & (2**64 - 1)

    def insert(self, keys: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        n = keys.numel()
        out = self._out(out, n, keys)
        _check(lib().cpht_insert(self._h, self._keys(keys), n, _dev_ptr(out, "out"), _stream(stream)),
               "cpht_insert")
        return out

    def bulk_build(self, keys: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        n = keys.numel()
        out = self._out(out, n, keys)
        _check(lib().cpht_bulk_build(self._h, self._keys(keys), n, _dev_ptr(out, "out"), _stream(stream)),
               "cpht_bulk_build")
        return out

    def find(self, keys: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        n = keys.numel()
        out = self._out(out, n, keys)
        _check(lib().cpht_find(self._h, self._keys(keys), n, _dev_ptr(out, "out"), _stream(stream)),
               "cpht_find")
        return out

    def mixed(self, keys: torch.Tensor, ops: torch.Tensor, out: torch.Tensor | None = None,
              stream=None) -> torch.Tensor:
        n = keys.numel()
        if ops.dtype != torch.uint8 or ops.numel() != n:
            raise ValueError("ops must be a uint8 tensor with one opcode per key")
        out = self._out(out, n, keys)
        _check(lib().cpht_mixed(self._h, self._keys(keys), _dev_ptr(ops, "ops"), n, _dev_ptr(out, "out"),
                                _stream(stream)), "cpht_mixed")
        return out

    def delete(self, keys: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """Delete by tombstone: out[i] = 1 if this call removed keys[i]."""
        n = keys.numel()
        out = self._out(out, n, keys)
        _check(lib().cpht_delete(self._h, self._keys(keys), n, _dev_ptr(out, "out"), _stream(stream)),
               "cpht_delete")
        return out

    def _values(self, values: torch.Tensor, n: int) -> int:
        vb = self.config.value_bytes
        want = torch.int64 if vb == 8 else torch.int32
        if values.dtype != want or values.numel() < n:
            raise ValueError(f"values must be a {want} device tensor with one value per key (value_bytes={vb})")
        return _dev_ptr(values, "values")

    def insert_values(self, keys: torch.Tensor, values: torch.Tensor, out: torch.Tensor | None = None,
                      stream=None) -> torch.Tensor:
        """Map find-or-put: the insert that stores keys[i] writes values[i]."""
        n = keys.numel()
        out = self._out(out, n, keys)
        _check(lib().cpht_insert_values(self._h, self._keys(keys), self._values(values, n), n,
                                        _dev_ptr(out, "out"), _stream(stream)), "cpht_insert_values")
        return out

    def find_values(self, keys: torch.Tensor, found: torch.Tensor | None = None, values: torch.Tensor | None = None,
                    stream=None):
        """Map lookup: (found, values); values of keys not found are left as given (zero when allocated here)."""
        n = keys.numel()
        found = self._out(found, n, keys)
        if values is None:
            values = torch.zeros(n, dtype=torch.int64 if self.config.value_bytes == 8 else torch.int32,
                                 device=keys.device)
        _check(lib().cpht_find_values(self._h, self._keys(keys), n, _dev_ptr(found, "found"),
                                      self._values(values, n), _stream(stream)), "cpht_find_values")
        return found, values

    def import_image(self, level: int, image) -> None:
        """Restore image `level` from a host array written by export (checkpoint / resume)."""
        import numpy as np  # host staging buffer only

        buf = np.ascontiguousarray(image, dtype=np.uint8)
        _check(lib().cpht_import(self._h, level, buf.ctypes.data_as(_VP), buf.size), "cpht_import")

    def import_values(self, level: int, values) -> None:
        import numpy as np  # host staging buffer only

        buf = np.ascontiguousarray(values, dtype=np.uint8)
        _check(lib().cpht_import_values(self._h, level, buf.ctypes.data_as(_VP), buf.size), "cpht_import_values")

    def checkpoint(self) -> dict:
        """Configuration and every image (and value array) in host memory."""
        state = {"config": self.config.as_dict(), "images": [self.export(x) for x in range(self.nimages)]}
        if self.config.value_bytes:
            state["values"] = [self.export_values(x) for x in range(3 if self.config.pool_slabs else 2)]
        return state

    @classmethod
    def restore(cls, state: dict) -> "Table":
        """A new table with the checkpoint's configuration and contents."""
        t = cls(**state["config"])
        for x, img in enumerate(state["images"]):
            t.import_image(x, img)
        for x, v in enumerate(state.get("values", [])):
            t.import_values(x, v)
        return t

    def export_values(self, level: int):
        """Value array of level 0, 1 or 2 (third-level pool) in host memory (numpy uint8)."""
        import numpy as np  # host staging buffer only

        b = _U64(0)
        _check(lib().cpht_values_bytes(self._h, level, ctypes.byref(b)), "cpht_values_bytes")
        buf = np.empty(b.value, dtype=np.uint8)
        _check(lib().cpht_export_values(self._h, level, buf.ctypes.data_as(_VP), b.value), "cpht_export_values")
        return buf

    def sorted_fop_workspace(self, n: int) -> int:
        b = _U64(0)
        _check(lib().cpht_sorted_fop_workspace(self._h, n, ctypes.byref(b)), "cpht_sorted_fop_workspace")
        return b.value

    def sorted_fop(self, keys: torch.Tensor, out: torch.Tensor | None = None, workspace: torch.Tensor | None = None,
                   stream=None) -> torch.Tensor:
        """Cuckoo find-or-put by sorting the batch (duplicates and stored keys
        allowed).  `workspace`: a uint8 device tensor of at least
        sorted_fop_workspace(n) bytes, allocated here when not given."""
        n = keys.numel()
        out = self._out(out, n, keys)
        need = self.sorted_fop_workspace(n)
        if workspace is None:
            workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=keys.device)
            if stream is not None:
                # allocated on the current stream, used on `stream`: keep the caching
                # allocator from handing it out again before `stream` is done with it
                s = stream if isinstance(stream, torch.cuda.Stream) else torch.cuda.ExternalStream(stream)
                workspace.record_stream(s)
        if workspace.dtype != torch.uint8 or workspace.numel() < need:
            raise ValueError(f"workspace must be a uint8 device tensor of at least {need} bytes")
        _check(lib().cpht_sorted_fop(self._h, self._keys(keys), n, _dev_ptr(out, "out"),
                                     _dev_ptr(workspace, "workspace"), workspace.numel(), _stream(stream)),
               "cpht_sorted_fop")
        return out

    def sorted_fop_noalloc(self, keys: torch.Tensor, out: torch.Tensor, stream=None) -> torch.Tensor:
        """sorted_fop without a workspace: the library's fixed per-GPU scratch
        is used and nothing is allocated (n <= 2^20; `out` is required)."""
        n = keys.numel()
        if out is None:
            raise ValueError("out is required (the call allocates nothing)")
        out = self._out(out, n, keys)
        _check(lib().cpht_sorted_fop_noalloc(self._h, self._keys(keys), n, _dev_ptr(out, "out"), _stream(stream)),
               "cpht_sorted_fop_noalloc")
        return out

    def split(self, perm_index: int, keys: torch.Tensor, stream=None):
        n = keys.numel()
        addr = torch.empty(n, dtype=torch.int64, device=keys.device)
        stored = torch.empty(n, dtype=torch.int64, device=keys.device)
        _check(lib().cpht_split(self._h, perm_index, self._keys(keys), n, _dev_ptr(addr, "addr"),
                                _dev_ptr(stored, "stored"), _stream(stream)), "cpht_split")
        return addr, stored

    # -- synchronous queries ------------------------------------------------
    def count(self, stream=None) -> tuple[int, int]:
        occ, cap = _U64(0), _U64(0)
        _check(lib().cpht_count(self._h, ctypes.byref(occ), ctypes.byref(cap), _stream(stream)), "cpht_count")
        return occ.value, cap.value

    def fill_factor(self, stream=None) -> float:
        occ, cap = self.count(stream)
        return occ / cap

    def level_bytes(self, level: int) -> int:
        b = _U64(0)
        _check(lib().cpht_level_bytes(self._h, level, ctypes.byref(b)), "cpht_level_bytes")
        return b.value

    def level_ptr(self, level: int) -> int:
        """Device address of image `level` (for callers that read it themselves)."""
        p = _VP()
        _check(lib().cpht_level_ptr(self._h, level, ctypes.byref(p)), "cpht_level_ptr")
        return p.value or 0

    def export(self, level: int):
        """Raw slot image of a level in host memory (numpy uint8)."""
        import numpy as np  # host staging buffer only

        nbytes = self.level_bytes(level)
        buf = np.empty(nbytes, dtype=np.uint8)
        _check(lib().cpht_export(self._h, level, buf.ctypes.data_as(_VP), nbytes), "cpht_export")
        return buf


class MultiTable:
    """A set of independent tables served by one launch per kernel variant
    (cpht_multi_t).  `table_configs` is a list of Config (one key width for all); batches are CSR: the keys
    of all tables concatenated plus int64 device offsets (n + 1)."""

    def __init__(self, table_configs, max_keys: int):
        arr = (Config * len(table_configs))()
        for i, c in enumerate(table_configs):
            ctypes.memmove(ctypes.byref(arr[i]), ctypes.byref(c), ctypes.sizeof(Config))
        h = _VP()
        _check(lib().cpht_multi_create(len(table_configs), ctypes.cast(arr, _VP), max_keys, ctypes.byref(h)),
               "cpht_multi_create")
        self._h = h
        self.n = len(table_configs)
        self.key_dtype = torch.int32 if table_configs[0].key_bits <= 32 else torch.int64

    def close(self):
        if getattr(self, "_h", None):
            lib().cpht_multi_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def table(self, i: int) -> Table:
        v = _VP()
        _check(lib().cpht_multi_table(self._h, i, ctypes.byref(v)), "cpht_multi_table")
        return Table._view(v, self)

    def info(self) -> dict:
        a, g, c = _U64(0), _U32(0), _U64(0)
        _check(lib().cpht_multi_info(self._h, ctypes.byref(a), ctypes.byref(g), ctypes.byref(c)), "cpht_multi_info")
        return {"arena_bytes": a.value, "groups": g.value, "max_chunks": c.value}

    def clear(self, stream=None):
        _check(lib().cpht_multi_clear(self._h, _stream(stream)), "cpht_multi_clear")

    def _run(self, fn, name, keys, offsets, out, stream):
        if keys.dtype != self.key_dtype:
            raise ValueError(f"keys must be {self.key_dtype}")
        if offsets.dtype != torch.int64 or offsets.numel() != self.n + 1:
            raise ValueError("offsets must be int64 with n_tables + 1 entries")
        n = keys.numel()
        if out is None:
            out = torch.empty(n, dtype=torch.uint8, device=keys.device)
        if out.dtype != torch.uint8 or out.numel() < n:
            raise ValueError("out must be a uint8 device tensor with one byte per key")
        _check(fn(self._h, _dev_ptr(keys, "keys"), _dev_ptr(offsets, "offsets"), n, _dev_ptr(out, "out"),
                  _stream(stream)), name)
        return out

    def insert(self, keys, offsets, out=None, stream=None):
        return self._run(lib().cpht_multi_insert, "cpht_multi_insert", keys, offsets, out, stream)

    def find(self, keys, offsets, out=None, stream=None):
        return self._run(lib().cpht_multi_find, "cpht_multi_find", keys, offsets, out, stream)

    def error_flags(self) -> int:
        f = _U32(0)
        _check(lib().cpht_multi_error(self._h, ctypes.byref(f)), "cpht_multi_error")
        return f.value


class ServerConfig(ctypes.Structure):
    """Mirror of cpht_server_config_t."""

    _fields_ = [
        ("max_inflight", ctypes.c_uint32),
        ("coalesce", ctypes.c_uint32),
        ("staging_keys", ctypes.c_uint64),
        ("max_batch_keys", ctypes.c_uint64),
        ("zero_copy", ctypes.c_uint32),
        ("resident", ctypes.c_uint32),
        ("idle_us", ctypes.c_uint32),
        ("pad", ctypes.c_uint32),
    ]


def _host_ptr(t, name: str) -> int:
    if t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous host tensor (pinned for asynchronous copies)")
    return t.data_ptr()


class Server:
    """Continuous-batching request loop over one iceberg table (cpht_server_t).
    Request buffers are host tensors (pinned: tensor.pin_memory(); required
    with zero_copy=1, where the device reads and writes them in place) that
    must stay alive until the request completes."""

    def __init__(self, table: Table, **fields):
        cfg = ServerConfig()
        lib().cpht_server_config_default(ctypes.byref(cfg))
        for k, v in fields.items():
            setattr(cfg, k, int(v))
        h = _VP()
        _check(lib().cpht_server_start(table._h, ctypes.byref(cfg), ctypes.byref(h)), "cpht_server_start")
        self._h, self._table, self.config = h, table, cfg
        self._keep = {}

    def submit(self, keys, ops, out) -> int:
        if keys.dtype != self._table.key_dtype:
            raise ValueError(f"keys must be {self._table.key_dtype}")
        n = keys.numel()
        if ops.numel() != n or out.numel() < n or ops.dtype != torch.uint8 or out.dtype != torch.uint8:
            raise ValueError("ops and out must be uint8 with one entry per key")
        tk = _U64(0)
        _check(lib().cpht_server_submit(self._h, _host_ptr(keys, "keys"), _host_ptr(ops, "ops"), n,
                                        _host_ptr(out, "out"), ctypes.byref(tk)), "cpht_server_submit")
        self._keep[tk.value] = (keys, ops, out)
        return tk.value

    def poll(self, ticket: int):
        d, lat = _I32(0), _U64(0)
        _check(lib().cpht_server_poll(self._h, ticket, ctypes.byref(d), ctypes.byref(lat)), "cpht_server_poll")
        if d.value:
            self._keep.pop(ticket, None)
        return bool(d.value), lat.value

    def wait(self, ticket: int) -> int:
        lat = _U64(0)
        _check(lib().cpht_server_wait(self._h, ticket, ctypes.byref(lat)), "cpht_server_wait")
        self._keep.pop(ticket, None)
        return lat.value

    def stats(self) -> dict:
        v = [_U64(0) for _ in range(4)]
        _check(lib().cpht_server_stats(self._h, *[ctypes.byref(x) for x in v]), "cpht_server_stats")
        return dict(zip(("launches", "requests_done", "ops_done", "max_queue"), (x.value for x in v)))

    def replay(self, arrival_ns, offsets, keys, ops, out):
        """Replay a trace (see cpht_server_replay); returns (latency_ns array, makespan_ns)."""
        import numpy as np

        arr = np.ascontiguousarray(np.asarray(arrival_ns, dtype=np.uint64))
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.uint64))
        if keys.dtype != self._table.key_dtype:
            raise ValueError(f"keys must be {self._table.key_dtype}")
        if off.size != arr.size + 1 or (arr.size and int(off[0]) != 0):
            raise ValueError("offsets must hold n_requests + 1 entries starting at 0")
        if arr.size and int(off[-1]) > min(keys.numel(), ops.numel(), out.numel()):
            raise ValueError("offsets reach past the key, opcode or result buffer")
        if ops.dtype != torch.uint8 or out.dtype != torch.uint8:
            raise ValueError("ops and out must be uint8")
        lat = np.zeros(arr.size, dtype=np.uint64)
        mk = _U64(0)
        _check(lib().cpht_server_replay(self._h, arr.size, arr.ctypes.data_as(_VP), off.ctypes.data_as(_VP),
                                        _host_ptr(keys, "keys"), _host_ptr(ops, "ops"), _host_ptr(out, "out"),
                                        lat.ctypes.data_as(_VP), ctypes.byref(mk)), "cpht_server_replay")
        return lat, mk.value

    def stop(self):
        if getattr(self, "_h", None):
            h, self._h = self._h, None
            _check(lib().cpht_server_stop(h), "cpht_server_stop")
            self._keep.clear()

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass
