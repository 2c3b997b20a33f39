"""Sequential CPU oracle for compact cuckoo and compact iceberg hash tables.

TEST INFRASTRUCTURE ONLY: the GPU library is checked against this package.
Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import it; the library itself never does, and this package
never imports the library.

Two layers, both following "Compact Parallel Hash Tables on the GPU"
(arXiv 2406.09255):

* ``sets``: the plain definition of what a batch computes -- set membership
  for finds, and for inserts PUT exactly once per new key and FOUND otherwise
  (Theorem 1 (c), (d) and the corollary closing Appendix A).  Written with
  numpy sort/unique as the only library steps.
* ``liboracle.so`` (``cpht_oracle.c``): the sequential scheme model -- the
  quotienting permutation (Sec. 2.4), iceberg find-or-put as Alg. 5 over the
  slot order of Definition 1, the iceberg lookup of Sec. 2.3, compact cuckoo
  put (Alg. 4) and lookup (Sec. 4.4), and the table checker of Definition 2.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cpht_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

CUCKOO, ICEBERG = 0, 1
NONE, PUT, FOUND, FULL = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-fPIC", "-shared", _SRC, "-o", tmp]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Cfg(ctypes.Structure):
    """Mirror of or_cfg_t in cpht_oracle.c."""

    _fields_ = [
        ("scheme", ctypes.c_uint32),
        ("w", ctypes.c_uint32),
        ("log2_slots0", ctypes.c_uint32),
        ("log2_slots1", ctypes.c_uint32),
        ("B0", ctypes.c_uint32),
        ("B1", ctypes.c_uint32),
        ("s0", ctypes.c_uint32),
        ("s1", ctypes.c_uint32),
        ("H", ctypes.c_uint32),
        ("C", ctypes.c_uint32),
        ("compact", ctypes.c_uint32),
        ("log2_lists", ctypes.c_uint32),
        ("pool_slabs", ctypes.c_uint32),
        ("pad", ctypes.c_uint32),
        ("seed", ctypes.c_uint64),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        L = ctypes.CDLL(_LIB_PATH)
        u64, u32, i32 = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
        vp = ctypes.c_void_p
        L.or_mix64.restype = u64
        L.or_mix64.argtypes = [u64]
        L.or_sm64.restype = u64
        L.or_sm64.argtypes = [u64, u64]
        L.or_mulinv.restype = u64
        L.or_mulinv.argtypes = [u64, u32]
        L.or_perm_apply.restype = i32
        L.or_perm_apply.argtypes = [u32, u64, u32, i32, vp, vp, u64]
        L.or_perm_constants.restype = i32
        L.or_perm_constants.argtypes = [u32, u64, u32, vp, vp, vp]
        L.or_order_less.restype = i32
        L.or_order_less.argtypes = [u32, u32, u32, u32]
        L.or_order_list.restype = i32
        L.or_order_list.argtypes = [u32, u32, vp, vp]
        L.or_new.restype = vp
        L.or_new.argtypes = [ctypes.POINTER(Cfg)]
        L.or_free.restype = None
        L.or_free.argtypes = [vp]
        L.or_insert.restype = i32
        L.or_insert.argtypes = [vp, vp, u64, vp, vp]
        L.or_find.restype = i32
        L.or_find.argtypes = [vp, vp, u64, vp, vp]
        L.or_mixed.restype = i32
        L.or_mixed.argtypes = [vp, vp, vp, u64, vp]
        L.or_occupied.restype = u64
        L.or_occupied.argtypes = [vp]
        L.or_tombstones.restype = u64
        L.or_tombstones.argtypes = [vp]
        L.or_delete.restype = i32
        L.or_delete.argtypes = [vp, vp, u64, vp]
        L.or_capacity.restype = u64
        L.or_capacity.argtypes = [vp]
        L.or_level_bytes.restype = u64
        L.or_level_bytes.argtypes = [vp, i32]
        L.or_export.restype = i32
        L.or_export.argtypes = [vp, i32, vp, u64]
        L.or_check.restype = i32
        L.or_check.argtypes = [ctypes.POINTER(Cfg), vp, vp, vp, ctypes.POINTER(u64), ctypes.c_char_p, i32]
        L.or_check3.restype = i32
        L.or_check3.argtypes = [ctypes.POINTER(Cfg), vp, vp, vp, vp, vp, ctypes.POINTER(u64), ctypes.c_char_p, i32]
        L.or_l3_used.restype = ctypes.c_uint32
        L.or_l3_used.argtypes = [vp]
        L.or_bucket_of.restype = u64
        L.or_bucket_of.argtypes = [vp, i32, u32, u64]
        L.or_stored_form.restype = u64
        L.or_stored_form.argtypes = [vp, i32, u32, u64, u64]
        L.or_max_key_bits.restype = u32
        L.or_max_key_bits.argtypes = [u32, u32, u32, u32, u32]
        L.or_split_array.restype = i32
        L.or_split_array.argtypes = [vp, u32, vp, u64, vp, vp]
        L.or_check_full.restype = i32
        L.or_check_full.argtypes = [ctypes.POINTER(Cfg), vp, vp, vp, u64, ctypes.c_char_p, i32]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _u64(keys) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(keys).astype(np.uint64, copy=False))


# -- splitmix64 and the permutations (Sec. 2.4) ------------------------------

def sm64(seed: int, i: int) -> int:
    return int(lib().or_sm64(seed & (2**64 - 1), i))


def mix64(z: int) -> int:
    return int(lib().or_mix64(z & (2**64 - 1)))


def mulinv(m: int, w: int) -> int:
    return int(lib().or_mulinv(m, w))


def perm(w: int, seed: int, i: int, x, inverse: bool = False) -> np.ndarray:
    """pi_i (or its inverse) of the w-bit permutation family seeded by seed."""
    x = _u64(x)
    out = np.empty_like(x)
    rc = lib().or_perm_apply(w, seed & (2**64 - 1), i, int(inverse), _ptr(x), _ptr(out), x.size)
    if rc:
        raise ValueError("bad permutation arguments")
    return out


def perm_constants(w: int, seed: int, i: int):
    m = np.zeros(3, np.uint64)
    minv = np.zeros(3, np.uint64)
    c = np.zeros(3, np.uint64)
    if lib().or_perm_constants(w, seed & (2**64 - 1), i, _ptr(m), _ptr(minv), _ptr(c)):
        raise ValueError("bad permutation arguments")
    return m, minv, c


def split(w: int, nb: int, seed: int, i: int, x):
    """(address, remainder) of keys under pi_i: high nb bits / low w-nb bits."""
    y = perm(w, seed, i, x)
    r = y & np.uint64((1 << (w - nb)) - 1) if w - nb < 64 else y
    a = (y >> np.uint64(w - nb)) if nb > 0 else np.zeros_like(y)
    return a, r


def max_key_bits(log2_slots: int, B: int, s: int, tag_bits: int, compact: bool = True) -> int:
    """Widest key a level can hold (address bits + remainder room)."""
    return int(lib().or_max_key_bits(log2_slots, B, s, tag_bits, int(compact)))


def order_less(a, b) -> bool:
    return bool(lib().or_order_less(a[0], a[1], b[0], b[1]))


def order_list(B0: int, B1: int):
    n = B0 + 2 * B1
    xs = np.zeros(n, np.uint32)
    ys = np.zeros(n, np.uint32)
    m = lib().or_order_list(B0, B1, _ptr(xs), _ptr(ys))
    return [(int(xs[i]), int(ys[i])) for i in range(m)]


# -- sequential table model ---------------------------------------------------

class Table:
    """A host-memory table driven one operation at a time."""

    def __init__(self, scheme, w, log2_slots0, B0, s0, log2_slots1=0, B1=0, s1=32,
                 H=2, C=256, compact=True, seed=1, log2_lists=0, pool_slabs=0):
        self.cfg = Cfg(scheme=scheme, w=w, log2_slots0=log2_slots0, log2_slots1=log2_slots1,
                       B0=B0, B1=B1, s0=s0, s1=s1, H=H, C=C, compact=int(compact), log2_lists=log2_lists,
                       pool_slabs=pool_slabs, pad=0, seed=seed & (2**64 - 1))
        self._h = lib().or_new(ctypes.byref(self.cfg))
        if not self._h:
            raise ValueError("oracle rejected the table configuration")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and callable(lib):  # module globals may already be gone at interpreter exit
            lib().or_free(h)
            self._h = None

    @property
    def nlevels(self):
        return 2 if self.cfg.scheme == ICEBERG else 1

    def insert(self, keys, lines: bool = False):
        k = _u64(keys)
        out = np.zeros(k.size, np.uint8)
        ln = np.zeros(k.size, np.uint32) if lines else None
        lib().or_insert(self._h, _ptr(k), k.size, _ptr(out), _ptr(ln) if lines else None)
        return (out, ln) if lines else out

    def find(self, keys, lines: bool = False):
        k = _u64(keys)
        out = np.zeros(k.size, np.uint8)
        ln = np.zeros(k.size, np.uint32) if lines else None
        lib().or_find(self._h, _ptr(k), k.size, _ptr(out), _ptr(ln) if lines else None)
        return (out, ln) if lines else out

    def mixed(self, keys, ops):
        k = _u64(keys)
        o = np.ascontiguousarray(np.asarray(ops, np.uint8))
        out = np.zeros(k.size, np.uint8)
        if lib().or_mixed(self._h, _ptr(k), _ptr(o), k.size, _ptr(out)):
            raise ValueError("mixed batches need an iceberg table")
        return out

    def delete(self, keys):
        """Delete by tombstone, in order: 1 where the key was stored, else 0."""
        k = _u64(keys)
        out = np.zeros(k.size, np.uint8)
        lib().or_delete(self._h, _ptr(k), k.size, _ptr(out))
        return out

    def occupied(self) -> int:
        return int(lib().or_occupied(self._h))

    def tombstones(self) -> int:
        return int(lib().or_tombstones(self._h))

    def capacity(self) -> int:
        return int(lib().or_capacity(self._h))

    def export(self, level: int) -> np.ndarray:
        nbytes = int(lib().or_level_bytes(self._h, level))
        buf = np.zeros(nbytes, np.uint8)
        if lib().or_export(self._h, level, _ptr(buf), nbytes):
            raise ValueError("bad level")
        return buf

    def bucket_of(self, level: int, i: int, k: int) -> int:
        return int(lib().or_bucket_of(self._h, level, i, k))

    def stored_form(self, level: int, i: int, k: int, tag: int) -> int:
        return int(lib().or_stored_form(self._h, level, i, k, tag))

    def split(self, i: int, keys):
        """(address, stored form) of keys under permutation i (see or_split_array)."""
        k = _u64(keys)
        a = np.zeros(k.size, np.uint64)
        e = np.zeros(k.size, np.uint64)
        if lib().or_split_array(self._h, i, _ptr(k), k.size, _ptr(a), _ptr(e)):
            raise ValueError("bad permutation index")
        return a, e

    def l3_used(self) -> int:
        """Slabs of the third level handed out so far."""
        return int(lib().or_l3_used(self._h))

    def check(self):
        imgs = [self.export(x) for x in range(self.nlevels)]
        if self.cfg.pool_slabs:
            imgs += [self.export(2), self.export(3)]
        return check_images(self.cfg, *imgs)


def check_images(cfg: Cfg, img0: np.ndarray, img1: np.ndarray | None = None, pool: np.ndarray | None = None,
                 heads: np.ndarray | None = None):
    """Run the table checker over raw level images (`pool` and `heads`: the
    third level's slab pool and list heads, when the table has one).

    Returns (ok, message, sorted decoded key array)."""
    img0 = np.ascontiguousarray(img0, dtype=np.uint8)
    cap = img0.size * 8 // max(1, cfg.s0)
    if img1 is not None:
        img1 = np.ascontiguousarray(img1, dtype=np.uint8)
        cap += img1.size * 8 // max(1, cfg.s1)
    if pool is not None:
        pool = np.ascontiguousarray(pool, dtype=np.uint8)
        heads = np.ascontiguousarray(heads, dtype=np.uint8)
        cap += pool.size * 8 // 32
    keys = np.zeros(max(1, cap), np.uint64)
    nk = ctypes.c_uint64(0)
    msg = ctypes.create_string_buffer(512)
    rc = lib().or_check3(ctypes.byref(cfg), _ptr(img0), _ptr(img1) if img1 is not None else None,
                         _ptr(pool) if pool is not None else None, _ptr(heads) if heads is not None else None,
                         _ptr(keys), ctypes.byref(nk), msg, 512)
    if rc < 0:
        raise ValueError("checker rejected the configuration")
    return rc == 0, msg.value.decode(), keys[: nk.value].copy()


def check_full(cfg: Cfg, img0: np.ndarray, img1: np.ndarray, full_keys) -> tuple[bool, str]:
    """Theorem 1 (e): keys answered FULL are absent and their buckets full."""
    k = _u64(full_keys)
    img0 = np.ascontiguousarray(img0, dtype=np.uint8)
    img1 = np.ascontiguousarray(img1, dtype=np.uint8)
    msg = ctypes.create_string_buffer(512)
    rc = lib().or_check_full(ctypes.byref(cfg), _ptr(img0), _ptr(img1), _ptr(k), k.size, msg, 512)
    if rc < 0:
        raise ValueError("checker rejected the configuration")
    return rc == 0, msg.value.decode()


from . import sets  # noqa: E402,F401  (plain set-semantics definition)
