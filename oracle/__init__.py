"""Python view of the sequential CPU oracle (oracle/lpht_oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline leg use it.  The product library never imports it, and it imports
nothing from the product package.

Every call applies its operations one by one in index order on a plain
linear-probing table (Sec. 4 and 5.3-5.5 of Maier, Sanders, Dementiev,
arXiv 1601.04017).  Arrays are numpy arrays: u32 keys/values for the packed
layout, u64 for the 16-byte layout.
"""
import ctypes
import os

import numpy as np

from . import build as _build

PACKED32 = 0
KV64 = 1
ASSIGN = 0
ADD = 1
FLAG_RESERVED = 0xFE
FLAG_FULL = 0xFF
STICKY_FULL = 1
STICKY_RESERVED = 2

HASH_CRC32C_PAIR = 0
HASH_MULSHIFT = 1

SEED_HI = 0x9E3779B9
SEED_LO = 0xFFFFFFFF

_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = load(_build.build(force=False))
    return _lib


def load(path):
    """Loads an oracle build from `path` and declares its C signatures."""
    L = ctypes.CDLL(path)
    u8p = ctypes.c_void_p
    L.orc_crc32c_bytes.restype = ctypes.c_uint32
    L.orc_crc32c_bytes.argtypes = [ctypes.c_uint32, ctypes.c_char_p, ctypes.c_uint64]
    L.orc_crc32c_word.restype = ctypes.c_uint32
    L.orc_crc32c_word.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int]
    L.orc_hash.restype = ctypes.c_uint64
    L.orc_hash.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32]
    L.orc_hash_bulk.restype = None
    L.orc_hash_bulk.argtypes = [u8p, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32,
                                ctypes.c_uint32, u8p]
    L.orc_home.restype = ctypes.c_uint64
    L.orc_home.argtypes = [ctypes.c_uint64, ctypes.c_uint32]
    L.orc_create.restype = ctypes.c_void_p
    L.orc_create.argtypes = [ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                             ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int]
    L.orc_destroy.argtypes = [ctypes.c_void_p]
    L.orc_capacity.restype = ctypes.c_uint64
    L.orc_capacity.argtypes = [ctypes.c_void_p]
    L.orc_log2_capacity.restype = ctypes.c_uint32
    L.orc_log2_capacity.argtypes = [ctypes.c_void_p]
    L.orc_migrations.restype = ctypes.c_uint64
    L.orc_migrations.argtypes = [ctypes.c_void_p]
    L.orc_counts.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64),
                             ctypes.POINTER(ctypes.c_uint64)]
    L.orc_status.restype = ctypes.c_int
    L.orc_status.argtypes = [ctypes.c_void_p]
    L.orc_export.argtypes = [ctypes.c_void_p, u8p]
    L.orc_import.restype = ctypes.c_int
    L.orc_import.argtypes = [ctypes.c_void_p, u8p, ctypes.c_uint32]
    L.orc_probe_count.restype = ctypes.c_uint64
    L.orc_probe_count.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
    for name in ("orc_insert",):
        f = getattr(L, name)
        f.restype = ctypes.c_int
        f.argtypes = [ctypes.c_void_p, u8p, u8p, ctypes.c_uint64, u8p]
    for name in ("orc_insert_or_update", "orc_update"):
        f = getattr(L, name)
        f.restype = ctypes.c_int
        f.argtypes = [ctypes.c_void_p, u8p, u8p, ctypes.c_uint64, ctypes.c_int, u8p]
    L.orc_find.restype = ctypes.c_int
    L.orc_find.argtypes = [ctypes.c_void_p, u8p, ctypes.c_uint64, u8p, u8p]
    L.orc_erase.restype = ctypes.c_int
    L.orc_erase.argtypes = [ctypes.c_void_p, u8p, ctypes.c_uint64, u8p]
    L.orc_grow.restype = ctypes.c_int
    L.orc_grow.argtypes = [ctypes.c_void_p, ctypes.c_uint32]
    L.orc_migrate.restype = ctypes.c_int
    L.orc_migrate.argtypes = [ctypes.c_void_p, ctypes.c_uint32]
    L.orc_str_hash.restype = ctypes.c_uint64
    L.orc_str_hash.argtypes = [u8p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32]
    L.orc_str_create.restype = ctypes.c_void_p
    L.orc_str_create.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                 ctypes.c_uint32, ctypes.c_int]
    L.orc_str_destroy.argtypes = [ctypes.c_void_p]
    L.orc_str_capacity.restype = ctypes.c_uint64
    L.orc_str_capacity.argtypes = [ctypes.c_void_p]
    L.orc_str_counts.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)]
    L.orc_str_bulk.restype = ctypes.c_int
    L.orc_str_bulk.argtypes = [ctypes.c_void_p, ctypes.c_int, u8p, u8p, ctypes.c_uint64, u8p, ctypes.c_int, u8p, u8p]
    L.orc_str_grow.restype = ctypes.c_int
    L.orc_str_grow.argtypes = [ctypes.c_void_p, ctypes.c_uint32]
    L.orc_str_cell.restype = ctypes.c_int64
    L.orc_str_cell.argtypes = [ctypes.c_void_p, ctypes.c_uint64, u8p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64)]
    L.orc_set_full_keys.restype = ctypes.c_int
    L.orc_set_full_keys.argtypes = [ctypes.c_void_p, ctypes.c_int]
    L.orc_mulshift.restype = ctypes.c_uint64
    L.orc_mulshift.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    L.orc_set_hash.restype = ctypes.c_int
    L.orc_set_hash.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64]
    L.orc_bulk_merge.restype = ctypes.c_int
    L.orc_bulk_merge.argtypes = [ctypes.c_void_p, u8p, u8p, ctypes.c_uint64, ctypes.c_int, ctypes.c_int]
    return L


def crc32c_bytes(reg: int, data: bytes) -> int:
    return lib().orc_crc32c_bytes(reg, data, len(data))


def crc32c_word(reg: int, x: int, nbytes: int) -> int:
    return lib().orc_crc32c_word(reg, x, nbytes)


def hash64(key: int, key_bytes: int, seed_hi: int = SEED_HI, seed_lo: int = SEED_LO) -> int:
    return lib().orc_hash(key, key_bytes, seed_hi, seed_lo)


def hash_bulk(keys: np.ndarray, key_bytes: int, seed_hi: int = SEED_HI,
              seed_lo: int = SEED_LO) -> np.ndarray:
    keys = np.ascontiguousarray(keys, dtype=np.uint32 if key_bytes == 4 else np.uint64)
    out = np.empty(keys.size, dtype=np.uint64)
    lib().orc_hash_bulk(keys.ctypes.data, keys.size, key_bytes, seed_hi, seed_lo, out.ctypes.data)
    return out


def mulshift(key: int, mul: int) -> int:
    """The multiplicative hash (mul * key) mod 2^64 of HASH_MULSHIFT tables."""
    return lib().orc_mulshift(key, mul)


def home(h: int, log2c: int) -> int:
    return lib().orc_home(h, log2c)


def _ptr(a):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


class OracleTable:
    """Sequential linear-probing table with the device table's cell layout."""

    def __init__(self, layout: int, log2c: int, seed_hi: int = SEED_HI, seed_lo: int = SEED_LO,
                 alpha=(1, 2), auto_grow: bool = False, full_keys: bool = False,
                 hash: int = HASH_CRC32C_PAIR, mul: int = 0):
        self.layout = layout
        self.kdt = np.uint32 if layout == PACKED32 else np.uint64
        self._t = lib().orc_create(layout, log2c, seed_hi, seed_lo, alpha[0], alpha[1],
                                   1 if auto_grow else 0)
        if not self._t:
            raise ValueError("oracle table creation failed")
        if full_keys:
            lib().orc_set_full_keys(self._t, 1)
        if hash != HASH_CRC32C_PAIR and lib().orc_set_hash(self._t, hash, mul):
            raise ValueError("bad hash choice (MULSHIFT needs an odd multiplier)")

    def __del__(self):
        t = getattr(self, "_t", None)
        if t:
            lib().orc_destroy(t)
            self._t = None

    # -- metadata
    @property
    def capacity(self) -> int:
        return lib().orc_capacity(self._t)

    @property
    def log2c(self) -> int:
        return lib().orc_log2_capacity(self._t)

    @property
    def migrations(self) -> int:
        return lib().orc_migrations(self._t)

    def counts(self):
        u = ctypes.c_uint64()
        l = ctypes.c_uint64()
        lib().orc_counts(self._t, ctypes.byref(u), ctypes.byref(l))
        return u.value, l.value

    def status(self) -> int:
        return lib().orc_status(self._t)

    def cells(self) -> np.ndarray:
        wpc = 1 if self.layout == PACKED32 else 2
        out = np.empty(self.capacity * wpc, dtype=np.uint64)
        lib().orc_export(self._t, _ptr(out))
        return out

    def load_cells(self, cells: np.ndarray, log2c: int):
        cells = np.ascontiguousarray(cells, dtype=np.uint64)
        wpc = 1 if self.layout == PACKED32 else 2
        assert cells.size == (1 << log2c) * wpc
        rc = lib().orc_import(self._t, _ptr(cells), log2c)
        if rc:
            raise RuntimeError(f"orc_import failed: {rc}")

    def probe_count(self, key: int) -> int:
        return lib().orc_probe_count(self._t, key)

    # -- bulk operations
    def _keys(self, keys):
        return np.ascontiguousarray(keys, dtype=self.kdt)

    def insert(self, keys, vals=None):
        keys = self._keys(keys)
        vals = None if vals is None else np.ascontiguousarray(vals, dtype=self.kdt)
        flags = np.empty(keys.size, dtype=np.uint8)
        rc = lib().orc_insert(self._t, _ptr(keys), _ptr(vals), keys.size, _ptr(flags))
        if rc:
            raise RuntimeError(f"orc_insert failed: {rc}")
        return flags

    def insert_or_update(self, keys, vals=None, op=ADD):
        keys = self._keys(keys)
        vals = None if vals is None else np.ascontiguousarray(vals, dtype=self.kdt)
        flags = np.empty(keys.size, dtype=np.uint8)
        rc = lib().orc_insert_or_update(self._t, _ptr(keys), _ptr(vals), keys.size, op, _ptr(flags))
        if rc:
            raise RuntimeError(f"orc_insert_or_update failed: {rc}")
        return flags

    def update(self, keys, vals=None, op=ASSIGN):
        keys = self._keys(keys)
        vals = None if vals is None else np.ascontiguousarray(vals, dtype=self.kdt)
        flags = np.empty(keys.size, dtype=np.uint8)
        lib().orc_update(self._t, _ptr(keys), _ptr(vals), keys.size, op, _ptr(flags))
        return flags

    def find(self, keys):
        keys = self._keys(keys)
        vals = np.empty(keys.size, dtype=self.kdt)
        found = np.empty(keys.size, dtype=np.uint8)
        lib().orc_find(self._t, _ptr(keys), keys.size, _ptr(vals), _ptr(found))
        return vals, found

    def erase(self, keys):
        keys = self._keys(keys)
        flags = np.empty(keys.size, dtype=np.uint8)
        lib().orc_erase(self._t, _ptr(keys), keys.size, _ptr(flags))
        return flags

    def grow(self, log2_new: int):
        rc = lib().orc_grow(self._t, log2_new)
        if rc:
            raise RuntimeError(f"orc_grow failed: {rc}")

    def build(self, keys, vals=None, op=ASSIGN):
        """Replaces the contents by the batch (sort-based bulk build, Sec. 5.5)."""
        self._bulk(keys, vals, op, 0)

    def merge(self, keys, vals=None, op=ASSIGN):
        """Merges the batch into the table (sort-based batched merge, Sec. 5.5)."""
        self._bulk(keys, vals, op, 1)

    def _bulk(self, keys, vals, op, keep_old):
        keys = self._keys(keys)
        vals = None if vals is None else np.ascontiguousarray(vals, dtype=self.kdt)
        rc = lib().orc_bulk_merge(self._t, _ptr(keys), _ptr(vals), keys.size, op, keep_old)
        if rc:
            raise RuntimeError(f"orc_bulk_merge failed: {rc}")


def pack_strings(strings):
    """A list of bytes -> (bytes buffer u8, offsets u64 with n + 1 entries)."""
    offs = np.zeros(len(strings) + 1, dtype=np.uint64)
    offs[1:] = np.cumsum([len(x) for x in strings], dtype=np.uint64)
    buf = np.frombuffer(b"".join(strings), dtype=np.uint8).copy() if strings else np.zeros(0, dtype=np.uint8)
    if buf.size == 0:
        buf = np.zeros(1, dtype=np.uint8)
    return buf, offs


def str_hash(s: bytes, seed_hi: int = SEED_HI, seed_lo: int = SEED_LO) -> int:
    b = np.frombuffer(s, dtype=np.uint8).copy() if s else np.zeros(1, dtype=np.uint8)
    return lib().orc_str_hash(b.ctypes.data, len(s), seed_hi, seed_lo)


class OracleStrTable:
    """Sequential linear-probing table with byte-string keys and u64 values."""

    def __init__(self, log2c: int, seed_hi: int = SEED_HI, seed_lo: int = SEED_LO, alpha=(1, 2),
                 auto_grow: bool = False):
        self._t = lib().orc_str_create(log2c, seed_hi, seed_lo, alpha[0], alpha[1], 1 if auto_grow else 0)
        if not self._t:
            raise ValueError("oracle table creation failed")

    def __del__(self):
        t = getattr(self, "_t", None)
        if t and lib is not None:
            lib().orc_str_destroy(t)
            self._t = None

    @property
    def capacity(self) -> int:
        return lib().orc_str_capacity(self._t)

    def counts(self):
        u, l = ctypes.c_uint64(), ctypes.c_uint64()
        lib().orc_str_counts(self._t, ctypes.byref(u), ctypes.byref(l))
        return u.value, l.value

    def _bulk(self, kind, strings, vals=None, op=ASSIGN):
        buf, offs = pack_strings(strings)
        n = len(strings)
        v = None if vals is None else np.ascontiguousarray(vals, dtype=np.uint64)
        out = np.zeros(max(n, 1), dtype=np.uint64)
        flags = np.zeros(max(n, 1), dtype=np.uint8)
        rc = lib().orc_str_bulk(self._t, kind, buf.ctypes.data, offs.ctypes.data, n,
                                None if v is None else v.ctypes.data, op, out.ctypes.data, flags.ctypes.data)
        if rc:
            raise RuntimeError(f"orc_str_bulk failed: {rc}")
        return flags[:n], out[:n]

    def insert(self, strings, vals=None):
        return self._bulk(0, strings, vals)[0]

    def insert_or_update(self, strings, vals=None, op=ADD):
        return self._bulk(1, strings, vals, op)[0]

    def find(self, strings):
        f, v = self._bulk(2, strings)
        return v, f

    def erase(self, strings):
        return self._bulk(3, strings)[0]

    def grow(self, log2_new: int):
        rc = lib().orc_str_grow(self._t, log2_new)
        if rc:
            raise RuntimeError(f"orc_str_grow failed: {rc}")

    def cells(self):
        """Per cell: None (empty), False (tombstone) or (key bytes, value)."""
        out = []
        buf = np.zeros(1 << 16, dtype=np.uint8)
        for i in range(self.capacity):
            v = ctypes.c_uint64()
            ln = lib().orc_str_cell(self._t, i, buf.ctypes.data, buf.size, ctypes.byref(v))
            out.append(None if ln == -1 else False if ln == -2 else (bytes(buf[:ln]), v.value))
        return out
