"""ctypes binding of liblpht.so (C ABI in include/lpht.h).

Argument marshalling only: every table operation runs in the library's HIP
kernels.  Device arrays are torch tensors on the table's GPU (any integer
dtype of the right width; keys and values are bit patterns), streams are torch
streams.  If the library is missing this module raises instead of falling
back to anything else.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import sys
import weakref

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "liblpht.so")

OK = 0
ERR_INVALID = -1
ERR_OOM = -2
ERR_FULL = -3
ERR_RESERVED_KEY = -4
ERR_DEVICE = -5
ERR_UNSUPPORTED = -6

FLAG_RESERVED = 0xFE
FLAG_FULL = 0xFF

PACKED32 = 0
KV64 = 1
ASSIGN = 0
ADD = 1

HASH_CRC32C_PAIR = 0
HASH_MULSHIFT = 1

SEED_HI = 0x9E3779B9
SEED_LO = 0xFFFFFFFF

_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)


class lpht_config(ctypes.Structure):
    _fields_ = [
        ("layout", ctypes.c_uint32),
        ("log2_capacity", ctypes.c_uint32),
        ("seed_hi", ctypes.c_uint32),
        ("seed_lo", ctypes.c_uint32),
        ("max_fill_num", ctypes.c_uint32),
        ("max_fill_den", ctypes.c_uint32),
        ("auto_grow", ctypes.c_uint32),
        ("full_keys", ctypes.c_uint32),
        ("hash", ctypes.c_uint32),
        ("reserved0", ctypes.c_uint32),
        ("mul", ctypes.c_uint64),
        ("alloc", _ALLOC_FN),
        ("free", _FREE_FN),
        ("alloc_ctx", ctypes.c_void_p),
    ]


class lpht_tuning(ctypes.Structure):
    _fields_ = [
        ("block_threads", ctypes.c_uint32),
        ("group_width", ctypes.c_uint32),
        ("blocks_per_cu", ctypes.c_uint32),
        ("migrate_block", ctypes.c_uint32),
        ("aggregate", ctypes.c_uint32),
        ("g_find", ctypes.c_uint8 * 4),
        ("g_modify", ctypes.c_uint8 * 4),
        ("reserved", ctypes.c_uint32),
    ]


class lpht_autotune_report(ctypes.Structure):
    _fields_ = [
        ("find_ms", (ctypes.c_double * 5) * 4),
        ("insert_ms", (ctypes.c_double * 5) * 4),
        ("block_ms", ctypes.c_double * 3),
        ("migrate_ms", ctypes.c_double * 4),
    ]

TUNING_KEYS = ("block_threads", "group_width", "blocks_per_cu", "migrate_block", "aggregate",
               "g_find", "g_modify")


class lpht_stats(ctypes.Structure):
    _fields_ = [
        ("migrations", ctypes.c_uint64),
        ("resizes", ctypes.c_uint64),
        ("cells_migrated", ctypes.c_uint64),
        ("host_syncs", ctypes.c_uint64),
        ("migrate_ms", ctypes.c_double),
        ("shrinks", ctypes.c_uint64),
        ("bulk_merges", ctypes.c_uint64),
        ("async_growths", ctypes.c_uint64),
        ("async_fallbacks", ctypes.c_uint64),
    ]


class lpht_batch_op(ctypes.Structure):
    _fields_ = [
        ("table", ctypes.c_void_p),
        ("op", ctypes.c_uint32),
        ("up", ctypes.c_uint32),
        ("keys", ctypes.c_void_p),
        ("vals", ctypes.c_void_p),
        ("n", ctypes.c_uint64),
        ("vals_out", ctypes.c_void_p),
        ("flags", ctypes.c_void_p),
        ("kinds", ctypes.c_void_p),
        ("kind_sel", ctypes.c_uint32),
        ("count_sel", ctypes.c_uint32),
    ]


OP_FIND, OP_INSERT, OP_UPSERT, OP_UPDATE, OP_ERASE = 0, 1, 2, 3, 4

# name -> (restype, argtypes); names are the C ABI's
_VP = ctypes.c_void_p
_U64 = ctypes.c_uint64
_U32 = ctypes.c_uint32
_SIGS = {
    "lpht_config_default": (None, [ctypes.POINTER(lpht_config)]),
    "lpht_create": (ctypes.c_int, [ctypes.POINTER(lpht_config), _VP, ctypes.POINTER(_VP)]),
    "lpht_destroy": (ctypes.c_int, [_VP, _VP]),
    "lpht_clear": (ctypes.c_int, [_VP, _VP]),
    "lpht_insert": (ctypes.c_int, [_VP, _VP, _VP, _U64, _VP, _VP]),
    "lpht_find": (ctypes.c_int, [_VP, _VP, _U64, _VP, _VP, _VP]),
    "lpht_insert_or_update": (ctypes.c_int, [_VP, _VP, _VP, _U64, _U32, _VP, _VP]),
    "lpht_update": (ctypes.c_int, [_VP, _VP, _VP, _U64, _U32, _VP, _VP]),
    "lpht_erase": (ctypes.c_int, [_VP, _VP, _U64, _VP, _VP]),
    "lpht_grow": (ctypes.c_int, [_VP, _U32, _VP]),
    "lpht_build": (ctypes.c_int, [_VP, _VP, _VP, _U64, _U32, _VP]),
    "lpht_build_noalloc": (ctypes.c_int, [_VP, _VP, _VP, _U64, _U32, _VP]),
    "lpht_insert_async": (ctypes.c_int, [_VP, _VP, _VP, _U64, _U32, _VP, _VP]),
    "lpht_merge": (ctypes.c_int, [_VP, _VP, _VP, _U64, _U32, _VP]),
    "lpht_count": (ctypes.c_int, [_VP, ctypes.POINTER(_U64), ctypes.POINTER(_U64), _VP]),
    "lpht_capacity": (ctypes.c_int, [_VP, ctypes.POINTER(_U64), ctypes.POINTER(_U32)]),
    "lpht_cell_bytes": (_U32, [_U32]),
    "lpht_export_cells": (ctypes.c_int, [_VP, _VP, _VP]),
    "lpht_import_cells": (ctypes.c_int, [_VP, _VP, _U32, _VP]),
    "lpht_status": (ctypes.c_int, [_VP, _VP]),
    "lpht_set_tuning": (ctypes.c_int, [_VP, ctypes.POINTER(lpht_tuning)]),
    "lpht_autotune": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, _VP,
                                     ctypes.POINTER(lpht_tuning), ctypes.POINTER(lpht_autotune_report)]),
    "lpht_get_tuning": (ctypes.c_int, [_VP, ctypes.POINTER(lpht_tuning)]),
    "lpht_set_timing": (ctypes.c_int, [_VP, ctypes.c_int]),
    "lpht_get_stats": (ctypes.c_int, [_VP, ctypes.POINTER(lpht_stats)]),
    "lpht_batch_create": (ctypes.c_int, [_U32, ctypes.POINTER(_VP)]),
    "lpht_batch_destroy": (ctypes.c_int, [_VP]),
    "lpht_batch_run": (ctypes.c_int, [_VP, ctypes.POINTER(lpht_batch_op), _U32, _VP]),
    "lpht_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "lpht_version": (ctypes.c_char_p, []),
    "lpht_release_pools": (ctypes.c_int, []),
}

_lib = None


# Every open library object, so that the exit hook can close them in order
# (servers, then batches, then tables) while the HIP runtime is still whole.
_live = weakref.WeakValueDictionary()
_live_seq = [0]


def _track(obj):
    _live_seq[0] += 1
    _live[_live_seq[0]] = obj


def shutdown():
    """Closes every open server, batch and table of this process, then
    returns the library's pool memory (lpht_release_pools).  Registered with
    atexit when the library is loaded; may also be called directly."""
    if _lib is None:
        return
    objs = [o for _, o in sorted(_live.items())]
    for kind in (Server, Batch, StrTable, Table):
        for o in reversed(objs):
            if isinstance(o, kind):
                try:
                    o.close()
                except Exception:  # noqa: BLE001 - best effort at exit
                    pass
    if "torch" in sys.modules:
        import torch
        if torch.cuda.is_initialized():
            torch.cuda.synchronize()
    _lib.lpht_release_pools()


def load(path: str = LIB_PATH):
    """Loads liblpht.so and declares its signatures.  Raises if it is absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"liblpht.so not built ({path}); run python -m paper_1601_04017_amd.build")
        # torch first: its wheel carries its own HIP runtime (same soname as
        # the one liblpht.so was linked against), and loaded first it is the
        # one liblpht.so binds to.  Loaded after liblpht.so, the process would
        # hold two HIP runtimes, and torch's streams and errors would live in
        # the other one.  Also, atexit runs its hooks last-registered first,
        # so the hook below runs before torch's own exit handlers.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(path)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
        atexit.register(shutdown)
    return _lib


def exported_symbols():
    return list(_SIGS) + list(_STR_SIGS)


class LphtError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        msg = load().lpht_strerror(code).decode()
        super().__init__(f"{what}: {msg} ({code})" if what else f"{msg} ({code})")


def _check(rc: int, what: str):
    if rc != OK:
        raise LphtError(rc, what)


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return ctypes.c_void_p(t.data_ptr())


class Table:
    """One device table.  Methods map one-to-one onto the C ABI calls."""

    def __init__(self, layout: int = KV64, log2_capacity: int = 12, auto_grow: bool = False,
                 seed_hi: int = SEED_HI, seed_lo: int = SEED_LO, alpha=(1, 2), stream=None,
                 full_keys: bool = False, hash: int = HASH_CRC32C_PAIR, mul: int = 0):
        import torch
        L = load()
        self.layout = layout
        self.word = 4 if layout == PACKED32 else 8
        self.torch_dtype = torch.int32 if layout == PACKED32 else torch.int64
        cfg = lpht_config()
        L.lpht_config_default(ctypes.byref(cfg))
        cfg.layout = layout
        cfg.log2_capacity = log2_capacity
        cfg.seed_hi = seed_hi
        cfg.seed_lo = seed_lo
        cfg.max_fill_num, cfg.max_fill_den = alpha
        cfg.auto_grow = 1 if auto_grow else 0
        cfg.full_keys = 1 if full_keys else 0
        cfg.hash = hash
        cfg.mul = mul
        h = ctypes.c_void_p()
        self._stream = stream
        _check(L.lpht_create(ctypes.byref(cfg), _stream_handle(stream), ctypes.byref(h)), "lpht_create")
        self._h = h
        _track(self)

    def close(self, stream=None):
        if getattr(self, "_h", None):
            load().lpht_destroy(self._h, _stream_handle(stream if stream is not None else self._stream))
            self._h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # bound at definition: module globals may be gone during teardown,
        # when the exit hook has closed everything and no HIP call may follow
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def clear(self, stream=None):
        _check(load().lpht_clear(self._h, _stream_handle(stream)), "lpht_clear")

    # ---- helpers
    def _n(self, keys):
        if keys.element_size() != self.word:
            raise ValueError(f"keys must be {self.word}-byte integers")
        return keys.numel()

    def _flags(self, n, want):
        import torch
        return torch.empty(n, dtype=torch.uint8, device="cuda") if want else None

    # ---- operations (stream-ordered; results are device tensors)
    def insert(self, keys, vals=None, flags=True, stream=None):
        n = self._n(keys)
        f = self._flags(n, flags)
        _check(load().lpht_insert(self._h, _ptr(keys), _ptr(vals), n, _ptr(f), _stream_handle(stream)),
               "lpht_insert")
        return f

    def find(self, keys, vals_out=None, found=None, stream=None):
        import torch
        n = self._n(keys)
        if vals_out is None:
            vals_out = torch.empty(n, dtype=self.torch_dtype, device="cuda")
        if found is None:
            found = torch.empty(n, dtype=torch.uint8, device="cuda")
        _check(load().lpht_find(self._h, _ptr(keys), n, _ptr(vals_out), _ptr(found),
                                _stream_handle(stream)), "lpht_find")
        return vals_out, found

    def insert_or_update(self, keys, vals=None, op=ADD, flags=True, stream=None):
        n = self._n(keys)
        f = self._flags(n, flags)
        _check(load().lpht_insert_or_update(self._h, _ptr(keys), _ptr(vals), n, op, _ptr(f),
                                            _stream_handle(stream)), "lpht_insert_or_update")
        return f

    def update(self, keys, vals=None, op=ASSIGN, flags=True, stream=None):
        n = self._n(keys)
        f = self._flags(n, flags)
        _check(load().lpht_update(self._h, _ptr(keys), _ptr(vals), n, op, _ptr(f),
                                  _stream_handle(stream)), "lpht_update")
        return f

    def erase(self, keys, flags=True, stream=None):
        n = self._n(keys)
        f = self._flags(n, flags)
        _check(load().lpht_erase(self._h, _ptr(keys), n, _ptr(f), _stream_handle(stream)), "lpht_erase")
        return f

    def grow(self, log2_new: int, stream=None):
        _check(load().lpht_grow(self._h, log2_new, _stream_handle(stream)), "lpht_grow")

    def insert_async(self, keys, vals=None, add=False, flags=True, stream=None):
        """Insertion (or insert-or-add) that grows the table inside the kernel."""
        n = self._n(keys)
        f = self._flags(n, flags)
        _check(load().lpht_insert_async(self._h, _ptr(keys), _ptr(vals), n, 1 if add else 0, _ptr(f),
                                        _stream_handle(stream)), "lpht_insert_async")
        return f

    def build(self, keys, vals=None, op=ASSIGN, stream=None):
        """Sort-based bulk build: the table's contents become the batch."""
        n = self._n(keys)
        _check(load().lpht_build(self._h, _ptr(keys), _ptr(vals), n, op, _stream_handle(stream)), "lpht_build")

    def build_noalloc(self, keys, vals=None, op=ASSIGN, stream=None):
        """lpht_build with the library's fixed scratch, in place: no device
        allocation; returns the status code (no exception)."""
        n = self._n(keys)
        return load().lpht_build_noalloc(self._h, _ptr(keys), _ptr(vals), n, op, _stream_handle(stream))

    def merge(self, keys, vals=None, op=ASSIGN, stream=None):
        """Sort-based batched merge of the batch into the table."""
        n = self._n(keys)
        _check(load().lpht_merge(self._h, _ptr(keys), _ptr(vals), n, op, _stream_handle(stream)), "lpht_merge")

    def count(self, stream=None):
        u, l = ctypes.c_uint64(), ctypes.c_uint64()
        _check(load().lpht_count(self._h, ctypes.byref(u), ctypes.byref(l), _stream_handle(stream)),
               "lpht_count")
        return u.value, l.value

    @property
    def capacity(self) -> int:
        c, lg = ctypes.c_uint64(), ctypes.c_uint32()
        _check(load().lpht_capacity(self._h, ctypes.byref(c), ctypes.byref(lg)), "lpht_capacity")
        return c.value

    @property
    def log2_capacity(self) -> int:
        c, lg = ctypes.c_uint64(), ctypes.c_uint32()
        _check(load().lpht_capacity(self._h, ctypes.byref(c), ctypes.byref(lg)), "lpht_capacity")
        return lg.value

    def export_cells(self, stream=None):
        """Raw cells as an int64 device tensor: one word per cell (PACKED32)
        or key, value words (KV64)."""
        import torch
        words = self.capacity * (1 if self.layout == PACKED32 else 2)
        out = torch.empty(words, dtype=torch.int64, device="cuda")
        _check(load().lpht_export_cells(self._h, _ptr(out), _stream_handle(stream)), "lpht_export_cells")
        return out

    def import_cells(self, cells, log2_capacity: int, stream=None):
        _check(load().lpht_import_cells(self._h, _ptr(cells), log2_capacity, _stream_handle(stream)),
               "lpht_import_cells")

    def status(self, stream=None) -> int:
        return load().lpht_status(self._h, _stream_handle(stream))

    def set_tuning(self, block_threads=256, group_width=1, blocks_per_cu=8, migrate_block=512,
                   aggregate=1, g_find=(0, 0, 0, 0), g_modify=(0, 0, 0, 0)):
        """Launch shape; g_find / g_modify: group width by fill quarter (0 = group_width)."""
        t = _tuning_struct(dict(block_threads=block_threads, group_width=group_width,
                                blocks_per_cu=blocks_per_cu, migrate_block=migrate_block,
                                aggregate=aggregate, g_find=g_find, g_modify=g_modify))
        _check(load().lpht_set_tuning(self._h, ctypes.byref(t)), "lpht_set_tuning")

    def apply_tuning(self, tuning: dict):
        """Sets a tuning dict as returned by autotune() or get_tuning()."""
        self.set_tuning(**{k: tuning[k] for k in TUNING_KEYS if k in tuning})

    def get_tuning(self) -> dict:
        t = lpht_tuning()
        _check(load().lpht_get_tuning(self._h, ctypes.byref(t)), "lpht_get_tuning")
        return _tuning_dict(t)

    def set_timing(self, on: bool = True):
        _check(load().lpht_set_timing(self._h, 1 if on else 0), "lpht_set_timing")

    def stats(self) -> dict:
        s = lpht_stats()
        _check(load().lpht_get_stats(self._h, ctypes.byref(s)), "lpht_get_stats")
        return {k: getattr(s, k) for k, _ in lpht_stats._fields_}


def _tuning_struct(d: dict) -> "lpht_tuning":
    t = lpht_tuning(d["block_threads"], d["group_width"], d["blocks_per_cu"], d["migrate_block"],
                    d["aggregate"])
    for i in range(4):
        t.g_find[i] = int(d.get("g_find", (0,) * 4)[i])
        t.g_modify[i] = int(d.get("g_modify", (0,) * 4)[i])
    return t


def _tuning_dict(t: "lpht_tuning") -> dict:
    d = {k: getattr(t, k) for k in TUNING_KEYS[:5]}
    d["g_find"] = [int(x) for x in t.g_find]
    d["g_modify"] = [int(x) for x in t.g_modify]
    return d


def _cache_path() -> str:
    base = os.environ.get("XDG_CACHE_HOME") or os.path.join(os.path.expanduser("~"), ".cache")
    return os.path.join(base, "lpht", "autotune.json")


def _device_key() -> str:
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(p, "gcnArchName", p.name)
    return f"{arch}|hip {torch.version.hip}|cus {p.multi_processor_count}"


def autotune(layout: int = KV64, log2_capacity: int = 26, reps: int = 2, cache: bool = True,
             stream=None):
    """Runs lpht_autotune (see include/lpht.h) and returns (tuning dict,
    report dict).  Results are cached per device architecture, HIP version,
    layout and capacity in ~/.cache/lpht/autotune.json (XDG_CACHE_HOME
    respected); cache=False measures again and overwrites the entry."""
    import json
    import torch
    torch.cuda.init()
    key = f"{_device_key()}|layout {layout}|log2c {log2_capacity}"
    path = _cache_path()
    db = {}
    if os.path.exists(path):
        try:
            with open(path) as f:
                db = json.load(f)
        except (OSError, ValueError):
            db = {}
    if cache and key in db:
        e = db[key]
        return e["tuning"], e["report"]
    t = lpht_tuning()
    r = lpht_autotune_report()
    s = stream if stream is not None else torch.cuda.current_stream().cuda_stream
    _check(load().lpht_autotune(layout, log2_capacity, reps, ctypes.c_void_p(s), ctypes.byref(t),
                                ctypes.byref(r)), "lpht_autotune")
    tuning = _tuning_dict(t)
    report = {"widths": [1, 2, 4, 8, 16], "fills": [0.125, 0.375, 0.625, 0.875],
              "find_ms": [[round(r.find_ms[q][g], 4) for g in range(5)] for q in range(4)],
              "insert_ms": [[round(r.insert_ms[q][g], 4) for g in range(5)] for q in range(4)],
              "blocks": [256, 512, 1024], "block_ms": [round(x, 4) for x in r.block_ms],
              "migrate_blocks": [256, 512, 1024, 2048],
              "migrate_ms": [round(x, 4) for x in r.migrate_ms]}
    db[key] = {"tuning": tuning, "report": report}
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + f".{os.getpid()}.tmp"
        with open(tmp, "w") as f:
            json.dump(db, f, indent=1)
        os.replace(tmp, path)
    except OSError:
        pass
    return tuning, report


class Batch:
    """Descriptor staging context for lpht_batch_run."""

    def __init__(self, max_ops: int = 256):
        h = ctypes.c_void_p()
        _check(load().lpht_batch_create(max_ops, ctypes.byref(h)), "lpht_batch_create")
        self._h = h
        _track(self)
        self.max_ops = max_ops

    def close(self):
        if getattr(self, "_h", None):
            load().lpht_batch_destroy(self._h)
            self._h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # bound at definition: module globals may be gone during teardown,
        # when the exit hook has closed everything and no HIP call may follow
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def run(self, ops, stream=None):
        """ops: list of dicts with keys table, op, up, keys, vals, vals_out,
        flags, kinds, kind_sel (tensors or None)."""
        arr = (lpht_batch_op * len(ops))()
        for j, o in enumerate(ops):
            t = o["table"]
            keys = o["keys"]
            arr[j].table = t._h
            arr[j].op = o["op"]
            arr[j].up = o.get("up", ASSIGN)
            arr[j].keys = _ptr(keys)
            arr[j].vals = _ptr(o.get("vals"))
            arr[j].n = keys.numel()
            arr[j].vals_out = _ptr(o.get("vals_out"))
            arr[j].flags = _ptr(o.get("flags"))
            arr[j].kinds = _ptr(o.get("kinds"))
            arr[j].kind_sel = o.get("kind_sel", 0)
            arr[j].count_sel = o.get("count_sel", 0)
        _check(load().lpht_batch_run(self._h, arr, len(ops), _stream_handle(stream)), "lpht_batch_run")


# ---------------------------------------------------------------- string keys

class lpht_str_config(ctypes.Structure):
    _fields_ = [
        ("log2_capacity", ctypes.c_uint32),
        ("auto_grow", ctypes.c_uint32),
        ("seed_hi", ctypes.c_uint32),
        ("seed_lo", ctypes.c_uint32),
        ("max_fill_num", ctypes.c_uint32),
        ("max_fill_den", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32 * 2),
        ("pool_bytes", ctypes.c_uint64),
    ]


_STR_SIGS = {
    "lpht_str_config_default": (None, [ctypes.POINTER(lpht_str_config)]),
    "lpht_str_create": (ctypes.c_int, [ctypes.POINTER(lpht_str_config), _VP, ctypes.POINTER(_VP)]),
    "lpht_str_destroy": (ctypes.c_int, [_VP, _VP]),
    "lpht_str_insert": (ctypes.c_int, [_VP, _VP, _VP, _U64, _VP, _VP, _VP]),
    "lpht_str_insert_or_update": (ctypes.c_int, [_VP, _VP, _VP, _U64, _VP, _U32, _VP, _VP]),
    "lpht_str_find": (ctypes.c_int, [_VP, _VP, _VP, _U64, _VP, _VP, _VP]),
    "lpht_str_erase": (ctypes.c_int, [_VP, _VP, _VP, _U64, _VP, _VP]),
    "lpht_str_count": (ctypes.c_int, [_VP, ctypes.POINTER(_U64), ctypes.POINTER(_U64), _VP]),
    "lpht_str_capacity": (ctypes.c_int, [_VP, ctypes.POINTER(_U64), ctypes.POINTER(_U64), ctypes.POINTER(_U64), _VP]),
    "lpht_str_grow": (ctypes.c_int, [_VP, _U32, _VP]),
    "lpht_str_export": (ctypes.c_int, [_VP, _VP, _VP, _U64, _VP]),
    "lpht_str_status": (ctypes.c_int, [_VP, _VP]),
}


def _str_lib():
    L = load()
    if not getattr(L, "_str_declared", False):
        for name, (res, args) in _STR_SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        L._str_declared = True
    return L


def pack_strings(strings, device="cuda"):
    """A list of bytes -> (device u8 tensor, device int64 offsets of n + 1)."""
    import torch
    offs = np.zeros(len(strings) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([len(x) for x in strings], dtype=np.int64)
    raw = b"".join(strings) or b"\0"
    buf = torch.from_numpy(np.frombuffer(raw, dtype=np.uint8).copy()).to(device)
    return buf, torch.from_numpy(offs).to(device)


class StrTable:
    """A table with byte-string keys and u64 values (lpht_str_*)."""

    def __init__(self, log2_capacity: int = 12, auto_grow: bool = False, pool_bytes: int = 1 << 20,
                 seed_hi: int = SEED_HI, seed_lo: int = SEED_LO, alpha=(1, 2), stream=None):
        L = _str_lib()
        cfg = lpht_str_config()
        L.lpht_str_config_default(ctypes.byref(cfg))
        cfg.log2_capacity = log2_capacity
        cfg.auto_grow = 1 if auto_grow else 0
        cfg.pool_bytes = pool_bytes
        cfg.seed_hi, cfg.seed_lo = seed_hi, seed_lo
        cfg.max_fill_num, cfg.max_fill_den = alpha
        h = ctypes.c_void_p()
        self._stream = stream
        _check(L.lpht_str_create(ctypes.byref(cfg), _stream_handle(stream), ctypes.byref(h)), "lpht_str_create")
        self._h = h
        _track(self)

    def close(self):
        if getattr(self, "_h", None):
            _str_lib().lpht_str_destroy(self._h, _stream_handle(self._stream))
            self._h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # bound at definition: module globals may be gone during teardown,
        # when the exit hook has closed everything and no HIP call may follow
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def _run(self, name, strings, *extra):
        import torch
        buf, offs = pack_strings(strings)
        n = len(strings)
        flags = torch.zeros(max(n, 1), dtype=torch.uint8, device="cuda")
        out = torch.zeros(max(n, 1), dtype=torch.int64, device="cuda")
        args = [self._h, _ptr(buf), _ptr(offs), n]
        if name == "lpht_str_find":
            args += [_ptr(out), _ptr(flags)]
        else:
            args += list(extra) + [_ptr(flags)]
        _check(getattr(_str_lib(), name)(*args, _stream_handle(self._stream)), name)
        return flags[:n].cpu().numpy(), out[:n].cpu().numpy().view(np.uint64)

    def _vals(self, vals):
        import torch
        if vals is None:
            return None, None
        t = torch.from_numpy(np.ascontiguousarray(vals, dtype=np.uint64).view(np.int64)).cuda()
        return t, _ptr(t)

    def insert(self, strings, vals=None):
        keep, vp = self._vals(vals)
        return self._run("lpht_str_insert", strings, vp)[0]

    def insert_or_update(self, strings, vals=None, op=ADD):
        keep, vp = self._vals(vals)
        return self._run("lpht_str_insert_or_update", strings, vp, op)[0]

    def find(self, strings):
        f, v = self._run("lpht_str_find", strings)
        return v, f

    def erase(self, strings):
        return self._run("lpht_str_erase", strings)[0]

    def count(self):
        u, l = ctypes.c_uint64(), ctypes.c_uint64()
        _check(_str_lib().lpht_str_count(self._h, ctypes.byref(u), ctypes.byref(l), _stream_handle(self._stream)),
               "lpht_str_count")
        return u.value, l.value

    def capacity(self):
        c, pu, pc = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        _check(_str_lib().lpht_str_capacity(self._h, ctypes.byref(c), ctypes.byref(pu), ctypes.byref(pc),
                                            _stream_handle(self._stream)), "lpht_str_capacity")
        return c.value, pu.value, pc.value

    def grow(self, log2_new: int):
        _check(_str_lib().lpht_str_grow(self._h, log2_new, _stream_handle(self._stream)), "lpht_str_grow")

    def status(self) -> int:
        return _str_lib().lpht_str_status(self._h, _stream_handle(self._stream))

    def cells(self):
        """Per cell: None (empty), False (tombstone) or (key bytes, value),
        decoded from the exported cells and pool."""
        import torch
        c, pu, _ = self.capacity()
        cells = torch.zeros(2 * c, dtype=torch.int64, device="cuda")
        pool = torch.zeros(max(pu, 8), dtype=torch.uint8, device="cuda")
        _check(_str_lib().lpht_str_export(self._h, _ptr(cells), _ptr(pool), pool.numel(),
                                          _stream_handle(self._stream)), "lpht_str_export")
        w = cells.cpu().numpy().view(np.uint64)
        pb = pool.cpu().numpy().tobytes()
        out = []
        for i in range(c):
            r = int(w[2 * i])
            if r == 0:
                out.append(None)
            elif r == 1:
                out.append(False)
            else:
                off = r & ((1 << 48) - 1)
                ln = int.from_bytes(pb[off:off + 4], "little")
                out.append((pb[off + 4:off + 4 + ln], int(w[2 * i + 1])))
        return out


# ---------------------------------------------------------------- serving

SERVE_WAVES = 0
SERVE_SINGLE = 1
SERVE_PERSISTENT = 2
KIND_FIND, KIND_INCREMENT, KIND_ERASE = 0, 1, 2


class lpht_server_config(ctypes.Structure):
    _fields_ = [
        ("ntables", ctypes.c_uint32),
        ("layout", ctypes.c_uint32),
        ("log2_capacity", ctypes.POINTER(ctypes.c_uint32)),
        ("mode", ctypes.c_uint32),
        ("max_inflight", ctypes.c_uint32),
        ("streams", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
        ("hbm_budget", ctypes.c_uint64),
    ]


class lpht_request(ctypes.Structure):
    _fields_ = [
        ("table", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
        ("n", ctypes.c_uint64),
        ("keys", ctypes.c_void_p),
        ("kinds", ctypes.c_void_p),
        ("vals_out", ctypes.c_void_p),
        ("flags", ctypes.c_void_p),
    ]


class lpht_completion(ctypes.Structure):
    _fields_ = [
        ("ticket", ctypes.c_uint64),
        ("status", ctypes.c_int),
        ("wave", ctypes.c_uint32),
        ("submit_us", ctypes.c_double),
        ("admit_us", ctypes.c_double),
        ("done_us", ctypes.c_double),
    ]


class lpht_server_stats(ctypes.Structure):
    _fields_ = [
        ("completed", ctypes.c_uint64),
        ("waves", ctypes.c_uint64),
        ("launches_phases", ctypes.c_uint64),
        ("peak_hbm_bytes", ctypes.c_uint64),
        ("admission_waits", ctypes.c_uint64),
        ("busy_us", ctypes.c_double),
        ("kernel_growths", ctypes.c_uint64),
        ("kernel_growth_fallbacks", ctypes.c_uint64),
    ]


_SIGS.update({
    "lpht_server_create": (ctypes.c_int, [ctypes.POINTER(lpht_server_config), ctypes.POINTER(_VP)]),
    "lpht_server_submit": (ctypes.c_int, [_VP, ctypes.POINTER(lpht_request), ctypes.POINTER(_U64)]),
    "lpht_server_poll": (ctypes.c_int, [_VP, _U64, ctypes.POINTER(lpht_completion)]),
    "lpht_server_wait": (ctypes.c_int, [_VP, _U64, ctypes.POINTER(lpht_completion)]),
    "lpht_server_drain": (ctypes.c_int, [_VP]),
    "lpht_server_table": (ctypes.c_int, [_VP, _U32, ctypes.POINTER(_VP)]),
    "lpht_server_stats_get": (ctypes.c_int, [_VP, ctypes.POINTER(lpht_server_stats)]),
    "lpht_server_destroy": (ctypes.c_int, [_VP]),
    "lpht_server_run_closed_loop": (ctypes.c_int, [_VP, ctypes.POINTER(lpht_request), _U32, _U32,
                                                   ctypes.POINTER(lpht_completion),
                                                   ctypes.POINTER(ctypes.c_double)]),
})


class _TableView(Table):
    """A table owned by a server (not destroyed by Python)."""

    def __init__(self, handle, layout):
        import torch
        self._h = handle
        self.layout = layout
        self.word = 4 if layout == PACKED32 else 8
        self.torch_dtype = torch.int32 if layout == PACKED32 else torch.int64
        self._stream = None

    def close(self, stream=None):
        self._h = None


class Server:
    """Request loop over resident tables (lpht_server_*).  Requests carry
    host arrays; they are copied into pinned buffers owned by this object."""

    def __init__(self, log2_caps, layout=KV64, mode=SERVE_WAVES, max_inflight=64, streams=2,
                 hbm_budget=0):
        import torch
        torch.cuda.init()  # torch's device state first: the binding hands out torch tensors
        L = load()
        self.layout = layout
        self.kdt = "uint32" if layout == PACKED32 else "uint64"
        caps = (ctypes.c_uint32 * len(log2_caps))(*log2_caps)
        cfg = lpht_server_config(len(log2_caps), layout, caps, mode, max_inflight, streams, 0, hbm_budget)
        h = ctypes.c_void_p()
        _check(L.lpht_server_create(ctypes.byref(cfg), ctypes.byref(h)), "lpht_server_create")
        self._h = h
        _track(self)
        self.ntables = len(log2_caps)

    def close(self):
        if getattr(self, "_h", None):
            load().lpht_server_destroy(self._h)
            self._h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # bound at definition: module globals may be gone during teardown,
        # when the exit hook has closed everything and no HIP call may follow
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def make_requests(self, reqs):
        """reqs: list of (table, keys ndarray, kinds ndarray).  Returns
        (ctypes request array, list of (vals, flags) output tensors, buffers
        to keep alive).  All host arrays live in four pinned buffers."""
        import numpy as np
        import torch
        sizes = [len(k) for _, k, _ in reqs]
        total = int(sum(sizes))
        w = 4 if self.layout == PACKED32 else 8
        kdt = torch.int32 if self.layout == PACKED32 else torch.int64
        keys = torch.empty(total, dtype=kdt).pin_memory()
        kinds = torch.empty(total, dtype=torch.uint8).pin_memory()
        vals = torch.empty(total, dtype=kdt).pin_memory()
        flags = torch.empty(total, dtype=torch.uint8).pin_memory()
        knp, kdnp = keys.numpy(), kinds.numpy()
        arr = (lpht_request * len(reqs))()
        outs = []
        off = 0
        for j, (tab, k, kd) in enumerate(reqs):
            n = len(k)
            knp[off:off + n] = np.ascontiguousarray(k).view(np.int32 if w == 4 else np.int64)
            kdnp[off:off + n] = kd
            arr[j] = lpht_request(tab, 0, n, keys.data_ptr() + off * w, kinds.data_ptr() + off,
                                  vals.data_ptr() + off * w, flags.data_ptr() + off)
            outs.append((vals[off:off + n], flags[off:off + n]))
            off += n
        return arr, outs, [keys, kinds, vals, flags]

    def run_closed_loop(self, req_array, nclients):
        n = len(req_array)
        done = (lpht_completion * n)()
        wall = ctypes.c_double()
        _check(load().lpht_server_run_closed_loop(self._h, req_array, n, nclients, done,
                                                  ctypes.byref(wall)), "lpht_server_run_closed_loop")
        return done, wall.value

    def submit(self, req):
        t = ctypes.c_uint64()
        _check(load().lpht_server_submit(self._h, ctypes.byref(req), ctypes.byref(t)), "lpht_server_submit")
        return t.value

    def wait(self, ticket):
        c = lpht_completion()
        _check(load().lpht_server_wait(self._h, ticket, ctypes.byref(c)), "lpht_server_wait")
        return c

    def drain(self):
        _check(load().lpht_server_drain(self._h), "lpht_server_drain")

    def table(self, i):
        h = ctypes.c_void_p()
        _check(load().lpht_server_table(self._h, i, ctypes.byref(h)), "lpht_server_table")
        return _TableView(h, self.layout)

    def stats(self):
        s = lpht_server_stats()
        _check(load().lpht_server_stats_get(self._h, ctypes.byref(s)), "lpht_server_stats_get")
        return {k: getattr(s, k) for k, _ in lpht_server_stats._fields_}
