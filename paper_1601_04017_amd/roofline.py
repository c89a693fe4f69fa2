"""Measured memory-system ceilings for the table's access pattern (binding of
libroofline.so).  Used by the benchmark to report the table kernels' rates as
fractions of what the same GPU reaches on plain random gathers, random
atomics and streaming copies."""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libroofline.so")

_lib = None


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libroofline.so not built ({LIB_PATH})")
        # torch's HIP runtime first, so that this library binds to it (see
        # lpht.load)
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        vp, u64 = ctypes.c_void_p, ctypes.c_uint64
        L.rl_gather.argtypes = [vp, u64, ctypes.c_int, u64, u64, vp, vp]
        L.rl_cas.argtypes = [vp, u64, u64, u64, vp, vp]
        L.rl_add.argtypes = [vp, u64, u64, u64, vp, vp]
        L.rl_hot_add.argtypes = [vp, u64, ctypes.c_int, vp]
        L.rl_copy.argtypes = [vp, vp, u64, u64, vp]
        for f in (L.rl_gather, L.rl_cas, L.rl_add, L.rl_hot_add, L.rl_copy):
            f.restype = ctypes.c_int
        _lib = L
    return _lib


def measure(buf_bytes: int = 1 << 32, lanes: int = 1 << 24, reps: int = 3) -> dict:
    """Ceilings on the current GPU: random gathers of 8/16/64/128 bytes
    (G accesses/s and GB/s of whole accesses), random 64-bit CAS and
    fetch-and-add (G/s), same-address fetch-and-add (M/s) and a 16-byte
    streaming copy (GB/s, read + write)."""
    import torch

    L = load()
    dev = torch.device("cuda")
    buf = torch.zeros(buf_bytes // 8, dtype=torch.int64, device=dev)
    sink = torch.zeros(1, dtype=torch.int64, device=dev)
    s = torch.cuda.current_stream()
    sh = ctypes.c_void_p(s.cuda_stream)
    per_lane = 4

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        best = None
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(s)
            fn()
            b.record(s)
            b.synchronize()
            ms = a.elapsed_time(b)
            best = ms if best is None else min(best, ms)
        return best / 1e3

    out = {"buffer_bytes": buf_bytes}
    for w in (8, 16, 64, 128):
        t = timed(lambda: L.rl_gather(ctypes.c_void_p(buf.data_ptr()), buf_bytes, w, lanes, 7, ctypes.c_void_p(sink.data_ptr()), sh))
        acc = lanes * per_lane / t
        out[f"gather{w}_Gps"] = round(acc / 1e9, 3)
        out[f"gather{w}_GBs"] = round(acc * w / 1e9, 1)
    t = timed(lambda: L.rl_cas(ctypes.c_void_p(buf.data_ptr()), buf_bytes, lanes, 11, ctypes.c_void_p(sink.data_ptr()), sh))
    out["cas_Gps"] = round(lanes * per_lane / t / 1e9, 3)
    t = timed(lambda: L.rl_add(ctypes.c_void_p(buf.data_ptr()), buf_bytes, lanes, 13, ctypes.c_void_p(sink.data_ptr()), sh))
    out["add_Gps"] = round(lanes * per_lane / t / 1e9, 3)
    hot_lanes, hot_per = 1 << 16, 16
    t = timed(lambda: L.rl_hot_add(ctypes.c_void_p(sink.data_ptr()), hot_lanes, hot_per, sh))
    out["hot_add_Mps"] = round(hot_lanes * hot_per / t / 1e6, 2)
    half = buf_bytes // 2
    base = buf.data_ptr()
    # as many workgroups as there are tiles of 32 KiB, at most 65536 (the
    # table's zero-fill uses the same shape)
    tiles = min(65536, half // (16 * 256 * 8))
    t = timed(lambda: L.rl_copy(ctypes.c_void_p(base), ctypes.c_void_p(base + half), half, 256 * tiles, sh))
    out["copy_GBs"] = round(2 * half / t / 1e9, 1)
    del buf
    return out


if __name__ == "__main__":
    import json
    print(json.dumps(measure()))
