"""Small native helpers for the tests (built on demand with gcc)."""
import ctypes
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def load_crc_sse42():
    src = os.path.join(HERE, "crc_sse42.c")
    out = os.path.join(HERE, "libcrc_sse42.so")
    if not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        subprocess.run(["gcc", "-O2", "-msse4.2", "-fPIC", "-shared", "-o", out + ".tmp", src],
                       check=True)
        os.replace(out + ".tmp", out)
    L = ctypes.CDLL(out)
    L.hw_crc_u8.restype = ctypes.c_uint32
    L.hw_crc_u8.argtypes = [ctypes.c_uint32, ctypes.c_uint8]
    L.hw_crc_u32.restype = ctypes.c_uint32
    L.hw_crc_u32.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
    L.hw_crc_u64.restype = ctypes.c_uint32
    L.hw_crc_u64.argtypes = [ctypes.c_uint32, ctypes.c_uint64]
    L.hw_hash_bulk.restype = None
    L.hw_hash_bulk.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32,
                               ctypes.c_uint32, ctypes.c_void_p]
    return L
