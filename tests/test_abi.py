"""CPU-side checks of the C ABI: the library loads without a GPU and exports
every function that include/lpht.h declares, and the binding declares the same
set.  No compute call is made."""
import ctypes
import os
import re

import pytest

from paper_1601_04017_amd import build as libbuild
from paper_1601_04017_amd import lpht

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lpht.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(lpht_[a-z0-9_]+)\s*\(", src))
    # function-pointer typedefs are not functions
    return {n for n in names if not n.endswith("_fn")}


@pytest.fixture(scope="module")
def lib():
    libbuild.build(force=False)
    return lpht.load()


def test_header_declares_functions():
    d = _declared()
    assert {"lpht_create", "lpht_insert", "lpht_find", "lpht_insert_or_update", "lpht_update",
            "lpht_erase", "lpht_grow", "lpht_count", "lpht_destroy"} <= d


def test_library_exports_every_declared_symbol(lib):
    for name in sorted(_declared()):
        assert hasattr(lib, name), name
        assert isinstance(getattr(lib, name), ctypes._CFuncPtr)


def test_binding_covers_header(lib):
    assert set(lpht.exported_symbols()) == _declared()


def test_static_calls_need_no_gpu(lib):
    assert lib.lpht_version().startswith(b"lpht")
    assert lib.lpht_strerror(lpht.ERR_FULL).startswith(b"bounded table full")
    assert lib.lpht_cell_bytes(lpht.PACKED32) == 8 and lib.lpht_cell_bytes(lpht.KV64) == 16
    cfg = lpht.lpht_config()
    lib.lpht_config_default(ctypes.byref(cfg))
    assert (cfg.layout, cfg.log2_capacity, cfg.seed_hi, cfg.seed_lo) == (1, 12, 0x9E3779B9, 0xFFFFFFFF)
    assert (cfg.max_fill_num, cfg.max_fill_den, cfg.auto_grow) == (1, 2, 0)


def test_invalid_arguments_rejected_on_host(lib):
    # rejected before any device call
    out = ctypes.c_void_p()
    cfg = lpht.lpht_config()
    lib.lpht_config_default(ctypes.byref(cfg))
    cfg.log2_capacity = 3
    assert lib.lpht_create(ctypes.byref(cfg), None, ctypes.byref(out)) == lpht.ERR_INVALID
    cfg.log2_capacity = 12
    cfg.layout = 7
    assert lib.lpht_create(ctypes.byref(cfg), None, ctypes.byref(out)) == lpht.ERR_INVALID
    assert lib.lpht_insert(None, None, None, 0, None, None) == lpht.ERR_INVALID
    assert lib.lpht_grow(None, 10, None) == lpht.ERR_INVALID
    assert lib.lpht_destroy(None, None) == lpht.OK


def _c_sizes(tmp_path, types):
    # compiles a C program against include/lpht.h and prints sizeof of each type
    src = tmp_path / "sizes.c"
    body = "".join(f'  printf("%zu\\n", sizeof({t}));\n' for t in types)
    src.write_text('#include <stdio.h>\n#include "lpht.h"\nint main(void) {\n' + body + "  return 0;\n}\n")
    exe = tmp_path / "sizes"
    import subprocess
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    return [int(x) for x in out]


def test_struct_layouts_match_header(tmp_path):
    pairs = [("lpht_config", lpht.lpht_config), ("lpht_tuning", lpht.lpht_tuning),
             ("lpht_stats", lpht.lpht_stats), ("lpht_autotune_report", lpht.lpht_autotune_report),
             ("lpht_batch_op", lpht.lpht_batch_op), ("lpht_server_config", lpht.lpht_server_config),
             ("lpht_request", lpht.lpht_request), ("lpht_completion", lpht.lpht_completion),
             ("lpht_server_stats", lpht.lpht_server_stats), ("lpht_str_config", lpht.lpht_str_config)]
    sizes = _c_sizes(tmp_path, [c for c, _ in pairs])
    for (cname, py), n in zip(pairs, sizes):
        assert ctypes.sizeof(py) == n, cname


def test_autotune_arguments_rejected_on_host(lib):
    t = lpht.lpht_tuning()
    assert lib.lpht_autotune(7, 20, 1, None, ctypes.byref(t), None) == lpht.ERR_INVALID
    assert lib.lpht_autotune(lpht.KV64, 10, 1, None, ctypes.byref(t), None) == lpht.ERR_INVALID
    assert lib.lpht_autotune(lpht.KV64, 20, 0, None, ctypes.byref(t), None) == lpht.ERR_INVALID
    assert lib.lpht_autotune(lpht.KV64, 20, 1, None, None, None) == lpht.ERR_INVALID


def test_hash_choice_validated_on_host(lib):
    out = ctypes.c_void_p()
    cfg = lpht.lpht_config()
    lib.lpht_config_default(ctypes.byref(cfg))
    assert (cfg.hash, cfg.reserved0, cfg.mul) == (lpht.HASH_CRC32C_PAIR, 0, 0)
    cfg.hash = lpht.HASH_MULSHIFT
    cfg.mul = 0x9E3779B97F4A7C14  # even
    assert lib.lpht_create(ctypes.byref(cfg), None, ctypes.byref(out)) == lpht.ERR_INVALID
    cfg.hash = 7
    cfg.mul = 3
    assert lib.lpht_create(ctypes.byref(cfg), None, ctypes.byref(out)) == lpht.ERR_INVALID
    cfg.hash = lpht.HASH_MULSHIFT
    cfg.reserved0 = 1
    assert lib.lpht_create(ctypes.byref(cfg), None, ctypes.byref(out)) == lpht.ERR_INVALID
    assert not out.value


def test_library_binds_to_one_hip_runtime():
    # torch's wheel carries its own HIP runtime with the soname liblpht.so was
    # linked against; the binding loads torch first so that the process holds
    # one runtime (torch's streams and errors must be the library's own)
    import ast
    import subprocess
    import sys
    code = ("from paper_1601_04017_amd import lpht, roofline\n"
            "lpht.load()\n"
            "roofline.load()\n"
            "print(sorted({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    paths = ast.literal_eval(out.stdout.strip().splitlines()[-1])
    assert len(paths) == 1, paths
