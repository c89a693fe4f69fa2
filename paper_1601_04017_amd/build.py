"""Builds liblpht.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree.

    python -m paper_1601_04017_amd.build
"""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "liblpht.so")
SOURCES = ["lpht_kernels.hip", "lpht_part.hip", "lpht_shrink.hip", "lpht_bulk.hip", "lpht_async.hip", "lpht_special.hip", "lpht_str.hip", "lpht_str_api.cpp", "lpht_api.cpp", "lpht_server.cpp", "lpht_tune.cpp"]
ROOFLINE_OUT = os.path.join(PKG, "libroofline.so")
ROOFLINE_SOURCES = ["lpht_roofline.hip"]
HEADERS = ["lpht_internal.h", "lpht_host.h", "lpht_device.h", "lpht_migrate.h", "lpht_part.h", "lpht_shrink.h", "lpht_bulk.h", "lpht_async.h", "lpht_special.h", "lpht_str.h", os.path.join("..", "..", "include", "lpht.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Wall",
    "-pthread",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _stale(out, sources, headers) -> bool:
    if not os.path.exists(out):
        return True
    t = os.path.getmtime(out)
    for f in sources + headers:
        if os.path.getmtime(os.path.join(CSRC, f)) > t:
            return True
    return False


OBJ_DIR = os.path.join(ROOT, "_build")


def _run(cmd, what, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    return subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True), what


def _hipcc(out, sources, verbose):
    """Compiles every source to an object in parallel (each translation unit
    carries its own gfx950 code object), then links the shared library."""
    os.makedirs(OBJ_DIR, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include")]
    cflags = [f for f in FLAGS if f != "-shared"]
    objs, procs = [], []
    for f in sources:
        obj = os.path.join(OBJ_DIR, os.path.splitext(f)[0] + ".o")
        objs.append(obj)
        procs.append(_run([HIPCC, *cflags, *inc, "-c", "-o", obj, os.path.join(CSRC, f)], f, verbose))
    failed = []
    for p, what in procs:
        log = p.communicate()[0]
        if p.returncode != 0:
            sys.stderr.write(log)
            failed.append(what)
    if failed:
        raise RuntimeError(f"hipcc failed on {', '.join(failed)}")
    tmp = out + ".tmp"
    p, _ = _run([HIPCC, *FLAGS, "-o", tmp, *objs], out, verbose)
    log = p.communicate()[0]
    if p.returncode != 0:
        sys.stderr.write(log)
        raise RuntimeError(f"hipcc failed linking {os.path.basename(out)}")
    os.replace(tmp, out)


def build(force: bool = True, verbose: bool = False) -> str:
    """Builds liblpht.so (the table) and libroofline.so (memory ceilings)."""
    if force or _stale(OUT, SOURCES, HEADERS):
        _hipcc(OUT, SOURCES, verbose)
    if force or _stale(ROOFLINE_OUT, ROOFLINE_SOURCES, []):
        _hipcc(ROOFLINE_OUT, ROOFLINE_SOURCES, verbose)
    return OUT


if __name__ == "__main__":
    print(build(force="--if-stale" not in sys.argv, verbose=True))
