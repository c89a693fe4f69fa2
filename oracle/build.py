"""Builds the CPU oracle (test infrastructure) into oracle/liborc.so with gcc.

The oracle is a plain sequential C program; it is compiled without any
machine-specific flags so that the same source gives the same results on any
x86-64 host.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lpht_oracle.c")
OUT = os.path.join(HERE, "liborc.so")


def build(force: bool = True) -> str:
    if not force and os.path.exists(OUT) and os.path.getmtime(OUT) >= os.path.getmtime(SRC):
        return OUT
    tmp = OUT + ".tmp"
    cmd = ["gcc", "-O3", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, SRC]
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(force="--if-stale" not in sys.argv))
