"""lpht: lock-free linear-probing hash tables on AMD MI355X (gfx950).

The device path lives in the HIP library ``liblpht.so`` behind the C ABI of
``include/lpht.h``; :mod:`paper_1601_04017_amd.lpht` is the thin ctypes binding
over it.  Submodules are imported on first use so that the seeded input
generators in :mod:`paper_1601_04017_amd.inputs` work without a GPU.
"""
import importlib

__all__ = ["lpht", "inputs"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
