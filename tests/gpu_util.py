"""Helpers for the GPU tests: numpy <-> device tensors and table construction
through the C ABI binding."""
import numpy as np

import oracle


def torch():
    import torch as _t
    return _t


def to_dev(a: np.ndarray):
    t = torch()
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint64:
        a = a.view(np.int64)
    elif a.dtype == np.uint32:
        a = a.view(np.int32)
    return t.from_numpy(a).cuda()


def to_host(x, dtype=None) -> np.ndarray:
    a = x.cpu().numpy()
    if dtype is not None:
        a = a.view(dtype)
    return a


def keys_dtype(layout):
    return np.uint32 if layout == oracle.PACKED32 else np.uint64


def make_table(layout, log2c, **kw):
    from paper_1601_04017_amd import lpht
    return lpht.Table(layout=layout, log2_capacity=log2c, **kw)


def cells_host(tbl) -> np.ndarray:
    return to_host(tbl.export_cells(), np.uint64)
