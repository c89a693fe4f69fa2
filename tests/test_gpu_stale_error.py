"""A failed HIP call of another caller leaves its error with the thread (HIP
keeps it until hipGetLastError reads it, through later successful calls).
The library's calls report their own launches only: a stale error must not
fail them, and none is left behind for the caller."""
import ctypes

import numpy as np
import pytest

from tests.gpu_util import to_dev

pytestmark = pytest.mark.gpu


def _hip():
    # the HIP runtime of this process: the library binds to the one torch
    # loaded, and there must be only one
    with open("/proc/self/maps") as f:
        paths = {line.split()[-1] for line in f if "libamdhip64" in line}
    assert len(paths) == 1, paths
    return ctypes.CDLL(paths.pop())


def _leave_stale_error(hip):
    assert hip.hipSetDevice(ctypes.c_int(9999)) != 0  # no such device
    assert hip.hipPeekAtLastError() != 0


def test_stale_error_does_not_fail_table_calls():
    from paper_1601_04017_amd import lpht
    lpht.load()
    hip = _hip()
    keys = np.arange(2, 5002, dtype=np.uint64)
    dk = to_dev(keys)
    try:
        _leave_stale_error(hip)
        t = lpht.Table(layout=lpht.KV64, log2_capacity=14)
        _leave_stale_error(hip)
        t.insert(dk, dk)
        _leave_stale_error(hip)
        vals, found = t.find(dk)
        assert t.count()[1] == keys.size
        assert found.cpu().numpy().all()
        assert np.array_equal(vals.cpu().numpy().view(np.uint64), keys)
        t.close()
    finally:
        hip.hipGetLastError()


def test_stale_error_does_not_fail_server_creation():
    from paper_1601_04017_amd import lpht
    lpht.load()
    hip = _hip()
    try:
        _leave_stale_error(hip)
        srv = lpht.Server([12, 13, 14], mode=lpht.SERVE_WAVES, max_inflight=4, streams=2)
        srv.close()
    finally:
        hip.hipGetLastError()
