"""The entry point that allocates nothing (lpht_build_noalloc) against the
sort-based build it varies (lpht_build): identical cells (the build's layout
is a function of the key set) and counts, on two calls in a row on the same
table, the second with a smaller batch, for both layouts and both update
functions; then the refusals (growth needed, scratch too small) leave the
table unchanged."""
import numpy as np
import pytest

import oracle
from paper_1601_04017_amd import inputs
from tests.gpu_util import cells_host, keys_dtype, make_table, to_dev

pytestmark = pytest.mark.gpu

LAYOUTS = [oracle.PACKED32, oracle.KV64]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"


def _batch(layout, n, seed):
    if layout == oracle.PACKED32:
        k = inputs.distinct_keys_u32(n, seed)
    else:
        k = inputs.distinct_keys_u64(n, seed)
    rng = np.random.default_rng(seed)
    b = np.concatenate([k, k[rng.integers(0, n, n // 4)]])
    b = b[rng.permutation(b.size)]
    v = rng.integers(0, 1 << 31, b.size).astype(keys_dtype(layout))
    return b, v


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("op", [oracle.ASSIGN, oracle.ADD])
def test_noalloc_build_equals_build_twice(layout, op):
    from paper_1601_04017_amd import lpht
    log2c = 21
    ref = make_table(layout, log2c)
    na = make_table(layout, log2c)
    for call, n in enumerate((800_000, 90_000)):
        print(f"noalloc build: layout {layout} op {op} call {call} n {n}", flush=True)
        b, v = _batch(layout, n, 40 + call)
        db, dv = to_dev(b), to_dev(v)
        ref.build(db, dv, op=op)
        assert na.build_noalloc(db, dv, op=op) == lpht.OK
        assert np.array_equal(cells_host(na), cells_host(ref)), f"call {call}"
        assert na.count() == ref.count() == (np.unique(b).size, np.unique(b).size)
        assert na.status() == lpht.OK
    ref.close()
    na.close()


@pytest.mark.parametrize("layout", LAYOUTS)
def test_noalloc_refusals_change_nothing(layout):
    from paper_1601_04017_amd import lpht
    t = make_table(layout, 12, auto_grow=True)
    b, v = _batch(layout, 1000, 7)
    assert t.build_noalloc(to_dev(b), to_dev(v)) == lpht.OK
    before = cells_host(t)
    counts = t.count()
    big, bv = _batch(layout, 5000, 8)  # more than alpha * 4096 cells: the table would grow
    assert t.build_noalloc(to_dev(big), to_dev(bv)) == lpht.ERR_UNSUPPORTED
    assert np.array_equal(cells_host(t), before) and t.count() == counts
    t.close()
    # a batch whose scratch exceeds the fixed array
    t = make_table(layout, 26)
    huge = to_dev(np.arange(2, 2 + (1 << 22), dtype=keys_dtype(layout)))
    assert t.build_noalloc(huge) == lpht.ERR_INVALID
    assert t.count() == (0, 0)
    t.close()
