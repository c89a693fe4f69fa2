"""The partitioned insert-or-add (large LPHT_ADD upserts on large tables:
the batch is partitioned by table region, combined per bucket in LDS, and
each distinct key applied once) against the oracle, at sizes that take that
path (at least 2^22 operations, at least 2^20 cells): flags after
canonicalisation, counts, and the table modulo the order inside runs; with
and without values and flags, with reserved keys, on a table that already
holds keys and tombstones, and equal to the chunk-combining kernel."""
import numpy as np
import pytest

import oracle
from paper_1601_04017_amd import inputs
from tests import helpers as H
from tests.gpu_util import cells_host, keys_dtype, make_table, to_dev, to_host

pytestmark = pytest.mark.gpu

LAYOUTS = [oracle.PACKED32, oracle.KV64]
N = (1 << 22) + 4097  # ragged


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"


def _zipf(layout, n, universe, s, seed, scramble=False):
    z = inputs.zipf_keys_u64(n, universe, s, seed=seed)
    if scramble:
        z = inputs.scramble_keys_u64(z, seed + 1)
    if layout == oracle.PACKED32:
        z = (z & np.uint64(0xFFFFFFFF)).astype(np.uint32)
        z[z < 2] = 2
    return z


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("with_vals,with_flags", [(False, False), (False, True), (True, True), (True, False)])
def test_partitioned_upsert_add_matches_oracle(layout, with_vals, with_flags):
    log2c = 23  # used + n <= capacity: no insertion can find the table full
    z = _zipf(layout, N, 3_000_000, 1.0, 601, scramble=True)
    v = (np.arange(N) % 13 + 1).astype(keys_dtype(layout)) if with_vals else None
    print(f"partitioned upsert: layout {layout} vals {with_vals} flags {with_flags}", flush=True)
    o = oracle.OracleTable(layout, log2c)
    of = o.insert_or_update(z, v, oracle.ADD)
    t = make_table(layout, log2c)
    gf = t.insert_or_update(to_dev(z), None if v is None else to_dev(v), op=oracle.ADD, flags=with_flags)
    if with_flags:
        assert np.array_equal(H.canonical_flags(z, to_host(gf)), of)
    assert t.count() == o.counts()
    assert t.status() == 0
    H.assert_same_table_modulo_run_order(cells_host(t), o.cells(), layout)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_partitioned_with_reserved_keys_and_existing_contents(layout):
    log2c = 23
    base = inputs.distinct_keys_u32(400_000, 71).astype(keys_dtype(layout))
    z = _zipf(layout, N, 600_000, 1.2, 602)
    z = np.concatenate([z, base[::7]])
    z[::100_003] = 0
    z[5::200_003] = 1
    z = z[inputs.permutation(z.size, 603)]
    o = oracle.OracleTable(layout, log2c)
    t = make_table(layout, log2c)
    o.insert(base, base)
    t.insert(to_dev(base), to_dev(base))
    o.erase(base[::3])
    t.erase(to_dev(base[::3]))
    of = o.insert_or_update(z, None, oracle.ADD)
    gf = to_host(t.insert_or_update(to_dev(z), None, op=oracle.ADD))
    assert np.array_equal(H.canonical_flags(z, gf), of)
    assert t.count() == o.counts()
    from paper_1601_04017_amd import lpht
    assert t.status() == lpht.ERR_RESERVED_KEY
    H.assert_same_table_modulo_run_order(cells_host(t), o.cells(), layout)


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("s", [0.5, 1.5])
def test_partitioned_equals_chunk_combining(layout, s):
    log2c = 23
    z = _zipf(layout, N, 10 ** 7, s, 604)
    a = make_table(layout, log2c)
    b = make_table(layout, log2c)
    b.set_tuning(aggregate=2)
    fa = to_host(a.insert_or_update(to_dev(z), None, op=oracle.ADD))
    fb = to_host(b.insert_or_update(to_dev(z), None, op=oracle.ADD))
    assert np.array_equal(H.canonical_flags(z, fa), H.canonical_flags(z, fb))
    assert a.count() == b.count()
    H.assert_same_table_modulo_run_order(cells_host(a), cells_host(b), layout)
