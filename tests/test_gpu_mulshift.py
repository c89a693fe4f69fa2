"""Tables with the multiplicative hash (h = mul * key mod 2^64, the position
its top bits) on the GPU against the oracle built with the same hash: bulk
operations, migration cell for cell (Lemma 1 holds for any hash positioned by
the scaling map), shrinking, growth, the sort-based build and merge, and the
in-kernel growth.  Same bar as the CRC tables: integer results identical."""
import numpy as np
import pytest

import oracle
from paper_1601_04017_amd import inputs
from tests import helpers as H
from tests.gpu_util import cells_host, keys_dtype, make_table, to_dev, to_host

pytestmark = pytest.mark.gpu

LAYOUTS = [oracle.PACKED32, oracle.KV64]
MUL = 0xD6E8FEB86659FD93


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"


def _keys(layout, n, seed, absent=False):
    if layout == oracle.PACKED32:
        return inputs.distinct_keys_u32(n, seed, absent=absent)
    return inputs.distinct_keys_u64(n, seed, absent=absent)


def _pair(layout, log2c, **kw):
    from paper_1601_04017_amd import lpht
    t = make_table(layout, log2c, hash=lpht.HASH_MULSHIFT, mul=MUL, **kw)
    o = oracle.OracleTable(layout, log2c, hash=oracle.HASH_MULSHIFT, mul=MUL, **kw)
    return t, o


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("G", [1, 4])
def test_insert_find_match_oracle(layout, G):
    log2c = 17
    n = (1 << 16) + 77
    keys = _keys(layout, n, 301)
    vals = (np.arange(n) * 5 + 1).astype(keys_dtype(layout))
    fk = np.concatenate([keys[::3], _keys(layout, 9001, 301, absent=True)])
    t, o = _pair(layout, log2c)
    t.set_tuning(group_width=G)
    gf = to_host(t.insert(to_dev(keys), to_dev(vals)))
    gv, gfound = t.find(to_dev(fk))
    assert np.array_equal(gf, o.insert(keys, vals))
    ov, of = o.find(fk)
    assert np.array_equal(to_host(gfound), of)
    assert np.array_equal(to_host(gv, keys_dtype(layout)), ov)
    assert t.count() == o.counts()
    cells = cells_host(t)
    H.check_invariants(cells, layout, log2c, n, n, mul=MUL)
    H.assert_same_table_modulo_run_order(cells, o.cells(), layout)


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("agg", [0, 1])
def test_zipf_increment_histogram(layout, agg):
    z = inputs.zipf_keys_u64(400_003, 1_000_000, 1.0, seed=77).astype(keys_dtype(layout))
    t, o = _pair(layout, 20)
    t.set_tuning(aggregate=agg)
    gf = to_host(t.insert_or_update(to_dev(z), None, op=oracle.ADD))
    assert np.array_equal(H.canonical_flags(z, gf), o.insert_or_update(z, None, oracle.ADD))
    assert t.count() == o.counts()
    H.assert_same_table_modulo_run_order(cells_host(t), o.cells(), layout)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_update_erase_sequence(layout):
    keys = _keys(layout, 30000, 17)
    rng = np.random.default_rng(4)
    t, o = _pair(layout, 16)
    t.insert(to_dev(keys), to_dev(keys))
    o.insert(keys, keys)
    for r in range(4):
        sel = keys[rng.integers(0, keys.size, 8000)]
        d = rng.integers(0, 1 << 30, sel.size).astype(keys_dtype(layout))
        gu = to_host(t.update(to_dev(sel), to_dev(d), op=oracle.ADD))
        assert np.array_equal(gu, o.update(sel, d, oracle.ADD))
        er = np.unique(sel[:2000])
        ge = to_host(t.erase(to_dev(er)))
        assert np.array_equal(ge, o.erase(er))
        gv, gfo = t.find(to_dev(keys))
        ov, ofo = o.find(keys)
        assert np.array_equal(to_host(gfo), ofo)
        assert np.array_equal(to_host(gv, keys_dtype(layout)), ov)
    assert t.count() == o.counts()


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("gamma_log", [0, 1, 2])
def test_migration_cell_for_cell(layout, gamma_log):
    log2c = 16
    n = int(0.48 * (1 << log2c))
    keys = _keys(layout, n, 93)
    t, o = _pair(layout, log2c)
    o.insert(keys, keys)
    o.erase(keys[::5])
    t.import_cells(to_dev(o.cells()), log2c)
    t.grow(log2c + gamma_log)
    o.grow(log2c + gamma_log)
    assert np.array_equal(cells_host(t), o.cells())
    assert t.count() == o.counts()


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("shrink", [1, 3])
def test_shrink_matches_oracle_modulo_run_order(layout, shrink):
    log2c = 18
    keys = _keys(layout, 20000, 55)
    t, o = _pair(layout, log2c)
    t.insert(to_dev(keys), to_dev(keys))
    o.insert(keys, keys)
    t.grow(log2c - shrink)
    o.grow(log2c - shrink)
    assert t.count() == o.counts()
    H.assert_same_table_modulo_run_order(cells_host(t), o.cells(), layout)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_auto_grow_capacity_sequence(layout):
    keys = _keys(layout, 400_000, 71)
    t, o = _pair(layout, 10, auto_grow=True)
    for lo in range(0, keys.size, 37_000):
        b = keys[lo:lo + 37_000]
        gf = to_host(t.insert(to_dev(b), to_dev(b)))
        assert np.array_equal(gf, o.insert(b, b))
        assert t.capacity == o.capacity
        if lo % 74_000 == 0:
            ge = to_host(t.erase(to_dev(b[::4])))
            assert np.array_equal(ge, o.erase(b[::4]))
    assert t.count() == o.counts()
    H.assert_same_table_modulo_run_order(cells_host(t), o.cells(), layout)


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("op", [oracle.ASSIGN, oracle.ADD])
def test_bulk_build_and_merge_cell_for_cell(layout, op):
    # the twin keys make many ties of the upper hash half (see the oracle's
    # pin of the bulk order), so the tie rule is exercised
    rng = np.random.default_rng(12)
    base = _keys(layout, 150_000, 12).astype(np.uint64)
    if layout == oracle.KV64:
        step = np.uint64((pow(MUL, -1, 1 << 64) * ((1 << 64) - 5)) % (1 << 64))
        with np.errstate(over="ignore"):
            b = np.concatenate([base, base[:50_000] + step])
    else:
        b = base
    b = np.concatenate([b, b[rng.integers(0, b.size, 30_000)]]).astype(keys_dtype(layout))
    b = b[(b != 0) & (b != 1)]
    v = rng.integers(0, 1 << 30, b.size).astype(keys_dtype(layout))
    t, o = _pair(layout, 19)
    t.build(to_dev(b), to_dev(v), op=op)
    o.build(b, v, op)
    assert np.array_equal(cells_host(t), o.cells())
    extra = _keys(layout, 40_000, 13)
    m = np.concatenate([extra, b[:20_000]])
    vm = rng.integers(0, 1 << 30, m.size).astype(keys_dtype(layout))
    t.merge(to_dev(m), to_dev(vm), op=op)
    o.merge(m, vm, op)
    assert np.array_equal(cells_host(t), o.cells())
    assert t.count() == o.counts()


@pytest.mark.parametrize("layout", LAYOUTS)
def test_async_growth_contents_and_occupancy(layout):
    n = 1_500_000
    keys = _keys(layout, n, 9)
    vals = (np.arange(n) + 3).astype(keys_dtype(layout))
    from paper_1601_04017_amd import lpht
    t = make_table(layout, 12, auto_grow=True, hash=lpht.HASH_MULSHIFT, mul=MUL)
    f = to_host(t.insert_async(to_dev(keys), to_dev(vals)))
    assert (f == 1).all()
    assert t.count() == (n, n)
    g = cells_host(t)
    assert H.live_dict(g, layout) == dict(zip(keys.tolist(), vals.tolist()))
    ref = oracle.OracleTable(layout, t.log2_capacity, hash=oracle.HASH_MULSHIFT, mul=MUL)
    ref.insert(keys)
    assert np.array_equal(H.occupancy(g, layout), H.occupancy(ref.cells(), layout))
    H.check_invariants(g, layout, t.log2_capacity, n, n, mul=MUL)
