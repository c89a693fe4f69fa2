"""Parity of the HIP path (through the C ABI) with the CPU oracle, element by
element, on seeded inputs at sizes that span many workgroups and end in a
ragged tail.  Integer results must be identical: find flags and values,
canonicalised insert/upsert/erase flags, counts, the occupancy bitmap and the
set of keys in every run; migrations must match cell for cell."""
import numpy as np
import pytest

import oracle
from paper_1601_04017_amd import inputs
from tests import helpers as H
from tests.gpu_util import cells_host, keys_dtype, make_table, to_dev, to_host

pytestmark = pytest.mark.gpu

LAYOUTS = [oracle.PACKED32, oracle.KV64]
GROUPS = [1, 2, 4, 8, 16]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1601_04017_amd import lpht
    lpht.load()


def _keys(layout, n, seed, absent=False):
    if layout == oracle.PACKED32:
        return inputs.distinct_keys_u32(n, seed, absent=absent)
    return inputs.distinct_keys_u64(n, seed, absent=absent)


def _vals(layout, n, offset=0):
    return (np.arange(n, dtype=np.uint64) + offset).astype(keys_dtype(layout))


def _sync():
    import torch
    torch.cuda.synchronize()


@pytest.mark.parametrize("G", GROUPS)
def test_config1_packed32_insert_find(G):
    # 2^21 cells, 2^20 distinct u32 keys with value = index, then 2^20 finds
    # that are half present, half absent.
    layout, log2c, n = oracle.PACKED32, 21, 1 << 20
    keys = _keys(layout, n, 101)
    vals = _vals(layout, n)
    absent = _keys(layout, n // 2, 101, absent=True)
    present = keys[inputs.permutation(n, 102)[: n // 2]]
    fkeys, _ = inputs.shuffled_mix(present, absent, 103)

    orc = oracle.OracleTable(layout, log2c)
    of = orc.insert(keys, vals)
    ov, ofound = orc.find(fkeys)

    t = make_table(layout, log2c)
    t.set_tuning(group_width=G)
    gf = t.insert(to_dev(keys), to_dev(vals))
    gv, gfound = t.find(to_dev(fkeys))
    _sync()
    assert np.array_equal(to_host(gf), of)
    assert np.array_equal(to_host(gfound), ofound)
    assert np.array_equal(to_host(gv, np.uint32), ov)
    assert t.count() == orc.counts() == (n, n)
    assert t.status() == 0
    H.assert_same_table_modulo_run_order(cells_host(t), orc.cells(), layout)


@pytest.mark.parametrize("G", GROUPS)
@pytest.mark.parametrize("fill", [0.25, 0.5, 0.75, 0.95])
def test_kv64_insert_find_fill_levels(G, fill):
    layout, log2c = oracle.KV64, 16
    n = int(fill * (1 << log2c)) + 13  # ragged
    keys = _keys(layout, n, 7 + int(fill * 100))
    vals = _vals(layout, n, 1000)
    absent = _keys(layout, 5001, 7 + int(fill * 100), absent=True)
    fkeys = np.concatenate([keys[::3], absent])
    orc = oracle.OracleTable(layout, log2c)
    of = orc.insert(keys, vals)
    ov, ofound = orc.find(fkeys)
    t = make_table(layout, log2c)
    t.set_tuning(group_width=G, block_threads=128 if G < 4 else 256)
    gf = t.insert(to_dev(keys), to_dev(vals))
    gv, gfound = t.find(to_dev(fkeys))
    _sync()
    assert np.array_equal(to_host(gf), of)
    assert np.array_equal(to_host(gfound), ofound)
    assert np.array_equal(to_host(gv, np.uint64), ov)
    assert t.count() == orc.counts()
    cells = cells_host(t)
    H.check_invariants(cells, layout, log2c, n, n)
    H.assert_same_table_modulo_run_order(cells, orc.cells(), layout)


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("G", [1, 4, 16])
def test_insert_with_duplicates_one_winner(layout, G):
    # Exactly one of several insertions of the same absent key succeeds, and
    # the stored value is that operation's value.
    rng = np.random.default_rng(3)
    base = _keys(layout, 20000, 33)
    keys = base[rng.integers(0, base.size, 60000)]
    vals = _vals(layout, keys.size, 5)
    orc = oracle.OracleTable(layout, 16)
    of = orc.insert(keys, vals)
    t = make_table(layout, 16)
    t.set_tuning(group_width=G)
    gf = to_host(t.insert(to_dev(keys), to_dev(vals)))
    assert np.array_equal(H.canonical_flags(keys, gf), of)
    cells = cells_host(t)
    d = H.live_dict(cells, layout)
    winners = np.flatnonzero(gf == 1)
    assert len(d) == winners.size == np.unique(keys).size
    for i in winners[:5000]:
        assert d[int(keys[i])] == int(vals[i])
    ko, _, _ = H.key_run_starts(orc.cells(), layout)
    kg, _, _ = H.key_run_starts(cells, layout)
    assert np.array_equal(ko, kg)
    assert np.array_equal(H.occupancy(cells, layout), H.occupancy(orc.cells(), layout))


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("G,agg", [(1, 0), (8, 0), (1, 1)])
@pytest.mark.parametrize("s", [0.5, 1.0, 1.5])
def test_upsert_add_zipf_histogram(layout, G, agg, s):
    m = 300_001
    keys = inputs.zipf_keys_u64(m, 1_000_000, s, seed=400 + int(10 * s)).astype(keys_dtype(layout))
    vals = (np.arange(m) % 7 + 1).astype(keys_dtype(layout))
    orc = oracle.OracleTable(layout, 20)
    of = orc.insert_or_update(keys, vals, oracle.ADD)
    t = make_table(layout, 20)
    t.set_tuning(group_width=G, aggregate=agg)
    gf = to_host(t.insert_or_update(to_dev(keys), to_dev(vals), op=oracle.ADD))
    assert np.array_equal(H.canonical_flags(keys, gf), of)
    assert t.count() == orc.counts()
    H.assert_same_table_modulo_run_order(cells_host(t), orc.cells(), layout)


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("agg", [0, 1])
def test_upsert_increment_null_values(layout, agg):
    rng = np.random.default_rng(12)
    keys = rng.integers(2, 5000, size=100_000).astype(keys_dtype(layout))
    keys[::1000] = 1  # reserved keys among them
    orc = oracle.OracleTable(layout, 14)
    of = orc.insert_or_update(keys, None, oracle.ADD)
    t = make_table(layout, 14)
    t.set_tuning(aggregate=agg)
    gf = to_host(t.insert_or_update(to_dev(keys), None, op=oracle.ADD))
    assert np.array_equal(H.canonical_flags(keys, gf), of)
    from paper_1601_04017_amd import lpht
    assert t.status() == lpht.ERR_RESERVED_KEY
    H.assert_same_table_modulo_run_order(cells_host(t), orc.cells(), layout)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_upsert_add_hot_table_overflow(layout):
    # every key repeats in every chunk: more hot keys than a workgroup keeps
    rng = np.random.default_rng(14)
    keys = rng.integers(2, 260, size=2_000_000).astype(keys_dtype(layout))
    vals = rng.integers(0, 1 << 20, size=keys.size).astype(keys_dtype(layout))
    orc = oracle.OracleTable(layout, 12)
    of = orc.insert_or_update(keys, vals, oracle.ADD)
    t = make_table(layout, 12)
    gf = to_host(t.insert_or_update(to_dev(keys), to_dev(vals), op=oracle.ADD))
    assert np.array_equal(H.canonical_flags(keys, gf), of)
    H.assert_same_table_modulo_run_order(cells_host(t), orc.cells(), layout)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_upsert_add_bounded_near_full_falls_back(layout):
    # a bounded table that may fill up: combining is not used, and operations
    # on keys that find no empty cell all report "full"
    keys = _keys(layout, 70, 21)
    keys = np.concatenate([keys, keys[::-1]])
    orc = oracle.OracleTable(layout, 6)
    of = orc.insert_or_update(keys, None, oracle.ADD)
    t = make_table(layout, 6)
    gf = to_host(t.insert_or_update(to_dev(keys), None, op=oracle.ADD))
    assert (gf == 1).sum() == (of == 1).sum() == 64
    # every key that did not get a cell reports full on all its operations
    d = H.live_dict(cells_host(t), layout)
    for k, f in zip(keys.tolist(), gf.tolist()):
        assert (f == 0xFF) == (k not in d)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_upsert_assign_set_valued_under_duplicates(layout):
    rng = np.random.default_rng(13)
    base = _keys(layout, 3000, 13)
    keys = base[rng.integers(0, base.size, 20000)]
    vals = _vals(layout, keys.size, 1)
    t = make_table(layout, 14)
    gf = to_host(t.insert_or_update(to_dev(keys), to_dev(vals), op=oracle.ASSIGN))
    orc = oracle.OracleTable(layout, 14)
    of = orc.insert_or_update(keys, vals, oracle.ASSIGN)
    assert np.array_equal(H.canonical_flags(keys, gf), of)
    d = H.live_dict(cells_host(t), layout)
    allowed = {}
    for k, v in zip(keys.tolist(), vals.tolist()):
        allowed.setdefault(k, set()).add(v)
    assert set(d) == set(allowed)
    for k, v in d.items():
        assert v in allowed[k]
    # distinct keys: exact
    t2 = make_table(layout, 14)
    o2 = oracle.OracleTable(layout, 14)
    t2.insert_or_update(to_dev(base), to_dev(_vals(layout, base.size)), op=oracle.ASSIGN)
    t2.insert_or_update(to_dev(base[::2]), to_dev(_vals(layout, base[::2].size, 77)), op=oracle.ASSIGN)
    o2.insert_or_update(base, _vals(layout, base.size), oracle.ASSIGN)
    o2.insert_or_update(base[::2], _vals(layout, base[::2].size, 77), oracle.ASSIGN)
    H.assert_same_table_modulo_run_order(cells_host(t2), o2.cells(), layout)


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("G", [1, 4, 16])
def test_update_erase_find_sequence(layout, G):
    rng = np.random.default_rng(44 + G)
    log2c = 15
    keys = _keys(layout, 12000, 44)
    other = _keys(layout, 3000, 44, absent=True)
    orc = oracle.OracleTable(layout, log2c)
    t = make_table(layout, log2c)
    t.set_tuning(group_width=G)

    def both(kind, k, v=None, op=None):
        if kind == "insert":
            return t.insert(to_dev(k), None if v is None else to_dev(v)), orc.insert(k, v)
        if kind == "update":
            return (t.update(to_dev(k), None if v is None else to_dev(v), op=op), orc.update(k, v, op))
        if kind == "erase":
            return t.erase(to_dev(k)), orc.erase(k)
        raise ValueError(kind)

    g, o = both("insert", keys, _vals(layout, keys.size))
    assert np.array_equal(to_host(g), o)
    # erase with duplicates and absent keys
    ek = np.concatenate([keys[:4000], keys[:4000:2], other[:500]])
    ek = ek[rng.permutation(ek.size)]
    g, o = both("erase", ek)
    assert np.array_equal(H.canonical_flags(ek, to_host(g)), o)
    # update ADD on present, erased and absent keys (with repeats)
    uk = np.concatenate([keys[3000:6000], keys[3000:4000], other[:100]])
    g, o = both("update", uk, _vals(layout, uk.size, 3), oracle.ADD)
    assert np.array_equal(to_host(g), o)
    # update ASSIGN on distinct keys
    ak = keys[5000:9000]
    g, o = both("update", ak, _vals(layout, ak.size, 99), oracle.ASSIGN)
    assert np.array_equal(to_host(g), o)
    # re-insert some erased keys: they take new cells, tombstones stay
    g, o = both("insert", keys[:1000], _vals(layout, 1000, 7))
    assert np.array_equal(to_host(g), o)
    fk = np.concatenate([keys, other])
    gv, gfound = t.find(to_dev(fk))
    ov, ofound = orc.find(fk)
    assert np.array_equal(to_host(gfound), ofound)
    assert np.array_equal(to_host(gv, keys_dtype(layout)), ov)
    assert t.count() == orc.counts()
    cells = cells_host(t)
    H.check_invariants(cells, layout, log2c, *orc.counts())
    H.assert_same_table_modulo_run_order(cells, orc.cells(), layout)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_reserved_keys_and_status(layout):
    t = make_table(layout, 8)
    k = np.array([0, 1, 5, 6], dtype=keys_dtype(layout))
    f = to_host(t.insert(to_dev(k)))
    assert list(f) == [0xFE, 0xFE, 1, 1]
    from paper_1601_04017_amd import lpht
    assert t.status() == lpht.ERR_RESERVED_KEY
    assert t.status() == lpht.OK
    v, fo = t.find(to_dev(k))
    assert list(to_host(fo)) == [0xFE, 0xFE, 1, 1]
    assert t.count() == (2, 2)


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("G", [1, 16])
def test_bounded_table_full(layout, G):
    from paper_1601_04017_amd import lpht
    log2c = 6
    keys = _keys(layout, 80, 5)
    t = make_table(layout, log2c)
    t.set_tuning(group_width=G)
    gf = to_host(t.insert(to_dev(keys)))
    orc = oracle.OracleTable(layout, log2c)
    of = orc.insert(keys)
    # exactly 64 succeed on both; which ones depends on the order
    assert (gf == 1).sum() == 64 and (of == 1).sum() == 64
    assert (gf == 0xFF).sum() == 16
    assert t.status() == lpht.ERR_FULL
    assert t.count() == (64, 64)
    # every key that failed is absent, every key that succeeded is found
    v, fo = t.find(to_dev(keys))
    assert np.array_equal(to_host(fo) == 1, gf == 1)


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("gamma_log", [0, 1, 2])
@pytest.mark.parametrize("fill,erase_frac", [(0.45, 0.0), (0.5, 0.3), (0.8, 0.1)])
@pytest.mark.parametrize("mb", [256, 512, 1024])
def test_migration_matches_oracle_cell_for_cell(layout, gamma_log, fill, erase_frac, mb):
    log2c = 16
    n = int(fill * (1 << log2c))
    keys = _keys(layout, n, 91)
    orc = oracle.OracleTable(layout, log2c)
    orc.insert(keys, _vals(layout, n, 3))
    if erase_frac:
        rng = np.random.default_rng(5)
        orc.erase(keys[rng.random(n) < erase_frac])
    old = orc.cells()
    t = make_table(layout, log2c)
    t.set_tuning(migrate_block=mb)
    t.import_cells(to_dev(old), log2c)
    assert t.count() == orc.counts()
    t.grow(log2c + gamma_log)
    orc.grow(log2c + gamma_log)
    assert t.capacity == orc.capacity
    assert np.array_equal(cells_host(t), orc.cells())
    assert t.count() == orc.counts()


@pytest.mark.parametrize("layout", LAYOUTS)
def test_migration_wraparound_and_full_table(layout):
    log2c = 6
    kb = 4 if layout == oracle.PACKED32 else 8
    cand = np.arange(2, 400000, dtype=np.uint64)
    hm = (oracle.hash_bulk(cand, kb) >> np.uint64(64 - log2c)).astype(np.int64)
    wrap_keys = np.concatenate([cand[hm == 63][:5], cand[hm == 0][:3], cand[hm == 30][:2]])
    for ks in (wrap_keys, cand[:64]):  # the second fills the table completely
        ks = ks.astype(keys_dtype(layout))
        orc = oracle.OracleTable(layout, log2c)
        orc.insert(ks, _vals(layout, ks.size, 1))
        old = orc.cells()
        for gl in (0, 1, 3):
            t = make_table(layout, log2c)
            t.import_cells(to_dev(old), log2c)
            o2 = oracle.OracleTable(layout, log2c)
            o2.load_cells(old, log2c)
            t.grow(log2c + gl)
            o2.grow(log2c + gl)
            assert np.array_equal(cells_host(t), o2.cells()), (ks.size, gl)


def _keys_with_home(layout, log2c, home, count, start=2):
    kb = 4 if layout == oracle.PACKED32 else 8
    out = []
    lo = start
    while len(out) < count:
        cand = np.arange(lo, lo + 2_000_000, dtype=np.uint64)
        hm = (oracle.hash_bulk(cand, kb) >> np.uint64(64 - log2c)).astype(np.int64)
        out.extend(cand[hm == home].tolist())
        lo += 2_000_000
    return np.array(out[:count], dtype=keys_dtype(layout))


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("home", [100, 4095])
def test_migration_long_cluster_falls_back(layout, home):
    # one cluster of 300 cells, longer than the staging halo, plus random
    # keys; the wrapped variant starts at the last cell
    log2c = 12
    keys = np.concatenate([_keys_with_home(layout, log2c, home, 300), _keys(layout, 1200, 61)])
    orc = oracle.OracleTable(layout, log2c)
    orc.insert(keys, _vals(layout, keys.size, 9))
    old = orc.cells()
    for gl in (0, 1):
        for mb in (256, 512):
            t = make_table(layout, log2c)
            t.set_tuning(migrate_block=mb)
            t.import_cells(to_dev(old), log2c)
            o2 = oracle.OracleTable(layout, log2c)
            o2.load_cells(old, log2c)
            t.grow(log2c + gl)
            o2.grow(log2c + gl)
            assert np.array_equal(cells_host(t), o2.cells()), (gl, mb)
            assert t.count() == o2.counts()


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("log2c", [8, 9, 10])
@pytest.mark.parametrize("gamma_log", [0, 1])
def test_migration_small_tables_window_wraps(layout, log2c, gamma_log):
    # tables of one to four staging blocks: the staged window covers cells
    # twice and the wrapping cluster is seen as incoming and outgoing
    for seed, fill in ((71, 0.5), (72, 0.7), (73, 0.3)):
        n = int(fill * (1 << log2c))
        keys = np.concatenate([_keys_with_home(layout, log2c, (1 << log2c) - 2, 6), _keys(layout, n, seed)])
        orc = oracle.OracleTable(layout, log2c)
        orc.insert(keys, _vals(layout, keys.size, 3))
        orc.erase(keys[::7])
        old = orc.cells()
        t = make_table(layout, log2c)
        t.set_tuning(migrate_block=256)
        t.import_cells(to_dev(old), log2c)
        t.grow(log2c + gamma_log)
        orc.grow(log2c + gamma_log)
        assert np.array_equal(cells_host(t), orc.cells()), (seed, fill)
        assert t.count() == orc.counts()


@pytest.mark.parametrize("layout", LAYOUTS)
def test_auto_grow_batches_capacity_sequence(layout):
    # growing from 4096 cells, batches of 2^14 insertions, alpha = 1/2
    n, b = 300_000, 1 << 14
    keys = _keys(layout, n, 301)
    vals = _vals(layout, n)
    orc = oracle.OracleTable(layout, 12, auto_grow=True)
    t = make_table(layout, 12, auto_grow=True)
    t.set_timing(True)
    for lo in range(0, n, b):
        kk, vv = keys[lo:lo + b], vals[lo:lo + b]
        gf = to_host(t.insert(to_dev(kk), to_dev(vv)))
        of = orc.insert(kk, vv)
        assert np.array_equal(gf, of)
        assert t.capacity == orc.capacity, lo
    assert t.count() == orc.counts()
    st = t.stats()
    assert st["resizes"] == orc.migrations
    H.assert_same_table_modulo_run_order(cells_host(t), orc.cells(), layout)


def test_auto_grow_zipf_increment_with_cleanup():
    # insert-or-increment with erases in between: tombstones are dropped by
    # gamma = 1 or gamma = 2 migrations exactly when the oracle drops them
    layout = oracle.KV64
    orc = oracle.OracleTable(layout, 12, auto_grow=True)
    t = make_table(layout, 12, auto_grow=True)
    rng = np.random.default_rng(8)
    for r in range(12):
        keys = inputs.zipf_keys_u64(40000, 200000, 1.0, seed=900 + r)
        gf = to_host(t.insert_or_update(to_dev(keys), None, op=oracle.ADD))
        of = orc.insert_or_update(keys, None, oracle.ADD)
        assert np.array_equal(H.canonical_flags(keys, gf), of)
        ek = np.unique(keys)[rng.random(np.unique(keys).size) < 0.5]
        ge = to_host(t.erase(to_dev(ek)))
        oe = orc.erase(ek)
        assert np.array_equal(ge, oe)
        assert t.capacity == orc.capacity
        assert t.count() == orc.counts()
    H.assert_same_table_modulo_run_order(cells_host(t), orc.cells(), layout)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_empty_and_tiny_batches(layout):
    t = make_table(layout, 6)
    orc = oracle.OracleTable(layout, 6)
    e = np.zeros(0, dtype=keys_dtype(layout))
    assert to_host(t.insert(to_dev(e))).size == 0
    v, f = t.find(to_dev(e))
    assert to_host(f).size == 0
    one = np.array([12345], dtype=keys_dtype(layout))
    assert list(to_host(t.insert(to_dev(one)))) == list(orc.insert(one))
    v, f = t.find(to_dev(one))
    assert to_host(f)[0] == 1 and to_host(v)[0] == 1
    assert t.count() == (1, 1)
