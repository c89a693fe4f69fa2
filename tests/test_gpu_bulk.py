"""Sort-based bulk build and batched merge (Sec. 5.5) on the GPU against the
oracle, cell for cell: the layout (insertion in hash order) is a function of
the key set, so the device table must equal the oracle's exactly."""
import numpy as np
import pytest

import oracle
from paper_1601_04017_amd import inputs
from tests import helpers as H
from tests.gpu_util import cells_host, keys_dtype, make_table, to_dev

pytestmark = pytest.mark.gpu

LAYOUTS = [oracle.PACKED32, oracle.KV64]
OPS = [oracle.ASSIGN, oracle.ADD]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"


def _keys(layout, n, seed):
    if layout == oracle.PACKED32:
        return inputs.distinct_keys_u32(n, seed)
    return inputs.distinct_keys_u64(n, seed)


def _kb(layout):
    return 4 if layout == oracle.PACKED32 else 8


def _homed(layout, log2c, lo, hi, count, start=2):
    """`count` keys whose home lies in [lo, hi) of a 2^log2c-cell table."""
    out, base = [], start
    while len(out) < count:
        cand = np.arange(base, base + 4_000_000, dtype=np.uint64)
        hm = (oracle.hash_bulk(cand, _kb(layout)) >> np.uint64(64 - log2c)).astype(np.int64)
        out.extend(cand[(hm >= lo) & (hm < hi)].tolist())
        base += 4_000_000
    return np.array(out[:count], dtype=keys_dtype(layout))


def _batch(layout, n_distinct, dup_frac, seed):
    k = _keys(layout, n_distinct, seed)
    extra = k[np.random.default_rng(seed).integers(0, max(1, n_distinct), int(dup_frac * n_distinct))]
    b = np.concatenate([k, extra]) if n_distinct else k
    return b[inputs.permutation(b.size, seed + 1)]


def _vals(layout, n, seed):
    return np.random.default_rng(seed).integers(0, 1 << 31, n).astype(keys_dtype(layout))


def _same(t, orc, layout):
    g = cells_host(t)
    o = orc.cells()
    if not np.array_equal(g, o):
        gk, _ = H.split_cells(g, layout)
        ok, _ = H.split_cells(o, layout)
        bad = np.flatnonzero(gk != ok) if not np.array_equal(gk, ok) else np.flatnonzero(g != o)
        raise AssertionError(f"cells differ at {bad.size} places, first {bad[:8]}")
    assert t.count() == orc.counts()
    assert t.capacity == orc.capacity


# (log2 c, distinct keys, duplicate fraction): one block, several blocks,
# both partition levels, fills up to full
CASES = [(6, 10, 0.5), (6, 64, 2.0), (8, 200, 1.0), (10, 700, 0.3), (12, 4096, 0.1), (14, 9000, 1.5),
         (16, 32768, 0.5), (18, 200_000, 0.25), (20, 500_000, 0.1), (22, 2_000_000, 0.05)]


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("log2c,nd,dup", CASES)
def test_build_matches_oracle_cell_for_cell(layout, op, log2c, nd, dup):
    seed = log2c * 7 + nd % 97
    keys = _batch(layout, nd, dup, seed)
    vals = None if log2c % 4 == 0 else _vals(layout, keys.size, seed)
    t = make_table(layout, log2c)
    t.insert(to_dev(_keys(layout, (1 << log2c) // 8, seed + 5)))  # replaced by the build
    orc = oracle.OracleTable(layout, log2c)
    t.build(to_dev(keys), None if vals is None else to_dev(vals), op=op)
    orc.build(keys, vals, op)
    _same(t, orc, layout)
    assert t.status() == 0
    # the built table serves finds through the ordinary kernels
    probe = np.concatenate([keys[:: max(1, keys.size // 3000)], _keys(layout, 500, 12345)])
    gv, gf = t.find(to_dev(probe))
    ov, of = orc.find(probe)
    assert np.array_equal(gf.cpu().numpy(), of)
    assert np.array_equal(gv.cpu().numpy().view(keys_dtype(layout)), ov)


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("log2c,n_old,n_new", [(8, 100, 60), (12, 1500, 900), (16, 20000, 15000),
                                                (20, 300_000, 200_000)])
def test_merge_matches_oracle_cell_for_cell(layout, op, log2c, n_old, n_new):
    seed = log2c + n_old % 31
    old = _keys(layout, n_old, seed)
    ov = _vals(layout, n_old, seed)
    t = make_table(layout, log2c)
    orc = oracle.OracleTable(layout, log2c)
    t.insert(to_dev(old), to_dev(ov))
    orc.insert(old, ov)
    t.erase(to_dev(old[::5]))
    orc.erase(old[::5])
    # half the batch overlaps the table (erased keys included), with repeats
    fresh = _keys(layout, n_new, seed + 50)
    batch = np.concatenate([fresh[: n_new // 2], old[: n_new // 2], fresh[: n_new // 8]])
    batch = batch[inputs.permutation(batch.size, seed)]
    vals = _vals(layout, batch.size, seed + 1) if op == oracle.ADD or log2c % 8 else None
    t.merge(to_dev(batch), None if vals is None else to_dev(vals), op=op)
    orc.merge(batch, vals, op)
    _same(t, orc, layout)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_wrapping_and_full_tables(layout):
    log2c = 10
    c = 1 << log2c
    tail = _homed(layout, log2c, c - 8, c, 40)  # homes in the last 8 cells: they wrap
    head = _homed(layout, log2c, 0, 4, 6, start=9_000_000)
    rest = _keys(layout, 600, 77)
    for keys in (np.concatenate([tail, head, rest]), np.concatenate([tail, head, rest, tail])):
        t = make_table(layout, log2c)
        orc = oracle.OracleTable(layout, log2c)
        t.build(to_dev(keys))
        orc.build(keys)
        _same(t, orc, layout)
    # exactly c distinct keys: a full table; one more distinct key is refused
    full = np.unique(np.concatenate([tail, head, _keys(layout, 2000, 78)]))[:c]
    full = full[inputs.permutation(c, 3)]
    t = make_table(layout, log2c)
    orc = oracle.OracleTable(layout, log2c)
    t.build(to_dev(np.concatenate([full, full[:100]])))
    orc.build(np.concatenate([full, full[:100]]))
    _same(t, orc, layout)
    before = cells_host(t)
    from paper_1601_04017_amd import lpht
    with pytest.raises(lpht.LphtError):
        t.merge(to_dev(_keys(layout, 1, 999)))
    assert np.array_equal(cells_host(t), before) and t.count() == (c, c)


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("nhot", [600, 3000])
def test_large_blocks_sorted_by_workgroup_or_global_memory(layout, op, nhot):
    # nhot distinct keys homed in one 256-cell block (600: more than a
    # wavefront sorts, 3000: more than a workgroup sorts in LDS), each three
    # times in scattered order, plus background keys
    log2c = 16
    hot = _homed(layout, log2c, 256 * 7, 256 * 8, nhot)
    keys = np.concatenate([hot, hot, hot, _keys(layout, 5000, 31)])
    keys = keys[inputs.permutation(keys.size, 32)]
    vals = _vals(layout, keys.size, 33)
    t = make_table(layout, log2c)
    orc = oracle.OracleTable(layout, log2c)
    t.build(to_dev(keys), to_dev(vals), op=op)
    orc.build(keys, vals, op)
    _same(t, orc, layout)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_zipf_aggregation_and_auto_growth(layout):
    # insert-or-increment semantics by merging Zipf batches into a growing
    # table: values are exact counts
    t = make_table(layout, 8, auto_grow=True)
    orc = oracle.OracleTable(layout, 8, auto_grow=True)
    for r in range(3):
        z = inputs.zipf_keys_u64(400_000, 300_000, 1.0, seed=70 + r)
        z = z.astype(keys_dtype(layout))
        t.merge(to_dev(z), None, op=oracle.ADD)
        orc.merge(z, None, oracle.ADD)
        _same(t, orc, layout)
    # and a hot key a million times in one build
    hot = np.full(1_000_000, 12345, dtype=keys_dtype(layout))
    t.build(to_dev(hot), None, op=oracle.ADD)
    orc.build(hot, None, oracle.ADD)
    _same(t, orc, layout)
    assert H.live_dict(cells_host(t), layout) == {12345: 1_000_000}


@pytest.mark.parametrize("layout", LAYOUTS)
def test_edge_cases(layout):
    from paper_1601_04017_amd import lpht
    e = np.zeros(0, dtype=keys_dtype(layout))
    t = make_table(layout, 8)
    orc = oracle.OracleTable(layout, 8)
    keys = _keys(layout, 100, 5)
    t.insert(to_dev(keys))
    orc.insert(keys)
    t.erase(to_dev(keys[:40]))
    orc.erase(keys[:40])
    t.merge(to_dev(e))  # an empty batch canonicalises the table and drops tombstones
    orc.merge(e)
    _same(t, orc, layout)
    t.build(to_dev(e))  # an empty build empties it
    orc.build(e)
    _same(t, orc, layout)
    one = keys[:1]
    t.build(to_dev(one))
    orc.build(one)
    _same(t, orc, layout)
    # reserved keys are skipped and reported
    mixed = np.concatenate([keys[:10], np.array([0, 1, 0], dtype=keys_dtype(layout))])
    t.build(to_dev(mixed))
    orc.build(mixed)
    _same(t, orc, layout)
    assert t.status() == lpht.ERR_RESERVED_KEY
    with pytest.raises(lpht.LphtError):
        t.build(to_dev(keys), op=7)
    assert t.stats()["bulk_merges"] >= 4
