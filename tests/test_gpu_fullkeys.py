"""Full key space (Sec. 5.6) on the GPU: keys 0 and 1 in the special slots,
operation by operation against the oracle with the same mode, mixed with
ordinary keys, through the bulk calls, growth, the sort-based build / merge
and the in-kernel growing insert."""
import numpy as np
import pytest

import oracle
from paper_1601_04017_amd import inputs
from tests import helpers as H
from tests.gpu_util import cells_host, keys_dtype, make_table, to_dev, to_host

pytestmark = pytest.mark.gpu

LAYOUTS = [oracle.PACKED32, oracle.KV64]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"


def _mixed(layout, n, seed, p_special=0.02):
    rng = np.random.default_rng(seed)
    base = rng.integers(2, 5000, n).astype(keys_dtype(layout))
    sp = rng.random(n) < p_special
    base[sp] = rng.integers(0, 2, int(sp.sum())).astype(keys_dtype(layout))
    return base


@pytest.mark.parametrize("layout", LAYOUTS)
def test_operation_sequences_match_oracle(layout):
    rng = np.random.default_rng(4)
    t = make_table(layout, 12, auto_grow=True, full_keys=True)
    orc = oracle.OracleTable(layout, 12, auto_grow=True, full_keys=True)
    dt = keys_dtype(layout)
    for step in range(30):
        keys = _mixed(layout, int(rng.integers(1, 40000)), 100 + step)
        vals = rng.integers(0, 1 << 31, keys.size).astype(dt)
        kind = step % 5
        if kind == 0:
            # which of equal concurrent inserts wins is unspecified: ordinary
            # keys are distinct here (keys 0 and 1 go in index order)
            normal = np.unique(keys[keys > 1])
            normal = normal[np.random.default_rng(step).permutation(normal.size)]
            keys = np.concatenate([normal, keys[keys <= 1]])
            keys = keys[np.random.default_rng(step + 1).permutation(keys.size)]
            vals = vals[: keys.size]
            g = to_host(t.insert(to_dev(keys), to_dev(vals)))
            o = orc.insert(keys, vals)
            assert np.array_equal(H.canonical_flags(keys, g), o)
        elif kind == 1:
            g = to_host(t.insert_or_update(to_dev(keys), to_dev(vals), op=oracle.ADD))
            o = orc.insert_or_update(keys, vals, oracle.ADD)
            assert np.array_equal(H.canonical_flags(keys, g), o)
        elif kind == 2:
            g = to_host(t.update(to_dev(keys), to_dev(vals), op=oracle.ADD))
            o = orc.update(keys, vals, oracle.ADD)
            assert np.array_equal(g, o)
        elif kind == 3:
            ek = np.unique(keys)
            g = to_host(t.erase(to_dev(ek)))
            o = orc.erase(ek)
            assert np.array_equal(g, o)
        else:
            gv, gf = t.find(to_dev(keys))
            ov, of = orc.find(keys)
            assert np.array_equal(to_host(gf), of)
            assert np.array_equal(to_host(gv, dt), ov)
        assert t.count() == orc.counts(), step
        assert t.status() == 0
    # the special keys never enter the cells
    k, _ = H.split_cells(cells_host(t), layout)
    assert H.live_dict(cells_host(t), layout).keys() == H.live_dict(orc.cells(), layout).keys()
    probe = np.array([0, 1, 2, 3], dtype=dt)
    gv, gf = t.find(to_dev(probe))
    ov, of = orc.find(probe)
    assert np.array_equal(to_host(gf), of) and np.array_equal(to_host(gv, dt), ov)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_many_special_operations_in_one_call(layout):
    # more operations on keys 0 and 1 than the list holds: the ordered scan
    dt = keys_dtype(layout)
    keys = np.concatenate([np.zeros(6000, dtype=dt), np.ones(6000, dtype=dt), _keys2(layout)])
    keys = keys[inputs.permutation(keys.size, 3)]
    vals = (np.arange(keys.size) % 1000).astype(dt)
    t = make_table(layout, 14, full_keys=True)
    orc = oracle.OracleTable(layout, 14, full_keys=True)
    g = to_host(t.insert_or_update(to_dev(keys), to_dev(vals), op=oracle.ADD))
    o = orc.insert_or_update(keys, vals, oracle.ADD)
    assert np.array_equal(H.canonical_flags(keys, g), o)
    gv, gf = t.find(to_dev(np.array([0, 1], dtype=dt)))
    ov, of = orc.find(np.array([0, 1], dtype=dt))
    assert np.array_equal(to_host(gv, dt), ov) and t.count() == orc.counts()


def _keys2(layout):
    return inputs.distinct_keys_u32(3000, 8) if layout == oracle.PACKED32 else inputs.distinct_keys_u64(3000, 8)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_build_merge_and_async_insert_with_special_keys(layout):
    dt = keys_dtype(layout)
    keys = np.concatenate([_keys2(layout), np.array([1, 0, 1, 0, 1], dtype=dt)])
    keys = keys[inputs.permutation(keys.size, 5)]
    vals = (np.arange(keys.size) + 3).astype(dt)
    for op in (oracle.ASSIGN, oracle.ADD):
        t = make_table(layout, 14, full_keys=True)
        orc = oracle.OracleTable(layout, 14, full_keys=True)
        t.insert(to_dev(np.array([0], dtype=dt)), to_dev(np.array([77], dtype=dt)))
        orc.insert(np.array([0], dtype=dt), np.array([77], dtype=dt))
        t.merge(to_dev(keys), to_dev(vals), op=op)
        orc.merge(keys, vals, op)
        assert np.array_equal(cells_host(t), orc.cells())
        assert t.count() == orc.counts()
        probe = np.array([0, 1], dtype=dt)
        gv, _ = t.find(to_dev(probe))
        assert np.array_equal(to_host(gv, dt), orc.find(probe)[0])
        t.build(to_dev(keys[:10]), to_dev(vals[:10]), op=op)
        orc.build(keys[:10], vals[:10], op)
        assert np.array_equal(cells_host(t), orc.cells()) and t.count() == orc.counts()
        gv, gf = t.find(to_dev(probe))
        ov, of = orc.find(probe)
        assert np.array_equal(to_host(gf), of) and np.array_equal(to_host(gv, dt), ov)
    # the growing insert: keys 0 and 1 go to the slots
    t = make_table(layout, 12, auto_grow=True, full_keys=True)
    big = np.concatenate([inputs.distinct_keys_u32(100_000, 9).astype(dt) if layout == oracle.PACKED32
                          else inputs.distinct_keys_u64(100_000, 9), np.array([0, 1, 1], dtype=dt)])
    f = to_host(t.insert_async(to_dev(big), None, add=True))
    assert f[-3:].tolist() == [1, 1, 0]
    gv, gf = t.find(to_dev(np.array([0, 1], dtype=dt)))
    assert to_host(gv, dt).tolist() == [1, 2]
    assert t.count() == (100_002, 100_002)


def test_batch_api_refuses_full_key_tables():
    from paper_1601_04017_amd import lpht
    t = make_table(oracle.KV64, 10, full_keys=True)
    b = lpht.Batch(max_ops=4)
    with pytest.raises(lpht.LphtError):
        b.run([dict(table=t, op=lpht.OP_FIND, keys=to_dev(np.array([5], dtype=np.uint64)))])
    b.close()
