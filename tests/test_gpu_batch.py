"""Multi-table batches (one launch per operation group over many tables and
calls of uneven length) against the oracle: the same results as running each
call alone on its table, and phase order for mixed requests."""
import numpy as np
import pytest

import oracle
from paper_1601_04017_amd import inputs
from tests import helpers as H
from tests.gpu_util import cells_host, keys_dtype, make_table, to_dev, to_host

pytestmark = pytest.mark.gpu

FIND, INSERT, UPSERT, UPDATE, ERASE = 0, 1, 2, 3, 4


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"


def _keys(layout, n, seed, absent=False):
    if layout == oracle.PACKED32:
        return inputs.distinct_keys_u32(n, seed, absent=absent)
    return inputs.distinct_keys_u64(n, seed, absent=absent)


def _batch(max_ops=64):
    from paper_1601_04017_amd import lpht
    return lpht.Batch(max_ops)


LENGTHS = [0, 1, 127, 128, 129, 1000, 5000, 20000]


@pytest.mark.parametrize("G", [1, 4])
def test_batch_inserts_and_finds_many_tables(G):
    import torch
    rng = np.random.default_rng(1)
    tabs, orcs, data = [], [], []
    for j, n in enumerate(LENGTHS * 2):
        layout = oracle.PACKED32 if j % 2 else oracle.KV64
        log2c = 10 + j % 7
        n = min(n, (1 << log2c) // 2)
        k = _keys(layout, n, 100 + j)
        v = (np.arange(n) + 7 * j).astype(keys_dtype(layout))
        t = make_table(layout, log2c)
        t.set_tuning(group_width=G)
        tabs.append(t)
        orcs.append(oracle.OracleTable(layout, log2c))
        data.append((layout, k, v))
    b = _batch()
    ops, outs = [], []
    for t, (layout, k, v) in zip(tabs, data):
        f = torch.empty(k.size, dtype=torch.uint8, device="cuda")
        ops.append({"table": t, "op": INSERT, "keys": to_dev(k), "vals": to_dev(v), "flags": f})
        outs.append(f)
    b.run(ops)
    fops, fouts = [], []
    for t, (layout, k, v) in zip(tabs, data):
        fk = np.concatenate([k[::2], _keys(layout, 300, 900, absent=True)]) if k.size else k
        vo = torch.empty(fk.size, dtype=t.torch_dtype, device="cuda")
        fo = torch.empty(fk.size, dtype=torch.uint8, device="cuda")
        fops.append({"table": t, "op": FIND, "keys": to_dev(fk), "vals_out": vo, "flags": fo})
        fouts.append((fk, vo, fo))
    b.run(fops)
    for t, o, (layout, k, v), f, (fk, vo, fo) in zip(tabs, orcs, data, outs, fouts):
        of = o.insert(k, v)
        assert np.array_equal(to_host(f), of)
        ov, ofound = o.find(fk)
        assert np.array_equal(to_host(fo), ofound)
        assert np.array_equal(to_host(vo, keys_dtype(layout)), ov)
        assert t.count() == o.counts()
        H.assert_same_table_modulo_run_order(cells_host(t), o.cells(), layout)


@pytest.mark.parametrize("layout", [oracle.PACKED32, oracle.KV64])
def test_batch_mixed_requests_phase_order(layout):
    # one request per table with 60 % finds, 30 % insert-or-increment, 10 %
    # erases over Zipf keys; phases: finds see the state at request start,
    # then the increments, then the erases
    import torch
    tabs, orcs, reqs = [], [], []
    for j in range(10):
        log2c = 12 + j % 5
        t = make_table(layout, log2c, auto_grow=True)
        o = oracle.OracleTable(layout, log2c, auto_grow=True)
        pre = inputs.zipf_keys_u64(3000, 20000, 1.0, seed=700 + j).astype(keys_dtype(layout))
        t.insert_or_update(to_dev(pre), None, op=oracle.ADD)
        o.insert_or_update(pre, None, oracle.ADD)
        tabs.append(t)
        orcs.append(o)
    b = _batch()
    for rnd in range(3):
        ops, outs = [], []
        for j, t in enumerate(tabs):
            n = [0, 1, 500, 4000, 17000][(j + rnd) % 5]
            rng = np.random.default_rng(1000 * rnd + j)
            k = inputs.zipf_keys_u64(n, 20000, 1.0, seed=800 + 31 * rnd + j).astype(keys_dtype(layout))
            kinds = rng.choice(np.array([0, 1, 2], np.uint8), size=n, p=[0.6, 0.3, 0.1])
            dk, dkind = to_dev(k), to_dev(kinds)
            vo = torch.full((n,), -1, dtype=t.torch_dtype, device="cuda")
            fo = torch.full((n,), 0x77, dtype=torch.uint8, device="cuda")
            for op, sel in ((FIND, 0), (UPSERT, 1), (ERASE, 2)):
                d = {"table": t, "op": op, "keys": dk, "flags": fo, "kinds": dkind, "kind_sel": sel,
                     "count_sel": int((kinds == sel).sum())}
                if op == FIND:
                    d["vals_out"] = vo
                if op == UPSERT:
                    d["up"] = oracle.ADD
                ops.append(d)
            outs.append((k, kinds, vo, fo))
        b.run(ops)
        for t, o, (k, kinds, vo, fo) in zip(tabs, orcs, outs):
            gf = to_host(fo)
            gv = to_host(vo, keys_dtype(layout))
            m0, m1, m2 = kinds == 0, kinds == 1, kinds == 2
            ov, of = o.find(k[m0])
            assert np.array_equal(gf[m0], of)
            assert np.array_equal(gv[m0], ov)
            if m0.any():
                assert np.all(gv[~m0] == 0)
            ou = o.insert_or_update(k[m1], None, oracle.ADD)
            assert np.array_equal(H.canonical_flags(k[m1], gf[m1]), ou)
            oe = o.erase(k[m2])
            assert np.array_equal(H.canonical_flags(k[m2], gf[m2]), oe)
            assert t.count() == o.counts()
            assert t.capacity == o.capacity
    for t, o in zip(tabs, orcs):
        H.assert_same_table_modulo_run_order(cells_host(t), o.cells(), layout)


def test_batch_same_table_twice_in_a_group():
    import torch
    layout = oracle.KV64
    t = make_table(layout, 14)
    o = oracle.OracleTable(layout, 14)
    k = _keys(layout, 6000, 5)
    a, c = k[:2500], k[2000:]  # overlapping: 500 keys inserted by both
    fa = torch.empty(a.size, dtype=torch.uint8, device="cuda")
    fc = torch.empty(c.size, dtype=torch.uint8, device="cuda")
    _batch().run([{"table": t, "op": INSERT, "keys": to_dev(a), "flags": fa},
                  {"table": t, "op": INSERT, "keys": to_dev(c), "flags": fc}])
    both = np.concatenate([a, c])
    gf = np.concatenate([to_host(fa), to_host(fc)])
    of = o.insert(both)
    assert np.array_equal(H.canonical_flags(both, gf), of)
    assert t.count() == o.counts()
