"""Pins of the oracle's full key space (Sec. 5.6): with the mode on, keys 0
(empty_key) and 1 (del_key) behave like any other key, held in two special
slots, against a dictionary model; they survive migrations and follow the
bulk build / merge rules."""
import numpy as np
import pytest

import oracle
from paper_1601_04017_amd import inputs
from tests import helpers as H

LAYOUTS = [oracle.PACKED32, oracle.KV64]


def _dt(layout):
    return np.uint32 if layout == oracle.PACKED32 else np.uint64


def _mask(layout):
    return 0xFFFFFFFF if layout == oracle.PACKED32 else (1 << 64) - 1


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("seed", range(8))
def test_sequences_with_keys_0_and_1_match_dict_model(layout, seed):
    rng = np.random.default_rng(seed)
    t = oracle.OracleTable(layout, 6, full_keys=True)
    model = {}
    m = _mask(layout)
    for step in range(60):
        kind = rng.integers(0, 6)
        keys = rng.integers(0, 6, int(rng.integers(1, 12))).astype(_dt(layout))
        vals = rng.integers(0, 1 << 31, keys.size).astype(_dt(layout))
        if kind == 0:
            f = t.insert(keys, vals)
            want = []
            for k, v in zip(keys.tolist(), vals.tolist()):
                want.append(0 if k in model else 1)
                model.setdefault(k, v)
        elif kind in (1, 2):
            op = oracle.ADD if kind == 1 else oracle.ASSIGN
            f = t.insert_or_update(keys, vals, op)
            want = []
            for k, v in zip(keys.tolist(), vals.tolist()):
                want.append(0 if k in model else 1)
                model[k] = ((model.get(k, 0) + v) & m) if (op == oracle.ADD and k in model) else v
        elif kind == 3:
            f = t.update(keys, vals, oracle.ADD)
            want = []
            for k, v in zip(keys.tolist(), vals.tolist()):
                want.append(1 if k in model else 0)
                if k in model:
                    model[k] = (model[k] + v) & m
        elif kind == 4:
            f = t.erase(keys)
            want = []
            for k in keys.tolist():
                want.append(1 if k in model else 0)
                model.pop(k, None)
        else:
            v, f = t.find(keys)
            want = [1 if k in model else 0 for k in keys.tolist()]
            assert [int(x) for x in v] == [model.get(k, 0) for k in keys.tolist()]
        assert f.tolist() == want, (step, kind)
        used, live = t.counts()
        assert live == len(model)
        assert t.status() == 0  # nothing is reserved


@pytest.mark.parametrize("layout", LAYOUTS)
def test_special_keys_survive_migration_and_follow_bulk_rules(layout):
    keys = (inputs.distinct_keys_u32(500, 3) if layout == oracle.PACKED32 else inputs.distinct_keys_u64(500, 3))
    t = oracle.OracleTable(layout, 8, full_keys=True, auto_grow=True)
    t.insert(np.concatenate([keys, np.array([0, 1], dtype=_dt(layout))]), None)
    t.insert_or_update(np.array([1, 1], dtype=_dt(layout)), np.array([5, 6], dtype=_dt(layout)), oracle.ADD)
    assert t.counts() == (502, 502)
    t.grow(t.log2c + 1)
    t.erase(keys[:400])
    t.grow(t.log2c - 2)  # shrink
    v, f = t.find(np.array([0, 1], dtype=_dt(layout)))
    assert f.tolist() == [1, 1] and v.tolist() == [1, 12]
    assert t.counts() == (102, 102)
    # the cells never hold the special keys
    k, _ = H.split_cells(t.cells(), layout)
    assert set(H.live_dict(t.cells(), layout)) == set(keys[400:].tolist())
    # merge: the batch's special entries apply in order over the table's
    t.merge(np.array([1, 0, 1], dtype=_dt(layout)), np.array([2, 3, 4], dtype=_dt(layout)), oracle.ADD)
    v, f = t.find(np.array([0, 1], dtype=_dt(layout)))
    assert v.tolist() == [4, 18]
    # build: the slots start empty
    t.build(np.array([0, 5, 0], dtype=_dt(layout)), np.array([7, 8, 9], dtype=_dt(layout)))
    v, f = t.find(np.array([0, 1, 5], dtype=_dt(layout)))
    assert f.tolist() == [1, 0, 1] and v.tolist() == [9, 0, 8]
    assert t.counts() == (2, 2)
    # without the mode the keys stay reserved
    r = oracle.OracleTable(layout, 6)
    assert r.insert(np.array([0, 1], dtype=_dt(layout))).tolist() == [oracle.FLAG_RESERVED] * 2
