"""Pins for the oracle's table operations (Sec. 4, Algorithm 1 and its insert /
update variants, tombstone deletion of Sec. 5.4): brute force against a
dictionary model on tiny inputs, the linear-probing invariants, order
independence of the occupied cell set, and expected probe lengths."""
import numpy as np
import pytest
from hypothesis import given, settings
from hypothesis import strategies as st

import oracle
from paper_1601_04017_amd import inputs
from tests import helpers as H

LAYOUTS = [oracle.PACKED32, oracle.KV64]


def _vmask(layout):
    return 0xFFFFFFFF if layout == oracle.PACKED32 else 0xFFFFFFFFFFFFFFFF


def _replay(layout, log2c, ops):
    """Apply (kind, keys, vals) batches to the oracle and to the dict model,
    comparing every flag and value.  Returns the oracle table."""
    t = oracle.OracleTable(layout, log2c)
    m = H.DictModel(1 << log2c, _vmask(layout))
    for kind, keys, vals in ops:
        keys = np.asarray(keys, dtype=t.kdt)
        v = None if vals is None else np.asarray(vals, dtype=t.kdt)
        vv = [1] * keys.size if vals is None else [int(x) for x in v]
        if kind == "insert":
            f = t.insert(keys, v)
            exp = [m.insert(int(k), x) for k, x in zip(keys, vv)]
        elif kind in ("upsert_add", "upsert_assign"):
            op = oracle.ADD if kind == "upsert_add" else oracle.ASSIGN
            f = t.insert_or_update(keys, v, op)
            exp = [m.upsert(int(k), x, op) for k, x in zip(keys, vv)]
        elif kind in ("update_add", "update_assign"):
            op = oracle.ADD if kind == "update_add" else oracle.ASSIGN
            f = t.update(keys, v, op)
            exp = [m.update(int(k), x, op) for k, x in zip(keys, vv)]
        elif kind == "find":
            got_v, f = t.find(keys)
            pairs = [m.find(int(k)) for k in keys]
            exp = [p[0] for p in pairs]
            assert [int(x) for x in got_v] == [p[1] for p in pairs]
        elif kind == "erase":
            f = t.erase(keys)
            exp = [m.erase(int(k)) for k in keys]
        else:
            raise ValueError(kind)
        assert [int(x) for x in f] == exp, kind
        used, live = t.counts()
        assert used == m.used and live == len(m.d)
        cells = t.cells()
        assert H.live_dict(cells, layout) == m.d
        H.check_invariants(cells, layout, log2c, used, live)
    return t


KINDS = ["insert", "upsert_add", "upsert_assign", "update_add", "update_assign", "find", "erase"]


def _random_ops(rng, nbatches, universe_hi, with_reserved=True):
    ops = []
    for _ in range(nbatches):
        kind = KINDS[int(rng.integers(0, len(KINDS)))]
        n = int(rng.integers(1, 12))
        lo = 0 if with_reserved and rng.random() < 0.1 else 2
        keys = rng.integers(lo, universe_hi, size=n)
        vals = None if rng.random() < 0.3 else rng.integers(0, 1 << 32, size=n)
        ops.append((kind, keys, vals))
    return ops


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("log2c", [3, 4, 5, 6])
def test_random_sequences_match_dict_model(layout, log2c):
    rng = np.random.default_rng(1000 * layout + log2c)
    for _ in range(30):
        _replay(layout, log2c, _random_ops(rng, 25, 41))


@settings(max_examples=150, deadline=None)
@given(layout=st.sampled_from(LAYOUTS), log2c=st.integers(3, 6),
       ops=st.lists(st.tuples(st.sampled_from(KINDS),
                              st.lists(st.integers(0, 40), min_size=1, max_size=10),
                              st.integers(0, 2 ** 32 - 1)),
                    min_size=1, max_size=30))
def test_property_sequences(layout, log2c, ops):
    batches = [(k, keys, [(v + i) % 2 ** 32 for i in range(len(keys))]) for k, keys, v in ops]
    _replay(layout, log2c, batches)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_fill_to_full_then_full_flag(layout):
    t = oracle.OracleTable(layout, 3)
    keys = np.arange(2, 12)
    f = t.insert(keys, keys)
    assert list(f[:8]) == [1] * 8
    assert list(f[8:]) == [oracle.FLAG_FULL] * 2
    assert t.status() == oracle.STICKY_FULL
    assert t.status() == 0
    # present keys are still found by a full scan; absent ones are not
    v, fl = t.find(np.array([2, 9, 11, 100]))
    assert list(fl) == [1, 1, 0, 0]
    # erase makes tombstones that are never reused: still full
    assert list(t.erase(np.array([2]))) == [1]
    assert list(t.insert(np.array([2]))) == [oracle.FLAG_FULL]


@pytest.mark.parametrize("layout", LAYOUTS)
def test_reserved_keys(layout):
    t = oracle.OracleTable(layout, 4)
    assert list(t.insert(np.array([0, 1, 5]))) == [0xFE, 0xFE, 1]
    assert t.status() == oracle.STICKY_RESERVED
    v, f = t.find(np.array([0, 1, 5]))
    assert list(f) == [0xFE, 0xFE, 1] and list(v) == [0, 0, 1]
    assert t.counts() == (1, 1)


def test_packed32_add_wraps_mod_2_32():
    t = oracle.OracleTable(oracle.PACKED32, 4)
    t.insert_or_update(np.array([7], np.uint32), np.array([0xFFFFFFF0], np.uint32), oracle.ADD)
    t.insert_or_update(np.array([7], np.uint32), np.array([0x20], np.uint32), oracle.ADD)
    v, f = t.find(np.array([7]))
    assert f[0] == 1 and v[0] == 0x10


def test_kv64_add_wraps_mod_2_64():
    t = oracle.OracleTable(oracle.KV64, 4)
    t.insert_or_update(np.array([7], np.uint64), np.array([2 ** 64 - 3], np.uint64), oracle.ADD)
    t.insert_or_update(np.array([7], np.uint64), np.array([5], np.uint64), oracle.ADD)
    v, f = t.find(np.array([7], np.uint64))
    assert f[0] == 1 and int(v[0]) == 2


@pytest.mark.parametrize("layout", LAYOUTS)
def test_occupancy_independent_of_insertion_order(layout):
    # With insert-only linear probing the set of occupied cells depends only on
    # the multiset of homes, and each maximal run holds the same keys.
    rng = np.random.default_rng(21)
    for log2c in (6, 10, 14):
        c = 1 << log2c
        n = int(c * 0.8)
        keys = inputs.distinct_keys_u32(n, seed=log2c)
        a = oracle.OracleTable(layout, log2c)
        b = oracle.OracleTable(layout, log2c)
        a.insert(keys, keys)
        b.insert(keys[::-1].copy(), keys[::-1].copy())
        ca, cb = a.cells(), b.cells()
        assert np.array_equal(H.occupancy(ca, layout), H.occupancy(cb, layout))
        assert H.runs_key_sets(ca, layout) == H.runs_key_sets(cb, layout)
        H.check_invariants(ca, layout, log2c, n, n)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_brute_force_histogram_of_upserts(layout):
    # insertOrIncrement over a stream with repeats: final counts equal the
    # histogram computed by sort + unique + count.
    rng = np.random.default_rng(31)
    keys = rng.integers(2, 3000, size=20000)
    t = oracle.OracleTable(layout, 13)
    f = t.insert_or_update(keys, None, oracle.ADD)
    uk, first, cnt = np.unique(keys, return_index=True, return_counts=True)
    d = H.live_dict(t.cells(), layout)
    assert d == dict(zip(uk.tolist(), cnt.tolist()))
    # exactly the first occurrence of each key reports "inserted"
    exp = np.zeros(keys.size, np.uint8)
    exp[first] = 1
    assert np.array_equal(f, exp)


@pytest.mark.parametrize("alpha", [0.25, 0.5, 0.75])
def test_expected_probe_lengths_knuth(alpha):
    # Linear probing with a random hash: successful searches inspect about
    # (1 + 1/(1-a))/2 cells, unsuccessful about (1 + 1/(1-a)^2)/2 (Knuth,
    # TAOCP vol. 3, 6.4; cited in Sec. 3).  Statistical sanity check.
    log2c = 18
    c = 1 << log2c
    n = int(alpha * c)
    rng = np.random.default_rng(int(alpha * 100))
    present = inputs.distinct_keys_u64(n, seed=int(alpha * 100))
    absent = inputs.distinct_keys_u64(20000, seed=int(alpha * 100), absent=True)
    t = oracle.OracleTable(oracle.KV64, log2c)
    t.insert(present, present)
    samp = present[rng.integers(0, n, 20000)]
    ls = np.mean([t.probe_count(int(k)) for k in samp])
    lu = np.mean([t.probe_count(int(k)) for k in absent])
    es = 0.5 * (1 + 1 / (1 - alpha))
    eu = 0.5 * (1 + 1 / (1 - alpha) ** 2)
    assert abs(ls - es) / es < 0.05, (ls, es)
    assert abs(lu - eu) / eu < 0.10, (lu, eu)
