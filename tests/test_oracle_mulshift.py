"""Pins for the oracle's second hash function, multiplicative hashing
h(x) = (a * x) mod 2^64 with an odd multiplier a, positioned by the scaling
map of Sec. 5.3.1 (the top log2 c bits).  The paper fixes only its CRC-32C
choice (Sec. 8.3); the table takes either.  (Like the CRC pair, it spreads
consecutive keys almost without collisions, so it is not a control for
consecutive Zipf ranks: scrambled keys are.)

Everything here is checked against numpy's wrapping u64 product, computed
without the oracle: the closed form, exact cell positions, the dictionary
model with the table invariants, migration, and the order of the sort-based
bulk build (Sec. 5.5) on inputs that contain ties of the upper hash half."""
import numpy as np
import pytest

import oracle
from paper_1601_04017_amd import inputs
from tests import helpers as H
from tests import test_oracle_table as TT

LAYOUTS = [oracle.PACKED32, oracle.KV64]
MULS = [0x9E3779B97F4A7C15, 0xD6E8FEB86659FD93, 3]


def test_mulshift_closed_form():
    rng = np.random.default_rng(41)
    for _ in range(3000):
        k = int(rng.integers(0, 1 << 63)) * 2 + int(rng.integers(0, 2))
        a = int(rng.integers(0, 1 << 62)) * 2 + 1
        assert oracle.mulshift(k, a) == (k * a) % (1 << 64)
    assert oracle.mulshift(0, MULS[0]) == 0
    assert oracle.mulshift(1, MULS[0]) == MULS[0]
    assert oracle.mulshift((1 << 64) - 1, 1) == (1 << 64) - 1


def test_even_multiplier_rejected():
    with pytest.raises(ValueError):
        oracle.OracleTable(oracle.KV64, 8, hash=oracle.HASH_MULSHIFT, mul=2)


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("mul", MULS[:2])
def test_keys_with_distinct_homes_sit_at_their_homes(layout, mul):
    # keys whose homes (closed form) are pairwise distinct must each land
    # exactly on its home: this fixes the position function cell by cell
    log2c = 12
    rng = np.random.default_rng(5)
    cand = rng.integers(2, 1 << 32 if layout == oracle.PACKED32 else 1 << 62, size=6000).astype(np.uint64)
    hm = H.homes(cand, layout, log2c, mul=mul)
    _, first = np.unique(hm, return_index=True)
    keys = cand[np.sort(first)][:1500]
    t = oracle.OracleTable(layout, log2c, hash=oracle.HASH_MULSHIFT, mul=mul)
    t.insert(keys, keys)
    k_cells, _ = H.split_cells(t.cells(), layout)
    exp = np.zeros(1 << log2c, np.uint64)
    exp[H.homes(keys, layout, log2c, mul=mul)] = keys
    assert np.array_equal(k_cells, exp)


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("log2c", [3, 5, 6])
def test_random_sequences_match_dict_model(layout, log2c):
    rng = np.random.default_rng(77 + 10 * layout + log2c)
    mul = MULS[log2c % 3]
    for _ in range(20):
        t = oracle.OracleTable(layout, log2c, hash=oracle.HASH_MULSHIFT, mul=mul)
        m = H.DictModel(1 << log2c, TT._vmask(layout))
        for kind, keys, vals in TT._random_ops(rng, 25, 41):
            keys = np.asarray(keys, dtype=t.kdt)
            v = None if vals is None else np.asarray(vals, dtype=t.kdt)
            vv = [1] * keys.size if vals is None else [int(x) for x in v]
            if kind == "insert":
                f, exp = t.insert(keys, v), [m.insert(int(k), x) for k, x in zip(keys, vv)]
            elif kind.startswith("upsert"):
                op = oracle.ADD if kind.endswith("add") else oracle.ASSIGN
                f, exp = t.insert_or_update(keys, v, op), [m.upsert(int(k), x, op) for k, x in zip(keys, vv)]
            elif kind.startswith("update"):
                op = oracle.ADD if kind.endswith("add") else oracle.ASSIGN
                f, exp = t.update(keys, v, op), [m.update(int(k), x, op) for k, x in zip(keys, vv)]
            elif kind == "find":
                gv, f = t.find(keys)
                pairs = [m.find(int(k)) for k in keys]
                exp = [p[0] for p in pairs]
                assert [int(x) for x in gv] == [p[1] for p in pairs]
            else:
                f, exp = t.erase(keys), [m.erase(int(k)) for k in keys]
            assert [int(x) for x in f] == exp, kind
            used, live = t.counts()
            cells = t.cells()
            assert H.live_dict(cells, layout) == m.d
            H.check_invariants(cells, layout, log2c, used, live, mul=mul)


def test_mulshift_is_a_bijection_of_u64():
    # an odd multiplier is invertible mod 2^64: distinct keys get distinct
    # 64-bit hashes (the CRC pair has only 2^32 values) and the inverse
    # multiplier recovers every key
    keys = inputs.distinct_keys_u64(1 << 20, 43)
    for mul in MULS:
        h = np.array([oracle.mulshift(int(k), mul) for k in keys[:2000]], np.uint64)
        assert np.array_equal(h, H.mulshift_hash(keys[:2000], mul))
        hh = H.mulshift_hash(keys, mul)
        assert np.unique(hh).size == keys.size
        assert np.array_equal(H.mulshift_hash(hh, pow(mul, -1, 1 << 64)), keys)


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("gamma_log", [0, 1, 2])
def test_migration_keeps_contents_and_positions(layout, gamma_log):
    # a grown (or cleaned) table holds the live keys, each reachable from its
    # closed-form home in the new size, with the occupied cells of inserting
    # them into an empty table (occupancy is order independent)
    log2c, mul = 12, MULS[0]
    keys = inputs.distinct_keys_u32(1800, 61).astype(np.uint64)
    t = oracle.OracleTable(layout, log2c, hash=oracle.HASH_MULSHIFT, mul=mul)
    t.insert(keys, keys)
    t.erase(keys[::3])
    t.grow(log2c + gamma_log)
    live = keys[np.arange(keys.size) % 3 != 0]
    cells = t.cells()
    assert H.live_dict(cells, layout) == {int(k): int(k) for k in live}
    H.check_invariants(cells, layout, log2c + gamma_log, live.size, live.size, mul=mul)
    ref = oracle.OracleTable(layout, log2c + gamma_log, hash=oracle.HASH_MULSHIFT, mul=mul)
    ref.insert(live[::-1].copy(), live[::-1].copy())
    assert np.array_equal(H.occupancy(cells, layout), H.occupancy(ref.cells(), layout))


@pytest.mark.parametrize("layout", LAYOUTS)
def test_bulk_build_order_upper_half_then_key(layout):
    # Sec. 5.5 sorts by hash: the oracle orders by the upper 32 hash bits,
    # then by key.  The batch holds keys whose products share the upper half
    # (x and x + d with a*d < 2^32 mod 2^64 differ only in the lower half),
    # so the tie rule matters; the build must equal inserting the elements
    # one by one in that order (computed here with numpy) into an empty table.
    # a * step = -5 (KV64) or -3 (u32 keys: a = 2^64 - 3, step 1) modulo
    # 2^64: x and x + step share the upper half unless a borrow crosses, and
    # the larger key has the smaller lower half, so ordering ties by key
    # differs from ordering by the whole hash
    mul = MULS[0] if layout == oracle.KV64 else (1 << 64) - 3
    log2c = 14
    rng = np.random.default_rng(8)
    base = rng.integers(2, 1 << 31, size=3000).astype(np.uint64)
    step = np.uint64((pow(mul, -1, 1 << 64) * ((1 << 64) - 5)) % (1 << 64)) if layout == oracle.KV64 \
        else np.uint64(1)
    with np.errstate(over="ignore"):
        twin = base + step
    keys = np.unique(np.concatenate([twin, base]))
    keys = keys[rng.permutation(keys.size)]
    h = H.mulshift_hash(keys, mul)
    up = h >> np.uint64(32)
    assert np.unique(up).size < keys.size - 1000  # many ties, or the test is vacuous
    assert not np.array_equal(np.lexsort((keys, up)), np.argsort(h, kind="stable"))
    order = np.lexsort((keys, up))
    b = oracle.OracleTable(layout, log2c, hash=oracle.HASH_MULSHIFT, mul=mul)
    b.build(keys, keys)
    ref = oracle.OracleTable(layout, log2c, hash=oracle.HASH_MULSHIFT, mul=mul)
    ref.insert(keys[order], keys[order])
    assert np.array_equal(b.cells(), ref.cells())
