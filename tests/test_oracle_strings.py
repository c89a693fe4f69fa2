"""Pins of the oracle's string-key table (Sec. 5.7): the string hash against
the pinned word hash and its closed form for the empty string, operation
sequences against a dictionary model (growth included), the linear probing
invariants, and occupancy independent of insertion order."""
import numpy as np
import pytest

import oracle


def _rand_strings(rng, n, universe, maxlen=24):
    pool = [bytes(rng.integers(0, 256, int(rng.integers(0, maxlen + 1))).astype(np.uint8)) for _ in range(universe)]
    return [pool[i] for i in rng.integers(0, universe, n)], pool


def test_string_hash_equals_word_hash_and_seed_closed_form():
    rng = np.random.default_rng(1)
    for w in rng.integers(0, 1 << 63, 200, dtype=np.uint64).tolist():
        assert oracle.str_hash(int(w).to_bytes(8, "little")) == oracle.hash64(int(w), 8)
        w32 = int(w) & 0xFFFFFFFF
        assert oracle.str_hash(w32.to_bytes(4, "little")) == oracle.hash64(w32, 4)
    # the register update over no byte leaves the seeds
    assert oracle.str_hash(b"") == (oracle.SEED_HI << 32) | oracle.SEED_LO
    assert oracle.str_hash(b"", 5, 7) == (5 << 32) | 7


def _check_invariants(t):
    cells = t.cells()
    c = len(cells)
    log2c = c.bit_length() - 1
    seen = set()
    for i, x in enumerate(cells):
        if not x:
            continue
        key, _ = x
        assert key not in seen
        seen.add(key)
        h = oracle.str_hash(key) >> (64 - log2c)
        j = h
        while j != i:  # reachable: no empty cell between home and position
            assert cells[j] is not None
            j = (j + 1) % c
    return seen


@pytest.mark.parametrize("seed", range(6))
def test_sequences_match_dict_model(seed):
    rng = np.random.default_rng(seed)
    t = oracle.OracleStrTable(4, auto_grow=True)
    model = {}
    for step in range(40):
        keys, _ = _rand_strings(rng, int(rng.integers(1, 30)), 40)
        vals = rng.integers(0, 1 << 40, len(keys)).astype(np.uint64)
        kind = int(rng.integers(0, 4))
        if kind == 0:
            f = t.insert(keys, vals)
            want = []
            for k, v in zip(keys, vals.tolist()):
                want.append(0 if k in model else 1)
                model.setdefault(k, v)
        elif kind == 1:
            f = t.insert_or_update(keys, vals, oracle.ADD)
            want = []
            for k, v in zip(keys, vals.tolist()):
                want.append(0 if k in model else 1)
                model[k] = (model[k] + v) % (1 << 64) if k in model else v
        elif kind == 2:
            v, f = t.find(keys)
            want = [1 if k in model else 0 for k in keys]
            assert v.tolist() == [model.get(k, 0) for k in keys]
        else:
            f = t.erase(keys)
            want = []
            for k in keys:
                want.append(1 if k in model else 0)
                model.pop(k, None)
        assert f.tolist() == want, (step, kind)
        assert t.counts()[1] == len(model)
        assert _check_invariants(t) == set(model)


def test_occupancy_independent_of_order_and_migration():
    rng = np.random.default_rng(9)
    _, pool = _rand_strings(rng, 1, 700)
    pool = list(dict.fromkeys(pool))
    a = oracle.OracleStrTable(11)
    a.insert(pool)
    b = oracle.OracleStrTable(11)
    b.insert([pool[i] for i in rng.permutation(len(pool))])
    occ = lambda t: [x is not None for x in t.cells()]
    assert occ(a) == occ(b)
    a.grow(12)
    c = oracle.OracleStrTable(12)
    c.insert(pool[::-1])
    assert occ(a) == occ(c)
    assert _check_invariants(a) == set(pool)
