"""String keys (Sec. 5.7) on the GPU against the oracle's string table:
flags, found values and counts per batch, the capacity after every batch
(the same growth rule), and at the end the occupied cells and each
cluster's key set (concurrent insertion orders keys inside clusters
differently)."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"


def _pool(rng, universe, maxlen):
    out = set()
    while len(out) < universe:
        out.add(bytes(rng.integers(0, 256, int(rng.integers(0, maxlen + 1))).astype(np.uint8)))
    return sorted(out)


def _canon(keys, flags):
    f = np.array(flags, dtype=np.uint8).copy()
    seen = {}
    for i, k in enumerate(keys):
        if f[i] == 1:
            f[i] = 0
            seen.setdefault(k, i)
    first = {}
    for i, k in enumerate(keys):
        first.setdefault(k, i)
    for k, i in seen.items():
        f[first[k]] = 1
    return f


def _clusters(cells):
    c = len(cells)
    occ = [x is not None for x in cells]
    if all(occ):
        return [frozenset(x[0] for x in cells if x)]
    start = occ.index(False)
    runs, cur = [], set()
    for q in range(1, c + 1):
        i = (start + q) % c
        if cells[i] is None:
            if cur:
                runs.append(frozenset(cur))
            cur = set()
        elif cells[i]:
            cur.add(cells[i][0])
    return sorted(runs, key=lambda s: sorted(s))


def _same_table(g, o):
    gc, oc = g.cells(), o.cells()
    assert [x is not None for x in gc] == [x is not None for x in oc]
    assert _clusters(gc) == _clusters(oc)
    assert {x[0]: x[1] for x in gc if x} == {x[0]: x[1] for x in oc if x}


@pytest.mark.parametrize("seed,maxlen", [(1, 8), (2, 40), (3, 200)])
def test_operation_sequences_match_oracle(seed, maxlen):
    from paper_1601_04017_amd import lpht
    rng = np.random.default_rng(seed)
    pool = _pool(rng, 3000, maxlen) + [b""]
    g = lpht.StrTable(log2_capacity=8, auto_grow=True, pool_bytes=4096)
    o = oracle.OracleStrTable(8, auto_grow=True)
    for step in range(24):
        n = int(rng.integers(1, 2500))
        keys = [pool[i] for i in rng.integers(0, len(pool), n)]
        kind = step % 4
        vals = rng.integers(0, 1 << 62, n).astype(np.uint64)
        if kind == 0:
            # equal concurrent inserts: one wins, which value is unspecified
            uniq = list(dict.fromkeys(keys))
            vals = vals[: len(uniq)]
            gf = g.insert(uniq, vals)
            of = o.insert(uniq, vals)
            assert np.array_equal(gf, of)
        elif kind == 1:
            gf = g.insert_or_update(keys, vals, oracle.ADD)
            of = o.insert_or_update(keys, vals, oracle.ADD)
            assert np.array_equal(_canon(keys, gf), of)
        elif kind == 2:
            gv, gf = g.find(keys)
            ov, of = o.find(keys)
            assert np.array_equal(gf, of) and np.array_equal(gv, ov)
        else:
            uniq = list(dict.fromkeys(keys))[: n // 2]
            gf = g.erase(uniq)
            of = o.erase(uniq)
            assert np.array_equal(gf, of)
        assert g.count() == o.counts(), step
        assert g.capacity()[0] == o.capacity, step
    assert g.status() == 0
    _same_table(g, o)


def test_signature_collisions_and_pool_compaction():
    from paper_1601_04017_amd import lpht
    # keys whose 16-bit signatures (low hash bits) are equal
    rng = np.random.default_rng(7)
    by_sig = {}
    for i in range(200_000):
        k = b"key-%d" % i
        by_sig.setdefault(oracle.str_hash(k) & 0xFFFF, []).append(k)
    coll = [v for v in by_sig.values() if len(v) >= 3][:50]
    keys = [k for v in coll for k in v]
    g = lpht.StrTable(log2_capacity=10, auto_grow=True, pool_bytes=256)
    o = oracle.OracleStrTable(10, auto_grow=True)
    vals = np.arange(len(keys), dtype=np.uint64) + 1
    assert np.array_equal(g.insert(keys, vals), o.insert(keys, vals))
    gv, gf = g.find(keys + [b"absent"])
    assert gf.tolist() == [1] * len(keys) + [0] and gv[: len(keys)].tolist() == vals.tolist()
    # erase most keys, then insert new ones: the pool is compacted at the next migration
    g.erase(keys[: len(keys) - 20])
    o.erase(keys[: len(keys) - 20])
    big = [bytes(rng.integers(0, 256, 300).astype(np.uint8)) for _ in range(400)]
    assert np.array_equal(g.insert(big), o.insert(big))
    c, pu, pc = g.capacity()
    assert pu <= pc
    assert g.count() == o.counts()
    _same_table(g, o)
    g.grow(g.capacity()[0].bit_length())  # doubling by hand
    o.grow(o.capacity.bit_length())
    _same_table(g, o)


def test_equal_keys_in_one_batch_add_exactly():
    # many lanes of one launch insert the same keys at once: the losers of a
    # race follow the winner's record, written during the same launch
    from paper_1601_04017_amd import lpht
    rng = np.random.default_rng(11)
    pool = _pool(rng, 2000, 60) + [b""]
    ranks = np.minimum(rng.zipf(1.3, 300_000) - 1, len(pool) - 1)
    keys = [pool[i] for i in ranks]
    vals = rng.integers(0, 1 << 40, len(keys)).astype(np.uint64)
    g = lpht.StrTable(log2_capacity=6, auto_grow=True, pool_bytes=64)
    o = oracle.OracleStrTable(6, auto_grow=True)
    gf = g.insert_or_update(keys, vals, oracle.ADD)
    of = o.insert_or_update(keys, vals, oracle.ADD)
    assert np.array_equal(_canon(keys, gf), of)
    assert g.count() == o.counts()
    assert g.capacity()[0] == o.capacity
    gv, gfl = g.find(pool)
    ov, ofl = o.find(pool)
    assert np.array_equal(gfl, ofl) and np.array_equal(gv, ov)
    assert g.status() == 0
    _same_table(g, o)


def test_full_table_without_growth():
    # 100 distinct keys into 64 cells, no growth: which 64 get in is decided
    # by concurrency; exactly the table's capacity is inserted, the rest get
    # 0xFF and the sticky FULL error, and probes of a table with no empty
    # cell end after one round
    from paper_1601_04017_amd import lpht
    rng = np.random.default_rng(13)
    keys = _pool(rng, 100, 30)
    vals = np.arange(1, 101, dtype=np.uint64)
    g = lpht.StrTable(log2_capacity=6, auto_grow=False, pool_bytes=1 << 16)
    f = g.insert(keys, vals)
    assert sorted(set(f.tolist())) == [1, 0xFF] and int((f == 1).sum()) == 64
    assert g.status() == lpht.ERR_FULL and g.status() == 0
    assert g.count() == (64, 64)
    gv, gf = g.find(keys + [b"absent"])
    assert np.array_equal(gf[:100], (f == 1).astype(np.uint8)) and gf[100] == 0
    assert np.array_equal(gv[:100][f == 1], vals[f == 1])
    # erasing makes tombstones, not room: a new key still finds no empty cell
    inside = [k for k, x in zip(keys, f) if x == 1]
    assert g.erase(inside[:10]).tolist() == [1] * 10
    assert g.insert([b"new key"]).tolist() == [0xFF]
    assert g.status() == lpht.ERR_FULL
    assert g.count() == (64, 54)
    # a same-size migration drops the tombstones; then it fits
    g.grow(6)
    assert g.count() == (54, 54)
    assert g.insert([b"new key"]).tolist() == [1]
    _, gf = g.find(inside[10:] + [b"new key"])
    assert gf.tolist() == [1] * 55
