"""Shrinking migration (Sec. 5.3.1, "Shrinking") and the cleanup rule that
uses it (Sec. 5.4): the GPU's two-phase shrink places keys in a different
order inside clusters than the oracle's sequential migration, so tables are
compared by occupancy, each live key's cluster and value, and the counts."""
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


def _keys(layout, n, seed):
    if layout == oracle.PACKED32:
        return inputs.distinct_keys_u32(n, seed)
    return inputs.distinct_keys_u64(n, seed)


def _keys_with_home(layout, log2c, home, count, start=2):
    kb = 4 if layout == oracle.PACKED32 else 8
    out, lo = [], start
    while len(out) < count:
        cand = np.arange(lo, lo + 2_000_000, dtype=np.uint64)
        hm = (oracle.hash_bulk(cand, kb) >> np.uint64(64 - log2c)).astype(np.int64)
        out.extend(cand[hm == home].tolist())
        lo += 2_000_000
    return np.array(out[:count], dtype=keys_dtype(layout))


def _old_table(layout, log2_old, log2_new, new_fill, erase_frac, seed):
    """An oracle table of 2^log2_old cells whose live keys fill 2^log2_new
    cells to `new_fill`, with tombstones, and keys whose new home is the last
    cell of the smaller table (their cluster wraps around)."""
    live = int(new_fill * (1 << log2_new))
    n = int(live / (1 - erase_frac)) if erase_frac else live
    wrap = _keys_with_home(layout, log2_new, (1 << log2_new) - 1, 12, start=2 + seed * 7_000_000)
    keys = np.unique(np.concatenate([wrap, _keys(layout, n, seed)]))
    keys = keys[inputs.permutation(keys.size, seed)]
    orc = oracle.OracleTable(layout, log2_old)
    orc.insert(keys, (np.arange(keys.size) * 5 + 3).astype(keys_dtype(layout)))
    if erase_frac:
        rng = np.random.default_rng(seed)
        drop = keys[12:][rng.random(keys.size - 12) < erase_frac]
        orc.erase(drop)
    return orc


# (log2_old, log2_new): below 2^19 target cells every element is inserted
# concurrently; from 2^19 on the two-phase path runs
CASES = [(10, 9), (12, 8), (16, 13), (18, 17), (20, 19), (21, 19), (22, 20), (24, 19)]


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("log2_old,log2_new", CASES)
@pytest.mark.parametrize("new_fill,erase_frac", [(0.3, 0.0), (0.6, 0.4), (0.93, 0.1)])
def test_shrink_matches_oracle_modulo_run_order(layout, log2_old, log2_new, new_fill, erase_frac):
    orc = _old_table(layout, log2_old, log2_new, new_fill, erase_frac, seed=log2_old * 3 + log2_new)
    old = orc.cells()
    t = make_table(layout, log2_old)
    t.import_cells(to_dev(old), log2_old)
    assert t.count() == orc.counts()
    t.grow(log2_new)
    orc.grow(log2_new)
    assert t.capacity == orc.capacity == 1 << log2_new
    g = cells_host(t)
    H.assert_same_table_modulo_run_order(g, orc.cells(), layout)
    assert t.count() == orc.counts()
    H.check_invariants(g, layout, log2_new, *orc.counts())
    assert t.status() == 0
    assert t.stats()["shrinks"] == 1
    # the shrunk table answers finds like the oracle
    live_keys = np.array(sorted(H.live_dict(old, layout)), dtype=keys_dtype(layout))
    probe = np.concatenate([live_keys[::3], _keys(layout, 500, 999)])
    gv, gf = t.find(to_dev(probe))
    ov, of = orc.find(probe)
    assert np.array_equal(to_host(gf), of)
    assert np.array_equal(to_host(gv, keys_dtype(layout)), ov)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_shrink_without_room_is_refused(layout):
    t = make_table(layout, 10)
    keys = _keys(layout, 300, 4)
    t.insert(to_dev(keys))
    before = cells_host(t)
    from paper_1601_04017_amd import lpht
    with pytest.raises(lpht.LphtError):
        t.grow(8)  # 256 cells cannot hold 300 keys and an empty cell
    assert t.capacity == 1 << 10 and t.count() == (300, 300)
    assert np.array_equal(cells_host(t), before)
    with pytest.raises(lpht.LphtError):
        t.grow(5)  # below the smallest capacity


@pytest.mark.parametrize("layout", LAYOUTS)
def test_cleanup_shrinks_to_hand_computed_capacity(layout):
    # the oracle pin's scenario: 2^6 -> 2^16 by inserts, erase all but 10,
    # 3000 inserts trigger a cleanup that shrinks to 2^14
    keys = _keys(layout, 33000, 6)
    t = make_table(layout, 6, auto_grow=True)
    t.insert(to_dev(keys[:30000]))
    assert t.capacity == 1 << 16
    t.erase(to_dev(keys[10:30000]))
    t.insert(to_dev(keys[30000:]))
    assert t.capacity == 1 << 14
    assert t.count() == (3010, 3010)
    assert t.stats()["shrinks"] == 1
    live = H.live_dict(cells_host(t), layout)
    assert sorted(live) == sorted(np.concatenate([keys[:10], keys[30000:]]).tolist())


@pytest.mark.parametrize("layout", LAYOUTS)
def test_auto_grow_erase_heavy_batches_match_oracle(layout):
    # grow to 2^22 cells, erase 90 %, then batches that insert and erase:
    # cleanups shrink (two-phase path at 2^21) exactly when the oracle does
    n = 1 << 21
    keys = _keys(layout, n + 6 * (1 << 16), 77)
    vals = (np.arange(keys.size) + 11).astype(keys_dtype(layout))
    t = make_table(layout, 12, auto_grow=True)
    orc = oracle.OracleTable(layout, 12, auto_grow=True)
    for lo in range(0, n, 1 << 18):
        sl = slice(lo, lo + (1 << 18))
        assert np.array_equal(to_host(t.insert(to_dev(keys[sl]), to_dev(vals[sl]))), orc.insert(keys[sl], vals[sl]))
    assert t.capacity == orc.capacity == 1 << 22
    rng = np.random.default_rng(3)
    ek = keys[:n][rng.random(n) < 0.9]
    assert np.array_equal(to_host(t.erase(to_dev(ek))), orc.erase(ek))
    caps = []
    for r in range(6):
        sl = slice(n + r * (1 << 16), n + (r + 1) * (1 << 16))
        assert np.array_equal(to_host(t.insert(to_dev(keys[sl]), to_dev(vals[sl]))), orc.insert(keys[sl], vals[sl]))
        ek = keys[sl][::3]
        assert np.array_equal(to_host(t.erase(to_dev(ek))), orc.erase(ek))
        assert t.capacity == orc.capacity
        assert t.count() == orc.counts()
        caps.append(t.capacity)
    assert min(caps) < 1 << 22  # the rule shrank the table
    assert t.stats()["shrinks"] >= 1
    H.assert_same_table_modulo_run_order(cells_host(t), orc.cells(), layout)
