"""Insertion that grows the table inside the kernel (Sec. 5.3.2, the
synchronized protocol, with the approximate counter of Sec. 5.2).  The
capacity at the end depends on when the approximate count crossed alpha * c,
so the checks are: the contents against a dictionary model, exact counts,
flags, the capacity between the bounds the counter allows, and the occupied
cells and each cluster's keys against the oracle inserting the same keys into
a table of the final capacity (the occupancy of linear probing does not
depend on the order of insertion)."""
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


def _oracle_same_cells(t, layout, live):
    """The device table holds `live` ({key: value}) and occupies what
    inserting those keys into an empty table of its capacity occupies."""
    g = cells_host(t)
    assert H.live_dict(g, layout) == live
    ref = oracle.OracleTable(layout, t.log2_capacity)
    ks = np.array(list(live.keys()), dtype=keys_dtype(layout))
    ref.insert(ks)
    assert np.array_equal(H.occupancy(g, layout), H.occupancy(ref.cells(), layout))
    assert H.runs_key_sets(g, layout) == H.runs_key_sets(ref.cells(), layout)
    H.check_invariants(g, layout, t.log2_capacity, len(live), len(live))


@pytest.mark.parametrize("layout", LAYOUTS)
def test_distinct_inserts_grow_inside_the_kernel(layout):
    n = 3_000_000
    keys = _keys(layout, n, 5)
    vals = (np.arange(n) * 3 + 1).astype(keys_dtype(layout))
    t = make_table(layout, 12, auto_grow=True)
    f = to_host(t.insert_async(to_dev(keys), to_dev(vals)))
    assert (f == 1).all()
    assert t.count() == (n, n)
    st = t.stats()
    assert st["async_growths"] >= 1
    # the counter never exceeds the true count, so the table is never larger
    # than the smallest capacity c with n <= alpha * c
    c = t.capacity
    assert n <= c and c <= 1 << 23
    _oracle_same_cells(t, layout, dict(zip(keys.tolist(), vals.tolist())))
    assert t.status() == 0


@pytest.mark.parametrize("layout", LAYOUTS)
def test_zipf_insert_or_add_sizes_by_distinct_keys(layout):
    z = inputs.zipf_keys_u64(4_000_000, 3_000_000, 1.0, seed=81).astype(keys_dtype(layout))
    t = make_table(layout, 12, auto_grow=True)
    f = to_host(t.insert_async(to_dev(z), None, add=True))
    u, cnt = np.unique(z, return_counts=True)
    assert t.count() == (u.size, u.size)
    # exactly one insertion per distinct key
    assert np.array_equal(H.canonical_flags(z, f), np.isin(np.arange(z.size), np.unique(z, return_index=True)[1]).astype(np.uint8))
    # sized by the distinct keys, far below pre-growth by the batch length
    assert t.capacity < 1 << 24
    _oracle_same_cells(t, layout, dict(zip(u.tolist(), cnt.tolist())))


@pytest.mark.parametrize("layout", LAYOUTS)
def test_duplicates_existing_contents_and_reserved_keys(layout):
    from paper_1601_04017_amd import lpht
    t = make_table(layout, 12, auto_grow=True)
    pre = _keys(layout, 200_000, 9)
    t.insert(to_dev(pre), to_dev(pre))
    t.erase(to_dev(pre[::4]))
    new = _keys(layout, 2_500_000, 10)
    batch = np.concatenate([new, new[::3], pre[:50_000], np.array([0, 1], dtype=keys_dtype(layout))])
    batch = batch[inputs.permutation(batch.size, 11)]
    vals = (np.arange(batch.size) + 7).astype(keys_dtype(layout))
    f = to_host(t.insert_async(to_dev(batch), to_dev(vals)))
    assert np.array_equal(f[batch <= 1], np.full(2, 0xFE, dtype=np.uint8))
    ok = batch > 1
    b, fv = batch[ok], f[ok]
    # one true flag per key that was not live before the call
    live_before = set(pre.tolist()) - set(pre[::4].tolist())
    first = np.zeros(b.size, dtype=bool)
    first[np.unique(b, return_index=True)[1]] = True
    want = first & ~np.isin(b, np.array(sorted(live_before), dtype=b.dtype))
    assert np.array_equal(H.canonical_flags(b, fv), want.astype(np.uint8))
    live = H.live_dict(cells_host(t), layout)
    assert set(live) == live_before | set(b.tolist())
    # keys present before keep their value; a new key holds the value of the
    # operation whose flag is true
    for k in list(live_before)[:2000]:
        assert live[k] == k
    won = {int(k): int(v) for k, v, fl in zip(b, vals[ok], fv) if fl == 1}
    assert all(live[k] == v for k, v in won.items())
    assert t.count() == (len(live), len(live))
    assert t.status() == lpht.ERR_RESERVED_KEY
    _oracle_same_cells(t, layout, live)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_growths_use_the_block_migration(layout):
    # ordinary growths inside the kernel move clusters block by block (no
    # fallback), and the result is the oracle's
    n = 2_000_000
    keys = _keys(layout, n, 21)
    vals = (np.arange(n) + 5).astype(keys_dtype(layout))
    t = make_table(layout, 12, auto_grow=True)
    t.insert_async(to_dev(keys), to_dev(vals), flags=False)
    st = t.stats()
    assert st["async_growths"] >= 1 and st["async_fallbacks"] == 0
    _oracle_same_cells(t, layout, dict(zip(keys.tolist(), vals.tolist())))


@pytest.mark.parametrize("layout", LAYOUTS)
def test_cluster_longer_than_halo_takes_the_fallback(layout):
    # 300 keys whose homes in a 2^22-cell table lie in 256 cells form a
    # cluster far longer than the block migration's 128-cell halo (it stays
    # that long at 2^21 and 2^23 cells: positions nest); the growths that see
    # it re-insert by compare-and-swap, and the contents still match
    import oracle as O
    kb = 4 if layout == oracle.PACKED32 else 8
    cand = np.arange(2, 6_000_002, dtype=np.uint64)
    hm = (O.hash_bulk(cand.astype(keys_dtype(layout)), kb) >> np.uint64(64 - 22)).astype(np.int64)
    crowd = cand[(hm >= 70_000) & (hm < 70_256)][:300].astype(keys_dtype(layout))
    assert crowd.size == 300  # 6e6 candidates give about 366
    rest = _keys(layout, 1_200_000, 23)
    rest = rest[~np.isin(rest, crowd)]
    keys = np.concatenate([crowd, rest])
    keys = keys[inputs.permutation(keys.size, 24)]
    vals = (np.arange(keys.size) * 3 + 1).astype(keys_dtype(layout))
    t = make_table(layout, 12, auto_grow=True)
    t.insert_async(to_dev(keys), to_dev(vals), flags=False)
    st = t.stats()
    assert st["async_growths"] >= 1 and st["async_fallbacks"] >= 1
    _oracle_same_cells(t, layout, dict(zip(keys.tolist(), vals.tolist())))
