"""Pins for the oracle's migration (Sec. 5.3.1, Lemma 1; cleanup by migration,
Sec. 5.4) and for its growth rule (trigger at fill alpha, doubling, bulk
pre-growth of Sec. 5.5)."""
import numpy as np
import pytest

import oracle
from paper_1601_04017_amd import inputs
from tests import helpers as H

LAYOUTS = [oracle.PACKED32, oracle.KV64]


def _filled(layout, log2c, fill, erase_frac, seed):
    c = 1 << log2c
    n = int(c * fill)
    if layout == oracle.PACKED32:
        keys = inputs.distinct_keys_u32(n, seed)
    else:
        keys = inputs.distinct_keys_u64(n, seed)
    t = oracle.OracleTable(layout, log2c)
    t.insert(keys, np.arange(n) + 7)
    if erase_frac:
        rng = np.random.default_rng(seed)
        t.erase(keys[rng.random(n) < erase_frac])
    return t


def _clusters(occ):
    """Maximal cyclic runs of non-empty cells as (a, b) with b possibly >= c."""
    c = occ.size
    starts = [i for i in range(c) if occ[i] and not occ[(i - 1) % c]]
    out = []
    for a in starts:
        b = a
        while occ[(b + 1) % c]:
            b += 1
        out.append((a, b))
    return out


def _scan_order(cells, layout):
    """Live (key, value) pairs in the sequential migration's order: old-array
    order starting just after the first empty cell."""
    keys, vals = H.split_cells(cells, layout)
    c = keys.size
    empties = np.flatnonzero(keys == 0)
    e = int(empties[0]) if empties.size else c - 1
    order = (e + 1 + np.arange(c)) % c
    k, v = keys[order], vals[order]
    m = (k != 0) & (k != 1)
    return k[m], v[m]


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("gamma_log", [0, 1, 2])
@pytest.mark.parametrize("fill,erase_frac", [(0.3, 0.0), (0.5, 0.2), (0.75, 0.3), (0.9, 0.0)])
def test_migration_equals_insert_in_scan_order(layout, gamma_log, fill, erase_frac):
    log2c = 12
    t = _filled(layout, log2c, fill, erase_frac, seed=int(fill * 100) + gamma_log)
    old = t.cells()
    used, live = t.counts()
    k, v = _scan_order(old, layout)
    t.grow(log2c + gamma_log)
    new = t.cells()
    # independent construction: fresh table, ordinary inserts in that order
    ref = oracle.OracleTable(layout, log2c + gamma_log)
    ref.insert(k, v)
    assert np.array_equal(new, ref.cells())
    assert t.counts() == (live, live)
    assert H.live_dict(new, layout) == H.live_dict(old, layout)
    H.check_invariants(new, layout, log2c + gamma_log, live, live)


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("gamma_log", [0, 1, 2, 3])
def test_lemma1_cluster_ranges_and_blockwise_equivalence(layout, gamma_log):
    # Lemma 1: the elements of an old cluster a..b land inside
    # [gamma*a, gamma*(b+1)) of the new table whatever the rest of the table
    # holds; hence migrating clusters independently, in any order, gives the
    # sequential placement exactly.
    log2c = 11
    c = 1 << log2c
    g = 1 << gamma_log
    t = _filled(layout, log2c, 0.7, 0.15, seed=77 + gamma_log)
    old = t.cells()
    okeys, ovals = H.split_cells(old, layout)
    occ = okeys != 0
    t.grow(log2c + gamma_log)
    new = t.cells()
    nkeys, _ = H.split_cells(new, layout)
    pos = {int(k): i for i, k in enumerate(nkeys) if k > 1}
    newc = c * g
    clusters = _clusters(occ)
    for a, b in clusters:
        lo, hi = g * a, g * (b + 1)
        for i in range(a, b + 1):
            k = int(okeys[i % c])
            if k <= 1:
                continue
            p = pos[k]
            # cyclic membership in [lo, hi)
            assert (p - lo) % newc < hi - lo, (a, b, p)
    # blockwise re-migration: clusters processed in reverse order, each one
    # by itself, into an empty table of the new size
    ref = oracle.OracleTable(layout, log2c + gamma_log)
    acc = np.zeros_like(new)
    for a, b in reversed(clusters):
        idx = np.arange(a, b + 1) % c
        k, v = okeys[idx], ovals[idx]
        m = k > 1
        one = oracle.OracleTable(layout, log2c + gamma_log)
        one.insert(k[m], v[m])
        part = one.cells()
        if layout == oracle.PACKED32:
            nz = part != 0
        else:
            nz = np.repeat(part[0::2] != 0, 2)
        assert not np.any((acc != 0) & nz), "target ranges of two clusters overlap"
        acc[nz] = part[nz]
    assert np.array_equal(acc, new)
    del ref


@pytest.mark.parametrize("layout", LAYOUTS)
def test_wraparound_cluster_migrates_in_order(layout):
    log2c = 6
    c = 1 << log2c
    # keys whose home is the last cell, so their cluster wraps to cell 0
    kb = 4 if layout == oracle.PACKED32 else 8
    cand = np.arange(2, 200000, dtype=np.uint64)
    h = oracle.hash_bulk(cand, kb)
    hm = (h >> np.uint64(64 - log2c)).astype(np.int64)
    last = cand[hm == c - 1][:4]
    first = cand[hm == 0][:2]
    t = oracle.OracleTable(layout, log2c)
    t.insert(np.concatenate([last, first]), np.arange(6) + 1)
    old = t.cells()
    keys, _ = H.split_cells(old, layout)
    assert keys[c - 1] != 0 and keys[0] != 0  # the cluster wraps
    k, v = _scan_order(old, layout)
    for gl in (0, 1, 2):
        t2 = oracle.OracleTable(layout, log2c)
        t2.load_cells(old, log2c)
        t2.grow(log2c + gl)
        ref = oracle.OracleTable(layout, log2c + gl)
        ref.insert(k, v)
        assert np.array_equal(t2.cells(), ref.cells())
        H.check_invariants(t2.cells(), layout, log2c + gl, 6, 6)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_full_table_migration(layout):
    # No empty cell at all: the scan starts at cell 0.
    log2c = 4
    t = oracle.OracleTable(layout, log2c)
    keys = np.arange(2, 2 + 16)
    assert np.all(t.insert(keys, keys) == 1)
    old = t.cells()
    k, v = _scan_order(old, layout)
    t.grow(log2c + 1)
    ref = oracle.OracleTable(layout, log2c + 1)
    ref.insert(k, v)
    assert np.array_equal(t.cells(), ref.cells())


def _auto(layout, log2c=12):
    return oracle.OracleTable(layout, log2c, auto_grow=True)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_growth_insert_only_final_capacity_closed_form(layout):
    # Insert-only batches from 4096 cells with alpha = 1/2: the capacity ends at
    # the smallest power of two >= max(4096, 2 * n), reached by doublings only.
    n_total, b = 300_000, 1 << 14
    keys = (inputs.distinct_keys_u32(n_total, 3) if layout == oracle.PACKED32
            else inputs.distinct_keys_u64(n_total, 3))
    t = _auto(layout)
    caps = [t.capacity]
    for lo in range(0, n_total, b):
        f = t.insert(keys[lo:lo + b], np.arange(lo, min(n_total, lo + b)))
        assert np.all(f == 1)
        used, live = t.counts()
        assert 2 * used <= t.capacity  # fill never above alpha
        caps.append(t.capacity)
    expect = 1 << max(12, int(np.ceil(np.log2(2 * n_total))))
    assert t.capacity == expect
    assert t.migrations == int(np.log2(expect // 4096))
    assert all(b2 in (a2, 2 * a2, 4 * a2, 8 * a2) or b2 > a2 for a2, b2 in zip(caps, caps[1:]))
    H.check_invariants(t.cells(), layout, t.log2c, n_total, n_total)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_growth_capacity_minimal(layout):
    # Each growth stops at the first doubling that makes room for the batch.
    rng = np.random.default_rng(5)
    t = _auto(layout)
    keys = (inputs.distinct_keys_u32(200_000, 9) if layout == oracle.PACKED32
            else inputs.distinct_keys_u64(200_000, 9))
    lo = 0
    while lo < keys.size:
        b = int(rng.integers(1, 20000))
        used_before, _ = t.counts()
        c_before = t.capacity
        t.insert(keys[lo:lo + b])
        c_after = t.capacity
        bb = min(b, keys.size - lo)
        assert 2 * (used_before + bb) <= c_after
        if c_after > c_before:
            assert 2 * (used_before + bb) > c_after // 2
        lo += b


@pytest.mark.parametrize("layout", LAYOUTS)
def test_tombstone_cleanup_same_size(layout):
    # A table full of tombstones but with few live keys is cleaned with
    # gamma = 1 (same capacity) instead of grown.
    t = _auto(layout, 12)
    keys = (inputs.distinct_keys_u32(2000, 4) if layout == oracle.PACKED32
            else inputs.distinct_keys_u64(2000, 4))
    t.insert(keys)
    t.erase(keys[:1900])
    assert t.counts() == (2000, 100)
    more = (inputs.distinct_keys_u32(200, 4, absent=True) if layout == oracle.PACKED32
            else inputs.distinct_keys_u64(200, 4, absent=True))
    t.insert(more)
    assert t.capacity == 4096
    assert t.migrations == 1
    assert t.counts() == (300, 300)
    H.check_invariants(t.cells(), layout, 12, 300, 300)


def test_zipf_upsert_with_growth_matches_histogram():
    keys = inputs.zipf_keys_u64(400_000, 100_000, 1.0, seed=404)
    t = _auto(oracle.KV64)
    for lo in range(0, keys.size, 1 << 16):
        t.insert_or_update(keys[lo:lo + (1 << 16)], None, oracle.ADD)
    uk, cnt = np.unique(keys, return_counts=True)
    assert H.live_dict(t.cells(), oracle.KV64) == dict(zip(uk.tolist(), cnt.tolist()))
    used, live = t.counts()
    assert used == live == uk.size


@pytest.mark.parametrize("layout", LAYOUTS)
def test_cleanup_shrinks_to_hand_computed_capacity(layout):
    # Created at 2^6 cells, auto-grow, alpha = 1/2.  30000 inserts grow it to
    # 2^16 (30000 <= 32768 = alpha * 2^16, > alpha * 2^15).  Erasing all but 10
    # leaves used = 30000, live = 10.  A batch of b = 3000 inserts triggers a
    # migration (used + b = 33000 > 32768), and live + b = 3010 <= alpha*c/2 =
    # 16384 makes it a cleanup that may shrink: halving 2^16 -> 2^15 needs
    # 3010 <= alpha * 2^16 / 4 = 8192 (yes), 2^15 -> 2^14 needs 3010 <= 4096
    # (yes), 2^14 -> 2^13 needs 3010 <= 2048 (no): one migration to 2^14.
    keys = (inputs.distinct_keys_u32(33000, 6) if layout == oracle.PACKED32
            else inputs.distinct_keys_u64(33000, 6))
    t = oracle.OracleTable(layout, 6, auto_grow=True)
    t.insert(keys[:30000])
    assert t.capacity == 1 << 16
    t.erase(keys[10:30000])
    assert t.counts() == (30000, 10)
    m0 = t.migrations
    t.insert(keys[30000:33000])
    assert t.capacity == 1 << 14
    assert t.migrations == m0 + 1
    assert t.counts() == (3010, 3010)
    H.check_invariants(t.cells(), layout, 14, 3010, 3010)
    live = H.live_dict(t.cells(), layout)
    assert sorted(live) == sorted(np.concatenate([keys[:10], keys[30000:33000]]).tolist())


@pytest.mark.parametrize("layout", LAYOUTS)
def test_cleanup_never_shrinks_below_created_capacity(layout):
    # created at 2^12: however few keys stay live, cleanups keep >= 2^12 cells
    keys = (inputs.distinct_keys_u32(12000, 8) if layout == oracle.PACKED32
            else inputs.distinct_keys_u64(12000, 8))
    t = oracle.OracleTable(layout, 12, auto_grow=True)
    t.insert(keys[:6000])
    t.erase(keys[:5990])
    for lo in range(6000, 12000, 300):
        t.insert(keys[lo:lo + 300])
        t.erase(keys[lo:lo + 290])
        assert t.capacity >= 1 << 12
    assert t.migrations >= 1
    H.check_invariants(t.cells(), layout, t.log2c, *t.counts())


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("shrink", [1, 2, 3])
def test_explicit_shrink_keeps_contents_and_order_free_occupancy(layout, shrink):
    log2c = 12
    t = _filled(layout, log2c, 0.2, 0.5, 60 + shrink)  # about 410 live keys
    live_before = H.live_dict(t.cells(), layout)
    t.grow(log2c - shrink)
    cells = t.cells()
    assert t.capacity == 1 << (log2c - shrink)
    assert H.live_dict(cells, layout) == live_before
    H.check_invariants(cells, layout, log2c - shrink, len(live_before), len(live_before))
    # the occupancy of a linear-probing table does not depend on the order of
    # insertion: the same keys inserted in a random order give the same cells
    ks = np.array(list(live_before.keys()), dtype=np.uint64)
    vs = np.array([live_before[k] for k in ks.tolist()], dtype=np.uint64)
    perm = np.random.default_rng(shrink).permutation(ks.size)
    dt = np.uint32 if layout == oracle.PACKED32 else np.uint64
    ref = oracle.OracleTable(layout, log2c - shrink)
    ref.insert(ks[perm].astype(dt), vs[perm].astype(dt))
    assert np.array_equal(H.occupancy(cells, layout), H.occupancy(ref.cells(), layout))


@pytest.mark.parametrize("layout", LAYOUTS)
def test_shrink_without_room_is_refused(layout):
    t = oracle.OracleTable(layout, 10)
    keys = (inputs.distinct_keys_u32(300, 2) if layout == oracle.PACKED32
            else inputs.distinct_keys_u64(300, 2))
    t.insert(keys)
    with pytest.raises(RuntimeError):
        t.grow(8)  # 256 cells cannot hold 300 keys and an empty cell
    assert t.capacity == 1 << 10 and t.counts() == (300, 300)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_full_table_migrates_at_same_size(layout):
    # a bounded table with every cell live: a gamma = 1 migration keeps it
    # full (the scan starts at cell 0), only a smaller size is refused
    keys = (inputs.distinct_keys_u32(64, 12) if layout == oracle.PACKED32
            else inputs.distinct_keys_u64(64, 12))
    t = oracle.OracleTable(layout, 6)
    t.insert(keys)
    assert t.counts() == (64, 64)
    before = H.live_dict(t.cells(), layout)
    t.grow(6)
    assert t.counts() == (64, 64) and H.live_dict(t.cells(), layout) == before
    with pytest.raises(RuntimeError):
        t.grow(5)


def test_growth_capacity_of_distinct_batches_closed_form():
    # distinct keys in batches from 4096 cells at alpha = 1/2: after each
    # batch the capacity is the smallest power of two >= 4096 with
    # 2 * (keys so far) <= c (the full-size GPU test relies on this form)
    b = 1 << 12
    n = 70 * b + 333
    keys = inputs.distinct_keys_u64(n, 5)
    o = oracle.OracleTable(oracle.KV64, 12, auto_grow=True)
    for lo in range(0, n, b):
        hi = min(n, lo + b)
        o.insert(keys[lo:hi])
        assert o.capacity == 1 << max(12, (2 * hi - 1).bit_length()), hi
