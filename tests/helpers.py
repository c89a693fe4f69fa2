"""Test-side checks: table invariants, canonical forms and a dictionary model.

These work on raw cell arrays (numpy u64) of either layout, whether they come
from the oracle or from the device, so both are held to the same properties.
"""
from __future__ import annotations

import numpy as np

import oracle

EMPTY = 0
TOMB = 1


def split_cells(cells: np.ndarray, layout: int):
    """-> (keys u64, values u64) per cell."""
    cells = np.asarray(cells, dtype=np.uint64)
    if layout == oracle.PACKED32:
        return cells & np.uint64(0xFFFFFFFF), cells >> np.uint64(32)
    return cells[0::2].copy(), cells[1::2].copy()


def mulshift_hash(keys: np.ndarray, mul: int) -> np.ndarray:
    """(mul * key) mod 2^64 by numpy's wrapping u64 product (the closed form
    of the multiplicative hash, computed without the oracle)."""
    with np.errstate(over="ignore"):
        return np.asarray(keys).astype(np.uint64) * np.uint64(mul)


def homes(keys: np.ndarray, layout: int, log2c: int, seed_hi=oracle.SEED_HI, seed_lo=oracle.SEED_LO,
          mul=None):
    """Home cells: the top log2c bits of the CRC-32C pair hash, or of the
    multiplicative hash when `mul` is given."""
    if mul is not None:
        h = mulshift_hash(keys, mul)
    else:
        kb = 4 if layout == oracle.PACKED32 else 8
        k = keys.astype(np.uint32 if kb == 4 else np.uint64)
        h = oracle.hash_bulk(k, kb, seed_hi, seed_lo)
    return (h >> np.uint64(64 - log2c)).astype(np.int64)


def run_start(occ: np.ndarray) -> np.ndarray:
    """For each cell, the index (unwrapped, may be negative) where the maximal
    cyclic run of non-empty cells containing it starts.  Empty cells get their
    own index.  Requires at least one empty cell."""
    c = occ.size
    assert not occ.all()
    idx = np.arange(c)
    # last empty index at or before i (cyclic); -1 if none before -> wrap
    last_empty = np.where(~occ, idx, -1)
    last_empty = np.maximum.accumulate(last_empty)
    last_empty_global = np.flatnonzero(~occ)[-1]
    le = np.where(last_empty < 0, last_empty_global - c, last_empty)
    return np.where(occ, le + 1, idx)


def check_invariants(cells, layout, log2c, used=None, live=None, seed_hi=oracle.SEED_HI,
                     seed_lo=oracle.SEED_LO, mul=None):
    """U: no live key twice.  R: every live key is reachable from its home
    along non-empty cells.  C: counters match the cells.  V: empty cells hold
    value 0."""
    keys, vals = split_cells(cells, layout)
    c = 1 << log2c
    assert keys.size == c
    occ = keys != EMPTY
    live_mask = occ & (keys != TOMB)
    lk = keys[live_mask]
    assert np.unique(lk).size == lk.size, "U: duplicate live key"
    assert np.all(vals[~occ] == 0), "V: empty cell with nonzero value"
    if used is not None:
        assert int(occ.sum()) == used, "C: used"
    if live is not None:
        assert int(live_mask.sum()) == live, "C: live"
    if occ.all():
        return
    q = np.flatnonzero(live_mask)
    if q.size == 0:
        return
    p = homes(keys[q], layout, log2c, seed_hi, seed_lo, mul)
    rs = run_start(occ)[q]
    # home must lie in [run_start, q] cyclically: distance from home to q
    # (mod c) must not exceed distance from run start to q.
    d_home = (q - p) % c
    d_run = q - rs
    assert np.all(d_home <= d_run), "R: live key not reachable from its home"


def live_dict(cells, layout) -> dict:
    keys, vals = split_cells(cells, layout)
    m = (keys != EMPTY) & (keys != TOMB)
    return dict(zip(keys[m].tolist(), vals[m].tolist()))


def occupancy(cells, layout) -> np.ndarray:
    keys, _ = split_cells(cells, layout)
    return keys != EMPTY


def runs_key_sets(cells, layout):
    """Sorted tuple of (run start, frozenset of live keys) for maximal runs."""
    keys, _ = split_cells(cells, layout)
    occ = keys != EMPTY
    if occ.all():
        return [(0, frozenset(keys[keys != TOMB].tolist()))]
    rs = run_start(occ) % occ.size
    out = {}
    for i in np.flatnonzero(occ & (keys != TOMB)):
        out.setdefault(int(rs[i]), set()).add(int(keys[i]))
    return sorted((k, frozenset(v)) for k, v in out.items())


def canonical_flags(keys: np.ndarray, flags: np.ndarray) -> np.ndarray:
    """Moves each key's single true flag (if any) to its first occurrence.
    Asserts that no key carries more than one true flag."""
    keys = np.asarray(keys)
    flags = np.asarray(flags).astype(np.uint8).copy()
    if keys.size == 0:
        return flags
    truth = flags == 1
    order = np.argsort(keys, kind="stable")
    ks = keys[order]
    ts = truth[order]
    starts = np.flatnonzero(np.r_[True, ks[1:] != ks[:-1]])
    counts = np.add.reduceat(ts.astype(np.int64), starts)
    assert np.all(counts <= 1), "a key has more than one true flag"
    out = flags.copy()
    out[truth] = 0
    first_idx = order[starts]
    has = counts == 1
    out[first_idx[has]] = 1
    return out


class DictModel:
    """Sequential semantics of the bounded table, without cells: a dict of
    live keys, a count of used cells, and the capacity.  An insertion of an
    absent key fails with 'full' exactly when no empty cell is left."""

    def __init__(self, cap: int, value_mask: int):
        self.cap = cap
        self.d = {}
        self.used = 0
        self.mask = value_mask

    def insert(self, k, v):
        if k in (EMPTY, TOMB):
            return oracle.FLAG_RESERVED
        if k in self.d:
            return 0
        if self.used == self.cap:
            return oracle.FLAG_FULL
        self.d[k] = v & self.mask
        self.used += 1
        return 1

    def upsert(self, k, v, op):
        if k in (EMPTY, TOMB):
            return oracle.FLAG_RESERVED
        if k in self.d:
            self.d[k] = ((self.d[k] + v) if op == oracle.ADD else v) & self.mask
            return 0
        if self.used == self.cap:
            return oracle.FLAG_FULL
        self.d[k] = v & self.mask
        self.used += 1
        return 1

    def update(self, k, v, op):
        if k in (EMPTY, TOMB):
            return oracle.FLAG_RESERVED
        if k in self.d:
            self.d[k] = ((self.d[k] + v) if op == oracle.ADD else v) & self.mask
            return 1
        return 0

    def find(self, k):
        if k in (EMPTY, TOMB):
            return oracle.FLAG_RESERVED, 0
        if k in self.d:
            return 1, self.d[k]
        return 0, 0

    def erase(self, k):
        if k in (EMPTY, TOMB):
            return oracle.FLAG_RESERVED
        if k in self.d:
            del self.d[k]
            return 1
        return 0


def key_run_starts(cells, layout):
    """Live keys sorted, with the start index of the maximal non-empty run
    holding each one and its value.  Two tables with equal occupancy and equal
    outputs here hold the same keys in the same runs."""
    keys, vals = split_cells(cells, layout)
    occ = keys != EMPTY
    live = occ & (keys != TOMB)
    rs = run_start(occ) % occ.size if not occ.all() else np.zeros(occ.size, np.int64)
    k = keys[live]
    o = np.argsort(k, kind="stable")
    return k[o], rs[live][o], vals[live][o]


def assert_same_table_modulo_run_order(cells_a, cells_b, layout):
    """Equal occupancy bitmaps, and every live key in the same run with the
    same value.  Within a run the order of keys may differ (it depends on the
    order in which concurrent insertions were linearized)."""
    oa, ob = occupancy(cells_a, layout), occupancy(cells_b, layout)
    assert oa.size == ob.size
    if not np.array_equal(oa, ob):
        bad = np.flatnonzero(oa != ob)
        raise AssertionError(f"occupancy differs at {bad.size} cells, first {bad[:8]}")
    ka, ra, va = key_run_starts(cells_a, layout)
    kb, rb, vb = key_run_starts(cells_b, layout)
    assert np.array_equal(ka, kb), "live key sets differ"
    assert np.array_equal(ra, rb), "a key sits in a different run"
    assert np.array_equal(va, vb), "values differ"
