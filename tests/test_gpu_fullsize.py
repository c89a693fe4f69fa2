"""The headline workload at full size, in the launch shape the benchmark
times (the autotuner's shape for 2^28 KV64 cells), on the benchmark's own
seeded inputs: 10^8 distinct keys inserted into a presized 2^28-cell table
(and the fills 0.25, 0.5, 0.75), as many successful and unsuccessful finds,
10^8 keys inserted in batches into a table growing from 4096 cells, and
10^8 Zipf insert-or-increments over a universe of 10^8, presized and growing.

Replaying 10^8 operations through the oracle does not fit a test, so these
checks are exact properties that hold at any size:
  * distinct keys: every insert reports 1 and the counts equal the keys;
    every key is found with its value (its index), every absent key is not;
    empty cells hold value 0; and for a sample of the stored keys, the key is
    reachable from its home (the oracle's hash) along non-empty cells;
  * Zipf: the final value of every distinct key equals its count in the
    stream (sort + unique + count), and nothing else is stored.
"""
import numpy as np
import pytest

import oracle
from paper_1601_04017_amd import inputs
from tests import helpers as H
from tests.gpu_util import cells_host, to_dev, to_host

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

N = 10 ** 8
LOG2C = 28


@pytest.fixture(scope="module")
def tuned():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1601_04017_amd import lpht
    shape, _ = lpht.autotune(lpht.KV64, LOG2C, reps=2)
    return shape


def _table(shape):
    from paper_1601_04017_amd import lpht
    t = lpht.Table(layout=lpht.KV64, log2_capacity=LOG2C)
    t.apply_tuning(shape)
    return t


def _distinct_inserts_and_finds(shape, n, sample_every):
    import torch
    print(f"full size: {n} distinct keys into 2^{LOG2C} cells, shape {shape}", flush=True)
    keys = inputs.distinct_keys_u64(n, 201)
    dk = to_dev(keys)
    dv = torch.arange(n, dtype=torch.int64, device="cuda")
    t = _table(shape)
    f = t.insert(dk, dv)
    assert int((f == 1).sum()) == n
    assert t.count() == (n, n) and t.status() == 0
    perm = torch.from_numpy(inputs.permutation(n, 203)).cuda()
    v, found = t.find(dk[perm])
    assert bool((found == 1).all())
    assert torch.equal(v, perm)
    del v, found, dv
    miss = to_dev(inputs.distinct_keys_u64(n, 201, absent=True))
    v, found = t.find(miss)
    assert not bool(found.any()) and not bool(v.any())
    del v, found, miss, dk, perm
    cells = cells_host(t)
    t.close()
    ks, vs = H.split_cells(cells, oracle.KV64)
    del cells
    occ = ks != H.EMPTY
    assert int(occ.sum()) == n
    assert not vs[~occ].any(), "empty cell with a nonzero value"
    # reachability for a sample of the stored keys: its home lies in the run
    # of non-empty cells that ends at its cell
    q = np.flatnonzero(occ)[::sample_every]
    p = H.homes(ks[q], oracle.KV64, LOG2C)
    rs = H.run_start(occ)[q]
    assert np.all((q - p) % (1 << LOG2C) <= q - rs), "stored key not reachable from its home"
    # the sampled keys are the inserted keys at the stored indices
    assert np.array_equal(ks[q], keys[vs[q].astype(np.int64)])


def test_distinct_inserts_and_finds_full_size(tuned):
    _distinct_inserts_and_finds(tuned, N, 5)


@pytest.mark.parametrize("fill", [0.25, 0.5, 0.75])
def test_fill_sweep_full_size(tuned, fill):
    # the same at the swept fills of the 2^28-cell table; at 0.75 the insert
    # is split where a fill quarter changes the group width
    _distinct_inserts_and_finds(tuned, int(fill * (1 << LOG2C)), 20)


def test_zipf_increments_full_size(tuned):
    from paper_1601_04017_amd import lpht
    z = inputs.zipf_keys_u64(N, N, 1.0, seed=402)
    uk, cnt = np.unique(z, return_counts=True)
    print(f"full size: {N} Zipf(1.0) increments, {uk.size} distinct keys", flush=True)
    t = _table(tuned)
    t.insert_or_update(to_dev(z), None, op=lpht.ADD, flags=False)
    del z
    assert t.count() == (uk.size, uk.size) and t.status() == 0
    v, found = t.find(to_dev(uk))
    assert bool((found == 1).all())
    assert np.array_equal(to_host(v, np.uint64), cnt.astype(np.uint64))
    t.close()


def test_growing_from_4096_full_size(tuned):
    # 10^8 distinct keys in batches of 2^20 into a table created with 4096
    # cells (alpha = 1/2): after every batch the capacity is the smallest
    # power of two >= 4096 that holds the keys so far at fill <= 1/2 (the
    # oracle's growth rule for distinct keys, checked against it on small
    # runs), and at the end every key is found with its value
    import torch
    from paper_1601_04017_amd import lpht
    b = 1 << 20
    print(f"full size: {N} distinct keys from 4096 cells in batches of {b}", flush=True)
    dk = to_dev(inputs.distinct_keys_u64(N, 201))
    dv = torch.arange(N, dtype=torch.int64, device="cuda")
    t = lpht.Table(layout=lpht.KV64, log2_capacity=12, auto_grow=True)
    t.apply_tuning(tuned)
    for lo in range(0, N, b):
        hi = min(N, lo + b)
        t.insert(dk[lo:hi], dv[lo:hi], flags=False)
        assert t.log2_capacity == max(12, (2 * hi - 1).bit_length()), hi
    assert t.count() == (N, N) and t.status() == 0
    perm = torch.from_numpy(inputs.permutation(N, 203)).cuda()
    v, found = t.find(dk[perm])
    assert bool((found == 1).all()) and torch.equal(v, perm)
    t.close()


@pytest.mark.parametrize("s", [0.5, 1.0, 1.25, 1.5])
def test_zipf_presized_and_growing_full_size(tuned, s):
    # the suite's Zipf streams: 10^8 keys from a universe of 10^8, counted
    # into a presized 2^28-cell table in one call and into a table growing
    # from 4096 cells in batches of 2^20; both must hold the exact histogram
    from paper_1601_04017_amd import lpht
    z = inputs.zipf_keys_u64(N, N, s, seed=400 + int(s * 4))
    uk, cnt = np.unique(z, return_counts=True)
    print(f"full size: Zipf({s}) increments, {uk.size} distinct keys", flush=True)
    dz, du = to_dev(z), to_dev(uk)
    del z
    for grow in (False, True):
        if grow:
            t = lpht.Table(layout=lpht.KV64, log2_capacity=12, auto_grow=True)
            t.apply_tuning(tuned)
            for lo in range(0, N, 1 << 20):
                t.insert_or_update(dz[lo:lo + (1 << 20)], None, op=lpht.ADD, flags=False)
        else:
            t = _table(tuned)
            t.insert_or_update(dz, None, op=lpht.ADD, flags=False)
        assert t.count() == (uk.size, uk.size) and t.status() == 0, grow
        v, found = t.find(du)
        assert bool((found == 1).all()), grow
        assert np.array_equal(to_host(v, np.uint64), cnt.astype(np.uint64)), grow
        t.close()


def test_zipf_scrambled_keys_full_size(tuned):
    # the control stream of the benchmark: the Zipf(1.0) keys renamed by the
    # seeded Feistel bijection, so the CRC pair no longer spreads consecutive
    # ranks over distinct cells; the presized table (and one growing from
    # 4096 cells in batches of 2^20) must hold the exact histogram, and every
    # stored key must be reachable from its home along non-empty cells
    from paper_1601_04017_amd import lpht
    z = inputs.scramble_keys_u64(inputs.zipf_keys_u64(N, N, 1.0, seed=402), 409)
    uk, cnt = np.unique(z, return_counts=True)
    print(f"full size: scrambled Zipf(1.0) increments, {uk.size} distinct keys", flush=True)
    dz, du = to_dev(z), to_dev(uk)
    del z
    for grow in (False, True):
        if grow:
            t = lpht.Table(layout=lpht.KV64, log2_capacity=12, auto_grow=True)
            t.apply_tuning(tuned)
            for lo in range(0, N, 1 << 20):
                t.insert_or_update(dz[lo:lo + (1 << 20)], None, op=lpht.ADD, flags=False)
        else:
            t = _table(tuned)
            t.insert_or_update(dz, None, op=lpht.ADD, flags=False)
        assert t.count() == (uk.size, uk.size) and t.status() == 0, grow
        v, found = t.find(du)
        assert bool((found == 1).all()), grow
        assert np.array_equal(to_host(v, np.uint64), cnt.astype(np.uint64)), grow
        if not grow:
            # reachability of every tenth stored key from its home
            ks, _ = H.split_cells(cells_host(t), oracle.KV64)
            occ = ks != H.EMPTY
            q = np.flatnonzero(occ)[::10]
            p = H.homes(ks[q], oracle.KV64, LOG2C)
            rs = H.run_start(occ)[q]
            assert np.all((q - p) % (1 << LOG2C) <= q - rs), "stored key not reachable from its home"
            del ks, occ
        t.close()
