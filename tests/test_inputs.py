"""Checks of the seeded workload generators (Sec. 8.3: precomputed uniform keys;
Zipf keys with P(k) = 1/(k^s H_{N,s}) over 1..N)."""
import numpy as np
import pytest

from paper_1601_04017_amd import inputs


def test_u64_keys_distinct_reproducible_and_disjoint():
    a = inputs.distinct_keys_u64(200_000, 201)
    b = inputs.distinct_keys_u64(200_000, 201)
    c = inputs.distinct_keys_u64(200_000, 201, absent=True)
    assert np.array_equal(a, b)
    assert np.unique(a).size == a.size
    assert np.intersect1d(a, c).size == 0
    assert a.min() >= 2 and c.min() >= 2
    # roughly uniform: each top-4-bit bucket holds about 1/16
    top = (a >> np.uint64(60)).astype(np.int64)
    frac = np.bincount(top, minlength=16) / a.size
    assert np.all(np.abs(frac - 1 / 16) < 0.005)


def test_u32_keys_distinct_and_disjoint():
    a = inputs.distinct_keys_u32(1 << 20, 101)
    c = inputs.distinct_keys_u32(1 << 19, 101, absent=True)
    assert a.dtype == np.uint32 and np.unique(a).size == a.size
    assert np.intersect1d(a, c).size == 0
    assert a.min() >= 2


@pytest.mark.parametrize("s", [0.5, 1.0, 1.25, 1.5])
def test_zipf_frequencies_match_pmf(s):
    N, m = 100_000, 2_000_000
    r = inputs.ZipfSampler(N, s).sample(m, seed=400 + int(s * 4))
    assert r.min() >= 1 and r.max() <= N
    cnt = np.bincount(r, minlength=N + 1)
    p = inputs.zipf_pmf(N, s, np.arange(1, 6))
    for k in range(1, 6):
        se = np.sqrt(p[k - 1] * (1 - p[k - 1]) / m)
        assert abs(cnt[k] / m - p[k - 1]) < 6 * se + 1e-6, (k, cnt[k] / m, p[k - 1])
    # tail mass beyond rank 1000
    pt = 1.0 - inputs.zipf_pmf(N, s, np.arange(1, 1001)).sum()
    got = cnt[1001:].sum() / m
    assert abs(got - pt) < 6 * np.sqrt(pt * (1 - pt) / m) + 1e-6


def test_zipf_distinct_count_matches_expectation():
    N, m, s = 200_000, 1_000_000, 1.0
    r = inputs.ZipfSampler(N, s).sample(m, seed=7)
    d = np.unique(r).size
    e = inputs.expected_distinct(m, N, s)
    assert abs(d - e) / e < 0.01


def test_zipf_top_probability_at_paper_universe():
    # N = 10^8 (Sec. 8.3): P(rank 1) for the four exponents of the aggregation runs
    exp = {0.5: 5.0e-5, 1.0: 0.0526, 1.25: 0.2195, 1.5: 0.3828}
    for s, p1 in exp.items():
        got = float(inputs.zipf_pmf(10 ** 8, s, [1])[0])
        assert abs(got - p1) / p1 < 0.01, (s, got)


def test_lognormal_sizes_clip():
    x = inputs.lognormal_sizes(10000, 16384, 1.35, 1024, 1 << 20, seed=503)
    assert x.min() >= 1024 and x.max() <= 1 << 20
    assert 12000 < np.median(x) < 21000


def test_scrambled_zipf_keeps_histogram_and_breaks_consecutive_spread():
    z = inputs.zipf_keys_u64(500_000, 10 ** 6, 1.0, seed=402)
    s1 = inputs.scramble_keys_u64(z, 7)
    s2 = inputs.scramble_keys_u64(z, 7)
    assert np.array_equal(s1, s2)
    assert s1.min() >= 2
    # a bijection: equal keys stay equal, distinct stay distinct, so the
    # multiset of counts is unchanged and first occurrences stay in place
    uz, iz, cz = np.unique(z, return_index=True, return_counts=True)
    us, is_, cs = np.unique(s1, return_index=True, return_counts=True)
    assert uz.size == us.size
    assert np.array_equal(np.sort(iz), np.sort(is_))
    assert np.array_equal(np.sort(cz), np.sort(cs))
    # another seed gives another bijection
    assert not np.array_equal(inputs.scramble_keys_u64(z[:1000], 8), s1[:1000])


def test_scramble_is_injective_and_avoids_reserved_keys():
    x = np.arange(2, 2 + (1 << 20), dtype=np.uint64)
    y = inputs.scramble_keys_u64(x, 11)
    assert np.unique(y).size == x.size and y.min() >= 2
    # cycle walking: inputs the network maps to 0 or 1 still land in [2, 2^64)
    rk = inputs._feistel_round_keys(11, 4)
    pre = []
    for target in (0, 1):
        # the inverse network gives the preimage of a reserved value
        lo, hi = np.uint64(target & 0xFFFFFFFF), np.uint64(target >> 32)
        for k in rk[::-1]:
            with np.errstate(over="ignore"):
                f = inputs._splitmix64_out(np.array([hi ^ k], np.uint64))[0] & np.uint64(0xFFFFFFFF)
            lo, hi = hi, lo ^ f
        pre.append((int(hi) << 32) | int(lo))
    p = np.array([v for v in pre if v >= 2], dtype=np.uint64)
    if p.size:
        q = inputs.scramble_keys_u64(p, 11)
        assert q.min() >= 2


def test_scrambled_consecutive_keys_collide_like_random_keys():
    import oracle
    from tests import helpers as H
    keys = np.arange(2, 2 + (1 << 16), dtype=np.uint64)
    c = 1 << 18
    plain = np.unique(H.homes(keys, oracle.KV64, 18)).size
    scr = np.unique(H.homes(inputs.scramble_keys_u64(keys, 3), oracle.KV64, 18)).size
    assert plain == keys.size  # the CRC pair spreads consecutive keys without collision
    expect = c * (1 - np.exp(-keys.size / c))  # distinct homes of random keys
    assert abs(scr - expect) < 0.01 * expect
