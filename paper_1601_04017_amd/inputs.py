"""Seeded synthetic workload generators.

This module only draws inputs.  It holds none of the hash table's arithmetic
(no hashing, no positions, no probing) and is shared, as a pure input source,
by the device path's tests and benchmark and by the CPU oracle's tests.

Workload shapes follow the paper's methodology (Sec. 8.3): precomputed
uniformly random keys, and Zipf-distributed keys with P(k) = 1/(k^s H_{N,s})
over the universe 1..N.

* Distinct uniform keys come from a seeded counter-based generator: the
  SplitMix64 output function (a bijection of the 64-bit integers) applied to
  disjoint counter ranges, so keys are distinct by construction and keys
  meant to be absent are guaranteed absent.  32-bit keys use the MurmurHash3
  32-bit finaliser, also a bijection.  Reserved keys 0 and 1 are removed.
* Zipf ranks use the rejection-inversion sampler of Hoermann and Derflinger
  (ACM TOMACS 6(3), 1996), vectorised with numpy; keys are rank + 1 so that
  the most frequent key is not the tombstone key 1.  The control stream maps
  those keys through a seeded Feistel bijection (scramble_keys_u64).
"""
from __future__ import annotations

import math

import numpy as np

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)
_ABSENT_BASE = np.uint64(1 << 62)


def _splitmix64_out(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= np.uint64(0xBF58476D1CE4E5B9)
        z ^= z >> np.uint64(27)
        z *= np.uint64(0x94D049BB133111EB)
        z ^= z >> np.uint64(31)
    return z


def _fmix32(h: np.ndarray) -> np.ndarray:
    h = h.astype(np.uint32, copy=True)
    with np.errstate(over="ignore"):
        h ^= h >> np.uint32(16)
        h *= np.uint32(0x85EBCA6B)
        h ^= h >> np.uint32(13)
        h *= np.uint32(0xC2B2AE35)
        h ^= h >> np.uint32(16)
    return h


def _seed64(seed: int) -> np.uint64:
    # Different seeds give different (but each bijective) streams.
    return _splitmix64_out(np.array([seed * 0x9E3779B97F4A7C15 & 0xFFFFFFFFFFFFFFFF],
                                    dtype=np.uint64))[0]


def _u64_stream(start: int, n: int, seed: int, chunk: int = 1 << 24) -> np.ndarray:
    out = np.empty(n, dtype=np.uint64)
    s = _seed64(seed)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        c = np.arange(start + lo, start + hi, dtype=np.uint64)
        with np.errstate(over="ignore"):
            out[lo:hi] = _splitmix64_out(c ^ s)
    return out


def distinct_keys_u64(n: int, seed: int, absent: bool = False) -> np.ndarray:
    """n distinct uniformly random u64 keys in [2, 2^64).

    Keys drawn with absent=False and absent=True for the same seed never
    coincide (disjoint counter ranges under one bijection)."""
    start = (1 << 62) if absent else 0
    keys = _u64_stream(start, n, seed)
    if np.any(keys < 2):  # probability ~1e-11 at n = 1e8; fail loudly instead
        raise ValueError(f"seed {seed} produced a reserved key; pick another seed")
    return keys


def distinct_keys_u32(n: int, seed: int, absent: bool = False) -> np.ndarray:
    """n distinct uniformly random u32 keys in [2, 2^32); n <= 2^30.

    absent=True draws from a counter range disjoint from absent=False."""
    if n > (1 << 30):
        raise ValueError("at most 2^30 keys per stream")
    s = np.uint32(int(_seed64(seed)) & 0xFFFFFFFF)
    start = (1 << 31) if absent else 0
    c = np.arange(start, start + n + 8, dtype=np.uint32)
    keys = _fmix32(c ^ s)
    keys = keys[keys >= 2][:n]
    assert keys.size == n
    return keys


def permutation(n: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).permutation(n)


def shuffled_mix(present: np.ndarray, absent: np.ndarray, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Concatenate present and absent keys and shuffle; returns (keys, is_present)."""
    keys = np.concatenate([present, absent])
    is_present = np.concatenate([np.ones(present.size, bool), np.zeros(absent.size, bool)])
    p = permutation(keys.size, seed)
    return keys[p], is_present[p]


# --------------------------------------------------------------------------- Zipf


def _helper1(x: np.ndarray) -> np.ndarray:
    # log(1+x)/x with the limit 1 at x = 0
    out = np.ones_like(x)
    nz = np.abs(x) > 1e-8
    out[nz] = np.log1p(x[nz]) / x[nz]
    sm = ~nz
    out[sm] = 1.0 - x[sm] * (0.5 - x[sm] * (1.0 / 3.0 - 0.25 * x[sm]))
    return out


def _helper2(x: np.ndarray) -> np.ndarray:
    # (exp(x)-1)/x with the limit 1 at x = 0
    out = np.ones_like(x)
    nz = np.abs(x) > 1e-8
    out[nz] = np.expm1(x[nz]) / x[nz]
    sm = ~nz
    out[sm] = 1.0 + x[sm] * 0.5 * (1.0 + x[sm] * (1.0 / 3.0) * (1.0 + 0.25 * x[sm]))
    return out


class ZipfSampler:
    """Ranks 1..N with P(k) proportional to k^-s (s > 0), by rejection-inversion."""

    def __init__(self, n_universe: int, s: float):
        if s <= 0 or n_universe < 1:
            raise ValueError("need s > 0 and N >= 1")
        self.N = int(n_universe)
        self.s = float(s)
        one = np.ones(1)
        self.hx1 = float(self._H(1.5 * one)[0]) - 1.0
        self.hN = float(self._H((self.N + 0.5) * one)[0])
        self.skip = 2.0 - float(self._Hinv(self._H(2.5 * one) - self._h(2.0 * one))[0])

    def _H(self, x):
        lx = np.log(x)
        return _helper2((1.0 - self.s) * lx) * lx

    def _Hinv(self, x):
        t = x * (1.0 - self.s)
        t = np.maximum(t, -1.0)
        return np.exp(_helper1(t) * x)

    def _h(self, x):
        return np.exp(-self.s * np.log(x))

    def sample(self, m: int, seed: int, chunk: int = 1 << 23) -> np.ndarray:
        rng = np.random.default_rng(seed)
        out = np.empty(m, dtype=np.int64)
        filled = 0
        while filled < m:
            want = min(chunk, m - filled)
            # draw a little extra to cover rejections
            u = rng.random(int(want * 1.1) + 64)
            u = self.hN + u * (self.hx1 - self.hN)
            x = self._Hinv(u)
            k = np.floor(x + 0.5)
            k = np.clip(k, 1, self.N)
            acc = (k - x <= self.skip) | (u >= self._H(k + 0.5) - self._h(k))
            ks = k[acc].astype(np.int64)[:want]
            out[filled:filled + ks.size] = ks
            filled += ks.size
        return out


def zipf_keys_u64(m: int, n_universe: int, s: float, seed: int) -> np.ndarray:
    """m keys = Zipf(s) rank over 1..N, plus one (so keys lie in 2..N+1)."""
    return (ZipfSampler(n_universe, s).sample(m, seed) + 1).astype(np.uint64)


def _feistel_round_keys(seed: int, rounds: int) -> np.ndarray:
    return _splitmix64_out(np.arange(rounds, dtype=np.uint64) ^ _seed64(seed))


def _feistel64(x: np.ndarray, rk: np.ndarray) -> np.ndarray:
    """A balanced Feistel network on the two 32-bit halves of x: each round
    (L, R) -> (R, L ^ F(R)), F = the low 32 bits of SplitMix64's output
    function of R ^ round key.  A bijection of the 64-bit integers for any
    round function."""
    lo = (x & np.uint64(0xFFFFFFFF)).astype(np.uint64)
    hi = (x >> np.uint64(32)).astype(np.uint64)
    for k in rk:
        f = _splitmix64_out(lo ^ k) & np.uint64(0xFFFFFFFF)
        lo, hi = hi ^ f, lo
    return (hi << np.uint64(32)) | lo


def scramble_keys_u64(keys: np.ndarray, seed: int, rounds: int = 4, chunk: int = 1 << 23) -> np.ndarray:
    """Maps keys through a seeded bijection g of [2, 2^64): a 4-round Feistel
    network, cycle-walked (applied again while the result is 0 or 1) so that
    reserved keys are neither produced nor needed.  Equal keys stay equal and
    distinct keys stay distinct, so a Zipf stream keeps its histogram (up to
    the renaming) while consecutive ranks lose their consecutive values: the
    control for hashes that spread consecutive keys without collisions."""
    keys = np.asarray(keys, dtype=np.uint64)
    if np.any(keys < 2):
        raise ValueError("keys must lie in [2, 2^64)")
    rk = _feistel_round_keys(seed, rounds)
    out = np.empty_like(keys)
    with np.errstate(over="ignore"):
        for lo in range(0, keys.size, chunk):
            y = _feistel64(keys[lo:lo + chunk], rk)
            bad = y < 2
            while np.any(bad):
                y[bad] = _feistel64(y[bad], rk)
                bad = y < 2
            out[lo:lo + chunk] = y
    return out


def zipf_pmf(n_universe: int, s: float, ranks) -> np.ndarray:
    """P(rank) = rank^-s / H_{N,s}; H summed in float64 in chunks."""
    H = 0.0
    for lo in range(1, n_universe + 1, 1 << 24):
        k = np.arange(lo, min(n_universe, lo + (1 << 24) - 1) + 1, dtype=np.float64)
        H += float(np.sum(k ** -s))
    r = np.asarray(ranks, dtype=np.float64)
    return r ** -s / H


def expected_distinct(m: int, n_universe: int, s: float) -> float:
    """E[#distinct ranks] in m Zipf draws = sum_k 1 - (1 - p_k)^m."""
    H = 0.0
    acc = 0.0
    chunks = []
    for lo in range(1, n_universe + 1, 1 << 24):
        k = np.arange(lo, min(n_universe, lo + (1 << 24) - 1) + 1, dtype=np.float64)
        w = k ** -s
        H += float(np.sum(w))
        chunks.append(w)
    for w in chunks:
        p = w / H
        acc += float(np.sum(-np.expm1(m * np.log1p(-p))))
    return acc


def lognormal_sizes(count: int, median: float, sigma: float, lo: int, hi: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    x = np.exp(rng.normal(math.log(median), sigma, size=count))
    return np.clip(np.rint(x), lo, hi).astype(np.int64)


def serving_trace(nreq: int, seed: int = 500, median: int = 16384, lo: int = 1024, hi: int = 1 << 20,
                  ntables: int = 64, e_lo: int = 12, e_hi: int = 26, universe: int = 10 ** 8,
                  zipf_s: float = 1.0):
    """The mixed serving workload: `ntables` tables of 2^e cells, e uniform in
    e_lo..e_hi (seed + 1); each request goes to a uniformly random table
    (seed + 2); request sizes lognormal with the given median and sigma 1.35,
    rounded and clipped to [lo, hi] (seed + 3); operation kinds find /
    insert-or-increment / erase with probabilities 0.6 / 0.3 / 0.1 (seed + 4);
    keys Zipf(zipf_s) ranks over 1..universe, plus one (seed + 5).
    Returns (log2 capacities, [(table, keys u64, kinds u8)], total ops)."""
    caps = [int(e) for e in np.random.default_rng(seed + 1).integers(e_lo, e_hi + 1, size=ntables)]
    tabs = np.random.default_rng(seed + 2).integers(0, ntables, size=nreq)
    sizes = lognormal_sizes(nreq, median, 1.35, lo, hi, seed=seed + 3)
    total = int(sizes.sum())
    kinds = np.random.default_rng(seed + 4).choice(np.array([0, 1, 2], np.uint8), size=total,
                                                   p=[0.6, 0.3, 0.1])
    keys = zipf_keys_u64(total, universe, zipf_s, seed=seed + 5)
    offs = np.concatenate([[0], np.cumsum(sizes)])
    reqs = [(int(tabs[i]), keys[offs[i]:offs[i + 1]], kinds[offs[i]:offs[i + 1]]) for i in range(nreq)]
    return caps, reqs, total
