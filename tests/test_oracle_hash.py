"""Pins for the oracle's hash (Sec. 8.3: two CRC-32C with different seeds) and
scaling map (Sec. 5.3.1), checked against published CRC-32C vectors, the host
CPU's SSE4.2 crc32 instruction, and algebraic properties of the CRC."""
import os

import numpy as np
import pytest

import oracle
from tests.native import load_crc_sse42

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "crc32c_vectors.txt")


def _golden_vectors():
    out = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        name, spec, hexv = line.split()
        kind, _, arg = spec.partition(":")
        if kind == "ascii":
            data = arg.encode()
        elif kind == "repeat":
            b, n = arg.split(":")
            data = bytes([int(b, 16)]) * int(n)
        elif kind == "range":
            a, n = map(int, arg.split(":"))
            data = bytes(range(a, a + n))
        elif kind == "rrange":
            a, n = map(int, arg.split(":"))
            data = bytes(range(a, a - n, -1))
        else:
            raise ValueError(kind)
        out.append((name, data, int(hexv, 16)))
    return out


@pytest.mark.parametrize("name,data,expected", _golden_vectors())
def test_crc32c_published_vectors(name, data, expected):
    got = oracle.crc32c_bytes(0xFFFFFFFF, data) ^ 0xFFFFFFFF
    assert got == expected, f"{name}: {got:08X} != {expected:08X}"


def test_crc32c_matches_sse42_instruction_bytes_and_words():
    hw = load_crc_sse42()
    rng = np.random.default_rng(7)
    for _ in range(2000):
        reg = int(rng.integers(0, 1 << 32))
        x = int(rng.integers(0, 1 << 63)) * 2 + int(rng.integers(0, 2))
        assert oracle.crc32c_word(reg, x, 8) == hw.hw_crc_u64(reg, x)
        assert oracle.crc32c_word(reg, x & 0xFFFFFFFF, 4) == hw.hw_crc_u32(reg, x & 0xFFFFFFFF)
        assert oracle.crc32c_bytes(reg, bytes([x & 0xFF])) == hw.hw_crc_u8(reg, x & 0xFF)


@pytest.mark.parametrize("key_bytes", [4, 8])
def test_hash_matches_sse42_on_1e6_keys(key_bytes):
    hw = load_crc_sse42()
    rng = np.random.default_rng(11 + key_bytes)
    dt = np.uint32 if key_bytes == 4 else np.uint64
    keys = rng.integers(0, np.iinfo(dt).max, size=1_000_000, dtype=dt, endpoint=True)
    keys[:4] = [0, 1, 2, np.iinfo(dt).max]
    ref = np.empty(keys.size, dtype=np.uint64)
    hw.hw_hash_bulk(keys.ctypes.data, keys.size, key_bytes, oracle.SEED_HI, oracle.SEED_LO,
                    ref.ctypes.data)
    got = oracle.hash_bulk(keys, key_bytes)
    assert np.array_equal(got, ref)


def test_crc_linearity_property():
    # The crc32 register update has no inversion, so it is linear over GF(2)
    # in (register, data): crc(a ^ b, x ^ y) = crc(a, x) ^ crc(b, y).
    rng = np.random.default_rng(3)
    for _ in range(500):
        a, b = (int(v) for v in rng.integers(0, 1 << 32, size=2))
        x, y = (int(v) for v in rng.integers(0, 1 << 62, size=2))
        lhs = oracle.crc32c_word(a ^ b, x ^ y, 8)
        rhs = oracle.crc32c_word(a, x, 8) ^ oracle.crc32c_word(b, y, 8)
        assert lhs == rhs
    # consequence used nowhere in the oracle: hi ^ lo depends only on the seeds
    k1, k2 = 123456789, 987654321
    h1, h2 = oracle.hash64(k1, 8), oracle.hash64(k2, 8)
    assert ((h1 >> 32) ^ (h1 & 0xFFFFFFFF)) == ((h2 >> 32) ^ (h2 & 0xFFFFFFFF))


def test_u32_key_hash_is_injective_in_high_word():
    # A 4-byte CRC update is a bijection of the 32-bit register, so distinct
    # u32 keys get distinct upper hash words.
    keys = np.arange(2, 2 + (1 << 18), dtype=np.uint32)
    h = oracle.hash_bulk(keys, 4)
    assert np.unique(h >> np.uint64(32)).size == keys.size


def test_scaling_map_closed_form():
    # h_c(x) = floor(h * c / 2^64) for c = 2^k
    rng = np.random.default_rng(5)
    for _ in range(2000):
        h = int(rng.integers(0, 1 << 63)) * 2 + int(rng.integers(0, 2))
        k = int(rng.integers(1, 41))
        assert oracle.home(h, k) == (h * (1 << k)) // (1 << 64)
    assert oracle.home(0xFFFFFFFFFFFFFFFF, 1) == 1
    assert oracle.home(0x7FFFFFFFFFFFFFFF, 1) == 0
    assert oracle.home(12345, 64) == 12345  # c = 2^64: identity


def test_scaling_map_monotone_and_nested():
    # Monotone in h, and the position at 2c is 2*pos or 2*pos+1 (Lemma 1's premise).
    rng = np.random.default_rng(9)
    hs = sorted(int(v) * 4 for v in rng.integers(0, 1 << 62, size=3000))
    for k in (4, 12, 21, 28):
        pos = [oracle.home(h, k) for h in hs]
        assert pos == sorted(pos)
        for h, p in zip(hs[:300], pos[:300]):
            assert oracle.home(h, k + 1) in (2 * p, 2 * p + 1)
