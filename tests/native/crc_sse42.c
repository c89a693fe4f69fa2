/* Test helper: calls the host CPU's SSE4.2 crc32 instruction so that the
 * oracle's bit-by-bit CRC-32C can be compared with an independent hardware
 * implementation.  Built with gcc -msse4.2 by the tests; never part of the
 * product or the oracle. */
#include <nmmintrin.h>
#include <stdint.h>

uint32_t hw_crc_u8(uint32_t reg, uint8_t x) { return _mm_crc32_u8(reg, x); }
uint32_t hw_crc_u32(uint32_t reg, uint32_t x) { return _mm_crc32_u32(reg, x); }
uint32_t hw_crc_u64(uint32_t reg, uint64_t x) { return (uint32_t)_mm_crc32_u64(reg, x); }

void hw_hash_bulk(const void *keys, uint64_t n, int key_bytes, uint32_t seed_hi, uint32_t seed_lo,
                  uint64_t *out) {
  for (uint64_t i = 0; i < n; ++i) {
    uint64_t hi, lo;
    if (key_bytes == 4) {
      uint32_t k = ((const uint32_t *)keys)[i];
      hi = _mm_crc32_u32(seed_hi, k);
      lo = _mm_crc32_u32(seed_lo, k);
    } else {
      uint64_t k = ((const uint64_t *)keys)[i];
      hi = (uint32_t)_mm_crc32_u64(seed_hi, k);
      lo = (uint32_t)_mm_crc32_u64(seed_lo, k);
    }
    out[i] = (hi << 32) | lo;
  }
}
