// Device helpers of liblpht shared by its kernel sources: the hash (CRC-32C
// pair, Sec. 8.3) and the position map (Sec. 5.3.1), device atomics, count
// reductions and cell access.  Included by lpht_kernels.hip and
// lpht_shrink.hip only.
#pragma once

#include <hip/hip_runtime.h>

#include <stdint.h>

#include "lpht_internal.h"

namespace lpht {

typedef unsigned long long u64;
typedef u64 u64x2 __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------------- CRC-32C

constexpr uint32_t kPolyRefl = 0x82F63B78u;  // Castagnoli, reflected

// T[j][b] = CRC register after feeding byte b and then j zero bytes,
// starting from register 0.
__device__ __forceinline__ void crc_tables_build(uint32_t (*T)[256]) {
  for (uint32_t b = threadIdx.x; b < 256; b += blockDim.x) {
    uint32_t r = b;
#pragma unroll
    for (int k = 0; k < 8; ++k) r = (r >> 1) ^ (kPolyRefl & (0u - (r & 1u)));
    T[0][b] = r;
  }
  __syncthreads();
  for (int j = 1; j < 8; ++j) {
    for (uint32_t b = threadIdx.x; b < 256; b += blockDim.x) {
      uint32_t r = T[j - 1][b];
      T[j][b] = (r >> 8) ^ T[0][r & 0xFFu];
    }
    __syncthreads();
  }
}

// CRC(0, x) over the 8 little-endian bytes of x: byte i contributes
// T[7 - i][byte].
__device__ __forceinline__ uint32_t crc0_u64(const uint32_t (*T)[256], u64 x) {
  uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
  return T[7][lo & 0xFF] ^ T[6][(lo >> 8) & 0xFF] ^ T[5][(lo >> 16) & 0xFF] ^ T[4][lo >> 24] ^
         T[3][hi & 0xFF] ^ T[2][(hi >> 8) & 0xFF] ^ T[1][(hi >> 16) & 0xFF] ^ T[0][hi >> 24];
}

// CRC(0, x) over the 4 little-endian bytes of a 32-bit key.
__device__ __forceinline__ uint32_t crc0_u32(const uint32_t (*T)[256], uint32_t x) {
  return T[3][x & 0xFF] ^ T[2][(x >> 8) & 0xFF] ^ T[1][(x >> 16) & 0xFF] ^ T[0][x >> 24];
}

// The table's 64-bit hash of a key.  mul == 0: the CRC-32C pair
// h = CRC(seed_hi, x) * 2^32 + CRC(seed_lo, x) (Sec. 8.3), where the CRC
// register update is linear over GF(2), so CRC(seed, x) = CRC(0, x) ^
// CRC(seed, 0) and both halves come from one table evaluation plus the host's
// constants crc_hi = CRC(seed_hi, 0), crc_lo = CRC(seed_lo, 0).  Otherwise the
// multiplicative hash mul * x mod 2^64.
template <int LAYOUT>
__device__ __forceinline__ u64 hash_of(const uint32_t (*T)[256], u64 key, uint32_t crc_hi,
                                       uint32_t crc_lo, u64 mul) {
  if (mul) return key * mul;
  uint32_t c = (LAYOUT == 0) ? crc0_u32(T, (uint32_t)key) : crc0_u64(T, key);
  return ((u64)(c ^ crc_hi) << 32) | (u64)(c ^ crc_lo);
}

// Position (Sec. 5.3.1's scaling map with U = 2^64): the top log2c bits.
template <int LAYOUT>
__device__ __forceinline__ u64 home_of(const uint32_t (*T)[256], u64 key, uint32_t crc_hi,
                                       uint32_t crc_lo, u64 mul, uint32_t log2c) {
  return hash_of<LAYOUT>(T, key, crc_hi, crc_lo, mul) >> (64 - log2c);
}

// ---------------------------------------------------------------- atomics

__device__ __forceinline__ u64 cas64(u64 *p, u64 expected, u64 desired) {
  __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
  return expected;  // the word found in memory (== the expected one on success)
}

__device__ __forceinline__ void add64(u64 *p, u64 d) {
  __hip_atomic_fetch_add(p, d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------- reductions

__device__ __forceinline__ long long wave_sum(long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Adds the per-lane deltas of used/live and ORs the error bits into the
// status block: wave reduction, LDS, then one atomic per workgroup.
__device__ __forceinline__ void flush_counts(DevStatus *st, long long d_used, long long d_live,
                                             uint32_t err, long long *s_acc, uint32_t *s_err) {
  if (threadIdx.x == 0) {
    s_acc[0] = 0;
    s_acc[1] = 0;
    *s_err = 0;
  }
  __syncthreads();
  long long u = wave_sum(d_used);
  long long l = wave_sum(d_live);
  uint64_t anyerr = __ballot(err != 0);
  uint32_t e = err;
  if (anyerr) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) e |= __shfl_xor(e, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    if (u) atomicAdd((unsigned long long *)&s_acc[0], (unsigned long long)u);
    if (l) atomicAdd((unsigned long long *)&s_acc[1], (unsigned long long)l);
    if (e) atomicOr(s_err, e);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    CountSlot *cs = &st->slot[blockIdx.x % kCountSlots];
    if (s_acc[0]) add64(&cs->used, (u64)s_acc[0]);
    if (s_acc[1]) add64(&cs->live, (u64)s_acc[1]);
    if (*s_err) atomicOr(&st->err, *s_err);
  }
}

// ---------------------------------------------------------------- cells

// Key and value of cell `i`.  PACKED32: one word, key low, value high.
// KV64: words 2i (key) and 2i+1 (value).
template <int LAYOUT>
struct Cells;

// COH: device-coherent reads (agent-scope relaxed atomic loads, which bypass
// the per-CU and per-XCD caches), used by the resident serving kernel whose
// phases synchronise without cache maintenance.
__device__ __forceinline__ u64 coh_load(const u64 *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <>
struct Cells<0> {
  template <bool COH = false>
  static __device__ __forceinline__ u64 word(const void *c, u64 i) {
    return COH ? coh_load((const u64 *)c + i) : ((const u64 *)c)[i];
  }
  static __device__ __forceinline__ u64 key_of(u64 w) { return w & 0xFFFFFFFFull; }
  static __device__ __forceinline__ u64 val_of(u64 w) { return w >> 32; }
};

template <>
struct Cells<1> {
  template <bool COH = false>
  static __device__ __forceinline__ u64x2 cell(const void *c, u64 i) {
    if (COH) {
      u64x2 v;
      v.x = coh_load((const u64 *)c + 2 * i);
      v.y = coh_load((const u64 *)c + 2 * i + 1);
      return v;
    }
    return ((const u64x2 *)c)[i];
  }
  template <bool COH = false>
  static __device__ __forceinline__ u64 key(const void *c, u64 i) {
    return COH ? coh_load((const u64 *)c + 2 * i) : ((const u64 *)c)[2 * i];
  }
};

// One insertOrUpdate(k, d, add) on the table by a single lane (Algorithm 1
// with fetch-and-add as atomicUpdate).  Returns the flag.
template <int LAYOUT>
__device__ __forceinline__ uint8_t upsert_add_one(const BulkArgs &A, const uint32_t (*T)[256], u64 k,
                                                  u64 d, long long &d_used, long long &d_live,
                                                  uint32_t &err) {
  const u64 cap = 1ull << A.log2c, mask = cap - 1;
  u64 p = home_of<LAYOUT>(T, k, A.crc_hi, A.crc_lo, A.mul, A.log2c);
  for (u64 probes = 0; probes < cap; ++probes, p = (p + 1) & mask) {
    if (LAYOUT == 0) {
      u64 *w = (u64 *)A.cells + p;
      u64 ck = *w & 0xFFFFFFFFull;
      if (ck == kEmpty) {
        const u64 old = cas64(w, 0ull, (d << 32) | k);
        if (old == 0) {
          d_used += 1;
          d_live += 1;
          return 1;
        }
        ck = old & 0xFFFFFFFFull;
      }
      if (ck == k) {
        add64(w, d << 32);
        return 0;
      }
    } else {
      u64 *kp = (u64 *)A.cells + 2 * p;
      u64 ck = *kp;
      if (ck == kEmpty) {
        const u64 old = cas64(kp, kEmpty, k);
        if (old == kEmpty) {
          add64(kp + 1, d);
          d_used += 1;
          d_live += 1;
          return 1;
        }
        ck = old;
      }
      if (ck == k) {
        add64(kp + 1, d);
        return 0;
      }
    }
  }
  err |= kErrFull;
  return 0xFF;
}

// Orders LDS accesses of the lanes of one wavefront.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace lpht
