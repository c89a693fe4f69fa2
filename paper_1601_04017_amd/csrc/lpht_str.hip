// String keys of liblpht (Sec. 5.7, "Complex Keys").
//
// The table stores references to keys held in a byte pool that the table
// manages.  A cell is two words: the reference word, (signature << 48) |
// pool offset, and the value.  The signature is the low 16 bits of the
// key's 64-bit hash, bits the position (the top log2 c bits) does not use,
// kept in bits of the reference a 48-bit offset leaves free; a probe
// compares signatures first and follows the reference only when they agree.
// Reference words 0 and 1 are the empty cell and the tombstone; pool offsets
// start at 8, so no reference is 0 or 1.
//
// A pool record is a 32-bit length followed by the bytes, rounded up to 8
// bytes.  Records are allocated by bumping a device cursor; an insertion
// writes its record, makes it visible (release fence), then publishes the
// reference with compare-and-swap; a reader that meets the reference fences
// (acquire) before reading the record.  Records of erased keys, and the rare
// record of an insertion that lost a race to an equal key, stay in the pool
// until the next migration, which copies only live keys into a new pool
// (the paper reclaims key space when the array is migrated).
//
// The hash is the pair of CRC-32C register updates over the key's bytes with
// the two seeds (Sec. 8.3), the same function as for word keys.

#include <hip/hip_runtime.h>

#include "lpht_device.h"
#include "lpht_str.h"

namespace lpht {

namespace {

constexpr u64 kOffMask = (1ull << 48) - 1;

__device__ __forceinline__ uint32_t crc_byte(const uint32_t (*T)[256], uint32_t r, uint32_t b) {
  return (r >> 8) ^ T[0][(r ^ b) & 0xFFu];
}

// 64-bit hash of bytes s[0..len) (global memory, any alignment).
__device__ __forceinline__ u64 str_hash(const uint32_t (*T)[256], const uint8_t *s, u64 len, uint32_t seed_hi,
                                        uint32_t seed_lo) {
  uint32_t hi = seed_hi, lo = seed_lo;
  for (u64 i = 0; i < len; ++i) {
    const uint32_t b = s[i];
    hi = crc_byte(T, hi, b);
    lo = crc_byte(T, lo, b);
  }
  return ((u64)hi << 32) | lo;
}

__device__ __forceinline__ u64 rec_bytes(u64 len) { return (4 + len + 7) & ~7ull; }

__device__ __forceinline__ bool rec_equal(const uint8_t *pool, u64 off, const uint8_t *s, u64 len) {
  if (*(const uint32_t *)(pool + off) != (uint32_t)len) return false;
  const uint8_t *r = pool + off + 4;
  for (u64 i = 0; i < len; ++i)
    if (r[i] != s[i]) return false;
  return true;
}

__device__ __forceinline__ u64 ld_ref(const u64 *cells, u64 p) {
  return __hip_atomic_load(cells + 2 * p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One operation per thread.
template <int KIND>
__global__ void __launch_bounds__(256) k_str_op(StrArgs a) {
  __shared__ uint32_t T[8][256];
  crc_tables_build(T);
  const u64 mask = (1ull << a.log2c) - 1;
  u64 *cells = (u64 *)a.cells;
  const u64 stride = (u64)gridDim.x * blockDim.x;
  uint32_t err = 0;
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += stride) {
    const u64 o0 = a.offsets[i], len = a.offsets[i + 1] - o0;
    const uint8_t *s = a.bytes + o0;
    const u64 h = str_hash(T, s, len, a.crc_hi, a.crc_lo);
    const u64 sig = h & 0xFFFFull;
    u64 p = h >> (64 - a.log2c);
    const u64 d = a.vals ? a.vals[i] : 1;
    uint8_t flag = (KIND == kStrFind || KIND == kStrErase) ? 0 : 0xFF;
    u64 out = 0;
    u64 mine = 0;  // reference of this operation's record, once written
    for (u64 step = 0; step <= mask; ++step, p = (p + 1) & mask) {
      u64 r = ld_ref(cells, p);
      if (r == kEmpty) {
        if (KIND == kStrFind || KIND == kStrErase) break;
        if (!mine) {
          const u64 need = rec_bytes(len);
          const u64 off = atomicAdd((unsigned long long *)&a.ctl->pool_used, (unsigned long long)need);
          if (off + need > a.pool_cap) {
            err |= kErrFull;
            break;  // flag stays 0xFF
          }
          *(uint32_t *)(a.pool + off) = (uint32_t)len;
          for (u64 q = 0; q < len; ++q) a.pool[off + 4 + q] = s[q];
          __threadfence();
          mine = (sig << 48) | off;
        }
        const u64 prev = cas64(cells + 2 * p, kEmpty, mine);
        if (prev == kEmpty) {
          if (KIND == kStrInsert || a.up == 0)
            __hip_atomic_store(cells + 2 * p + 1, d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          else
            add64(cells + 2 * p + 1, d);
          flag = 1;
          break;
        }
        r = prev;
      }
      if (r == kTomb || (r >> 48) != sig) continue;
      __threadfence();
      if (!rec_equal(a.pool, r & kOffMask, s, len)) continue;
      // the key is present in cell p
      if (KIND == kStrFind) {
        out = __hip_atomic_load(cells + 2 * p + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        flag = 1;
      } else if (KIND == kStrErase) {
        flag = cas64(cells + 2 * p, r, kTomb) == r ? 1 : 0;
      } else {
        if (KIND == kStrUpsert) {
          if (a.up == 0)
            __hip_atomic_store(cells + 2 * p + 1, d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          else
            add64(cells + 2 * p + 1, d);
        }
        flag = 0;
      }
      break;
    }
    if ((KIND == kStrInsert || KIND == kStrUpsert) && flag == 0xFF) err |= kErrFull;
    if (a.flags) a.flags[i] = flag;
    if (KIND == kStrFind && a.vals_out) a.vals_out[i] = out;
  }
  if (err) atomicOr(&a.ctl->err, err);
}

// Migration: every live key of the old table is copied into the new pool and
// inserted into the new (zeroed) table with compare-and-swap.
__global__ void __launch_bounds__(256) k_str_migrate(StrMigArgs a) {
  __shared__ uint32_t T[8][256];
  crc_tables_build(T);
  const u64 oc = 1ull << a.log2_old, nmask = (1ull << a.log2_new) - 1;
  const u64 stride = (u64)gridDim.x * blockDim.x;
  uint32_t err = 0;
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < oc; i += stride) {
    const u64 r = a.old_cells[2 * i];
    if (r == kEmpty || r == kTomb) continue;
    const u64 off = r & kOffMask;
    const u64 len = *(const uint32_t *)(a.old_pool + off);
    const uint8_t *s = a.old_pool + off + 4;
    const u64 h = str_hash(T, s, len, a.crc_hi, a.crc_lo);
    const u64 need = rec_bytes(len);
    const u64 noff = atomicAdd((unsigned long long *)&a.ctl->pool_used, (unsigned long long)need);
    if (noff + need > a.new_pool_cap) {
      err |= kErrFull;
      continue;
    }
    // records are 8-byte aligned: copy whole words
    for (u64 q = 0; q < need; q += 8) *(u64 *)(a.new_pool + noff + q) = *(const u64 *)(a.old_pool + off + q);
    const u64 ref = ((h & 0xFFFFull) << 48) | noff;
    u64 p = h >> (64 - a.log2_new);
    for (u64 step = 0; step <= nmask; ++step, p = (p + 1) & nmask) {
      if (cas64((u64 *)a.new_cells + 2 * p, kEmpty, ref) == kEmpty) {
        a.new_cells[2 * p + 1] = a.old_cells[2 * i + 1];
        break;
      }
    }
  }
  if (err) atomicOr(&a.ctl->err, err);
}

__global__ void __launch_bounds__(256) k_str_recount(const u64 *cells, u64 cap, StrCtl *ctl) {
  const u64 stride = (u64)gridDim.x * blockDim.x;
  long long u = 0, l = 0;
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < cap; i += stride) {
    const u64 r = cells[2 * i];
    u += r != kEmpty;
    l += r != kEmpty && r != kTomb;
  }
  u = wave_sum(u);
  l = wave_sum(l);
  if ((threadIdx.x & 63) == 0) {
    if (u) add64(&ctl->used, (u64)u);
    if (l) add64(&ctl->live, (u64)l);
  }
}

__global__ void k_str_ctl(StrCtl *ctl, u64 pool_used, int keep_pool) {
  if (threadIdx.x == 0) {
    ctl->used = 0;
    ctl->live = 0;
    if (!keep_pool) ctl->pool_used = pool_used;
  }
}

uint32_t grid_of(u64 items, uint32_t num_cus) {
  u64 b = (items + 255) / 256;
  const u64 cap = (u64)(num_cus ? num_cus : 1) * 8;
  if (b > cap) b = cap;
  return (uint32_t)(b ? b : 1);
}

}  // namespace

hipError_t launch_str_op(int kind, const StrArgs &a, uint32_t num_cus, hipStream_t s) {
  const uint32_t g = grid_of(a.n, num_cus);
  switch (kind) {
    case kStrInsert: hipLaunchKernelGGL(k_str_op<kStrInsert>, dim3(g), dim3(256), 0, s, a); break;
    case kStrUpsert: hipLaunchKernelGGL(k_str_op<kStrUpsert>, dim3(g), dim3(256), 0, s, a); break;
    case kStrFind: hipLaunchKernelGGL(k_str_op<kStrFind>, dim3(g), dim3(256), 0, s, a); break;
    case kStrErase: hipLaunchKernelGGL(k_str_op<kStrErase>, dim3(g), dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_str_migrate(const StrMigArgs &a, uint32_t num_cus, hipStream_t s) {
  hipLaunchKernelGGL(k_str_ctl, dim3(1), dim3(64), 0, s, a.ctl, (u64)8, 0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_str_migrate, dim3(grid_of(1ull << a.log2_old, num_cus)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_str_recount(const void *cells, uint32_t log2c, StrCtl *ctl, uint32_t num_cus, hipStream_t s) {
  hipLaunchKernelGGL(k_str_ctl, dim3(1), dim3(64), 0, s, ctl, (u64)0, 1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_str_recount, dim3(grid_of(1ull << log2c, num_cus)), dim3(256), 0, s, (const u64 *)cells,
                     1ull << log2c, ctl);
  return hipGetLastError();
}

hipError_t launch_str_init(StrCtl *ctl, hipStream_t s) {
  hipLaunchKernelGGL(k_str_ctl, dim3(1), dim3(64), 0, s, ctl, (u64)8, 0);
  return hipGetLastError();
}

}  // namespace lpht
