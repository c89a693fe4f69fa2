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
// reference with compare-and-swap; a reader that meets a reference written
// during its own launch fences (acquire) before reading the record.  Records
// of erased keys, and the rare
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

// 8 bytes at any alignment (one or two wide loads; never past p + 7).
__device__ __forceinline__ u64 ld8(const uint8_t *p) {
  u64 x;
  __builtin_memcpy(&x, p, 8);
  return x;
}

__device__ __forceinline__ void st8(uint8_t *p, u64 x) { __builtin_memcpy(p, &x, 8); }

// 64-bit hash of bytes s[0..len) (global memory, any alignment).  Eight
// bytes at a time: with the register XORed into their low word, the
// register after them is CRC(0, chunk) (the slicing tables); then the tail
// byte by byte.
__device__ __forceinline__ u64 str_hash(const uint32_t (*T)[256], const uint8_t *s, u64 len, uint32_t seed_hi,
                                        uint32_t seed_lo) {
  uint32_t hi = seed_hi, lo = seed_lo;
  u64 i = 0;
  for (; i + 8 <= len; i += 8) {
    const u64 x = ld8(s + i);
    hi = crc0_u64(T, x ^ hi);
    lo = crc0_u64(T, x ^ lo);
  }
  for (; i < len; ++i) {
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
  u64 i = 0;
  for (; i + 8 <= len; i += 8)
    if (ld8(r + i) != ld8(s + i)) return false;
  for (; i < len; ++i)
    if (r[i] != s[i]) return false;
  return true;
}

// Writes the record of s[0..len) at pool offset off (8-aligned).
__device__ __forceinline__ void rec_write(uint8_t *pool, u64 off, const uint8_t *s, u64 len) {
  *(uint32_t *)(pool + off) = (uint32_t)len;
  uint8_t *r = pool + off + 4;
  u64 i = 0;
  for (; i + 8 <= len; i += 8) st8(r + i, ld8(s + i));
  for (; i < len; ++i) r[i] = s[i];
}

__device__ __forceinline__ u64 ld_ref(const u64 *cells, u64 p) {
  return __hip_atomic_load(cells + 2 * p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Whether the cell's reference word r names the key s[0..len).  Records at
// pool offsets below `fresh_from` were written by earlier launches, which
// the kernel boundary has made visible; a record this launch may have
// written is read after an acquire fence, which pairs with the writer's
// release fence before its compare-and-swap.
__device__ __forceinline__ bool same_key(const uint8_t *pool, u64 r, u64 sig, const uint8_t *s, u64 len,
                                         u64 fresh_from) {
  if (r == kTomb || (r >> 48) != sig) return false;
  const u64 off = r & kOffMask;
  if (off >= fresh_from) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return rec_equal(pool, off, s, len);
}

// Exclusive prefix sum of v over the wavefront's 64 lanes (all active);
// `total` receives the sum.
__device__ __forceinline__ u64 wave_excl_scan(u64 v, u64 &total) {
  const int lane = threadIdx.x & 63;
  u64 x = v;
  for (int o = 1; o < 64; o <<= 1) {
    const u64 y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  total = __shfl(x, 63, 64);
  return x - v;
}

// Operations per lane between release fences in inserting launches: the
// fence writes back the L2 and costs far more than a probe.
constexpr int kStrGroup = 8;

// A lane takes K operations (K = kStrGroup when inserting, else 1); for each
// a read-only probe ends at the key or at the first empty cell.  Inserting
// operations that ended at an empty cell then take their records from one
// pool allocation per wavefront, write them, make them visible with one
// release fence per wavefront, and publish their references with
// compare-and-swap from that cell on; a lost race continues the probe, and
// finding the key there leaves the record unused until the next migration.
template <int KIND>
__global__ void __launch_bounds__(256) k_str_op(StrArgs a) {
  constexpr bool kInserting = KIND == kStrInsert || KIND == kStrUpsert;
  constexpr int K = kInserting ? kStrGroup : 1;
  __shared__ uint32_t T[8][256];
  crc_tables_build(T);
  const u64 mask = (1ull << a.log2c) - 1;
  u64 *cells = (u64 *)a.cells;
  // A table is used from one stream at a time, so only an inserting launch
  // can meet a record written while it runs.
  const u64 fresh_from = kInserting ? a.ctl->pool_start : ~0ull;
  const u64 stride = (u64)gridDim.x * blockDim.x * K;
  uint32_t err = 0;
  // the bound is uniform over the workgroup: every lane reaches the
  // wavefront's allocation, idle lanes with nothing to allocate
  for (u64 i0 = (u64)blockIdx.x * blockDim.x * K; i0 < a.n; i0 += stride) {
    u64 len[K], sig[K], p[K], step[K], r[K], d[K], mine[K];
    const uint8_t *s[K];
    bool found[K], at_empty[K];
    uint8_t flag[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const u64 i = i0 + (u64)j * blockDim.x + threadIdx.x;
      len[j] = sig[j] = p[j] = step[j] = mine[j] = 0;
      r[j] = kEmpty;
      d[j] = 1;
      s[j] = nullptr;
      found[j] = at_empty[j] = false;
      flag[j] = kInserting ? 0xFF : 0;
      if (i >= a.n) continue;
      const u64 o0 = a.offsets[i];
      len[j] = a.offsets[i + 1] - o0;
      s[j] = a.bytes + o0;
      if (a.vals) d[j] = a.vals[i];
      const u64 h = str_hash(T, s[j], len[j], a.crc_hi, a.crc_lo);
      sig[j] = h & 0xFFFFull;
      p[j] = h >> (64 - a.log2c);
      for (; step[j] <= mask; ++step[j], p[j] = (p[j] + 1) & mask) {
        r[j] = ld_ref(cells, p[j]);
        if (r[j] == kEmpty) {
          at_empty[j] = true;
          break;
        }
        if (same_key(a.pool, r[j], sig[j], s[j], len[j], fresh_from)) {
          found[j] = true;
          break;
        }
      }
    }
    if (kInserting) {
      // one allocation per wavefront, laid out by j: the records of the
      // wavefront's j-th operations are consecutive
      u64 total = 0;
#pragma unroll
      for (int j = 0; j < K; ++j) total += (u64)wave_sum((long long)(at_empty[j] ? rec_bytes(len[j]) : 0));
      u64 base = 0;
      if ((threadIdx.x & 63) == 0 && total)
        base = atomicAdd((unsigned long long *)&a.ctl->pool_used, (unsigned long long)total);
      base = __shfl(base, 0, 64);
      bool wrote = false;
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const u64 need = at_empty[j] ? rec_bytes(len[j]) : 0;
        u64 tj;
        const u64 off = base + wave_excl_scan(need, tj);
        base += tj;
        if (!need) continue;
        if (off + need > a.pool_cap) {
          err |= kErrFull;  // flag stays 0xFF
        } else {
          rec_write(a.pool, off, s[j], len[j]);
          mine[j] = (sig[j] << 48) | off;
          wrote = true;
        }
      }
      if (wrote) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
#pragma unroll
      for (int j = 0; j < K; ++j) {
        if (!mine[j]) continue;
        // cell p[j] was empty when the probe passed it
        for (r[j] = kEmpty; step[j] <= mask; ++step[j], p[j] = (p[j] + 1) & mask, r[j] = ld_ref(cells, p[j])) {
          if (r[j] == kEmpty) {
            const u64 prev = cas64(cells + 2 * p[j], kEmpty, mine[j]);
            if (prev == kEmpty) {
              if (KIND == kStrInsert || a.up == 0)
                __hip_atomic_store(cells + 2 * p[j] + 1, d[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              else
                add64(cells + 2 * p[j] + 1, d[j]);
              flag[j] = 1;
              break;
            }
            r[j] = prev;
          }
          if (same_key(a.pool, r[j], sig[j], s[j], len[j], fresh_from)) {
            found[j] = true;
            break;
          }
        }
      }
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const u64 i = i0 + (u64)j * blockDim.x + threadIdx.x;
      if (i >= a.n) continue;
      u64 out = 0;
      if (found[j]) {
        // the key is present in cell p[j], whose reference word is r[j]
        const u64 q = p[j];
        if (KIND == kStrFind) {
          out = __hip_atomic_load(cells + 2 * q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          flag[j] = 1;
        } else if (KIND == kStrErase) {
          flag[j] = cas64(cells + 2 * q, r[j], kTomb) == r[j] ? 1 : 0;
        } else {
          if (KIND == kStrUpsert) {
            if (a.up == 0)
              __hip_atomic_store(cells + 2 * q + 1, d[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            else
              add64(cells + 2 * q + 1, d[j]);
          }
          flag[j] = 0;
        }
      }
      if (kInserting && flag[j] == 0xFF) err |= kErrFull;
      if (a.flags) a.flags[i] = flag[j];
      if (KIND == kStrFind && a.vals_out) a.vals_out[i] = out;
    }
  }
  if (err) atomicOr(&a.ctl->err, err);
}

// Migration: every live key of the old table is copied into the new pool
// (one allocation per wavefront) and inserted into the new (zeroed) table
// with compare-and-swap.
__global__ void __launch_bounds__(256) k_str_migrate(StrMigArgs a) {
  __shared__ uint32_t T[8][256];
  crc_tables_build(T);
  const u64 oc = 1ull << a.log2_old, nmask = (1ull << a.log2_new) - 1;
  const u64 stride = (u64)gridDim.x * blockDim.x;
  uint32_t err = 0;
  for (u64 i0 = (u64)blockIdx.x * blockDim.x; i0 < oc; i0 += stride) {
    const u64 i = i0 + threadIdx.x;
    const u64 r = i < oc ? a.old_cells[2 * i] : kEmpty;
    const bool live = r != kEmpty && r != kTomb;
    const u64 off = r & kOffMask;
    const u64 len = live ? *(const uint32_t *)(a.old_pool + off) : 0;
    const u64 need = live ? rec_bytes(len) : 0;
    u64 total;
    const u64 pre = wave_excl_scan(need, total);
    u64 base = 0;
    if ((threadIdx.x & 63) == 0 && total)
      base = atomicAdd((unsigned long long *)&a.ctl->pool_used, (unsigned long long)total);
    base = __shfl(base, 0, 64);
    if (!live) continue;
    const u64 noff = base + pre;
    if (noff + need > a.new_pool_cap) {
      err |= kErrFull;
      continue;
    }
    const uint8_t *s = a.old_pool + off + 4;
    const u64 h = str_hash(T, s, len, a.crc_hi, a.crc_lo);
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

// Marks where records of the next launch will start.
__global__ void k_str_snap(StrCtl *ctl) {
  if (threadIdx.x == 0) ctl->pool_start = ctl->pool_used;
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
  drop_stale_error();
  const bool inserting = kind == kStrInsert || kind == kStrUpsert;
  const uint32_t g = grid_of(inserting ? (a.n + kStrGroup - 1) / kStrGroup : a.n, num_cus);
  if (inserting) {
    hipLaunchKernelGGL(k_str_snap, dim3(1), dim3(64), 0, s, a.ctl);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
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
  drop_stale_error();
  hipLaunchKernelGGL(k_str_ctl, dim3(1), dim3(64), 0, s, a.ctl, (u64)8, 0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_str_migrate, dim3(grid_of(1ull << a.log2_old, num_cus)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_str_recount(const void *cells, uint32_t log2c, StrCtl *ctl, uint32_t num_cus, hipStream_t s) {
  drop_stale_error();
  hipLaunchKernelGGL(k_str_ctl, dim3(1), dim3(64), 0, s, ctl, (u64)0, 1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_str_recount, dim3(grid_of(1ull << log2c, num_cus)), dim3(256), 0, s, (const u64 *)cells,
                     1ull << log2c, ctl);
  return hipGetLastError();
}

hipError_t launch_str_init(StrCtl *ctl, hipStream_t s) {
  drop_stale_error();
  hipLaunchKernelGGL(k_str_ctl, dim3(1), dim3(64), 0, s, ctl, (u64)8, 0);
  return hipGetLastError();
}

}  // namespace lpht
