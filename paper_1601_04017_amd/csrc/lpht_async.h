// Internal interface of the inserting kernel that grows the table while it
// runs (lpht_async.hip), used by the host side of liblpht.  Not part of the
// public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lpht_internal.h"

namespace lpht {

constexpr uint32_t kAsyncLadder = 16;     // most doublings one call can make
constexpr uint32_t kAsyncChunk = 64;      // operations of one round (one per lane)
constexpr uint32_t kAsyncMaxRounds = 64;  // rounds per chunk a wavefront takes at a time (at most)
constexpr uint32_t kAsyncFlushMax = 64;   // on the smallest tables a local count is flushed after 1..64 insertions
constexpr uint32_t kAsyncMigBlock = 4096; // old cells per work item of the fallback re-insertion

// Shared counters are split over kAsyncShards 128-byte lines, wavefront w
// using line w % kAsyncShards: one line takes about 80 million agent-scope
// read-modify-writes a second from all compute units together, far too few
// for thousands of wavefronts adding to one counter.
constexpr uint32_t kAsyncShards = 64;
struct alignas(128) AsyncLine {
  unsigned long long v;
  unsigned long long pad[15];
};

// Device control block (zeroed by the launcher).
struct alignas(128) AsyncCtl {
  AsyncLine count[kAsyncShards];  // flushed insertions since the current version began, per shard
  AsyncLine moved[kAsyncShards];  // elements moved by the running migration, per shard
  AsyncLine arrive[kAsyncShards]; // arrivals at the current growth's barriers, per shard
  unsigned long long base;        // non-empty cells of the current table when its version began
  unsigned long long pad0[15];
  unsigned int gen;              // 2 * epoch + 1 from a growth's trigger to its end, else 2 * epoch
  unsigned int arrived;          // shards whose wavefronts all passed the current barrier (cumulative)
  unsigned int epoch;            // completed migrations; the current table is ladder[epoch]
  unsigned int finished;         // wavefronts that found no work left
  unsigned int err;              // 1: a wait passed its bound; 2: the ladder ran out
  unsigned int pad1[27];
  // work items of the fallback, apart from the line waiting wavefronts poll
  unsigned int mig_overflow;     // 1: a block saw a cluster longer than the halo
  unsigned int mig_next2;        // fallback: next zero-fill work item
  unsigned int mig_next3;        // fallback: next re-insertion work item
  unsigned int fallbacks;        // growths that took the fallback
  unsigned int pad2[28];
};

struct AsyncArgs {
  uint32_t layout;        // 0 packed32, 1 kv64
  uint32_t add;           // 0 insert (first wins), 1 insert-or-add
  const void *keys, *vals;  // vals may be null: every value is 1
  uint64_t n;
  uint8_t *flags;         // may be null
  void *ladder[kAsyncLadder + 1];  // ladder[0]: the table; ladder[i]: 2^(log2c + i) cells (any contents)
  uint32_t nladder;       // tables in the ladder (>= 1)
  uint32_t log2c;         // capacity of ladder[0]
  uint64_t used0;         // non-empty cells of ladder[0] at the start (exact)
  uint32_t alpha_num, alpha_den;
  uint32_t crc_hi, crc_lo;
  uint64_t mul;           // nonzero: multiplicative hash mul * key (else the CRC-32C pair)
  AsyncCtl *ctl;
  DevStatus *status;      // sticky error bits (reserved keys)
  uint32_t grid;          // workgroups of 256 threads, all resident (cooperative launch)
};

// Workgroups the cooperative launch uses on this device (0 if unsupported).
uint32_t async_grid(int device);
// Smallest capacity (log2) the kernel accepts for alpha = num/den: the
// operations in flight and the unflushed counts must fit the free cells.
uint32_t async_min_log2(uint32_t grid, uint32_t alpha_num, uint32_t alpha_den);

hipError_t launch_async_insert(const AsyncArgs &a, hipStream_t s);

}  // namespace lpht
