// Internal interface of the sort-based bulk build and batched merge
// (lpht_bulk.hip), used by the host side of liblpht.  Not part of the public
// C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lpht_internal.h"

namespace lpht {

// Largest target table of a bulk build / merge (2^29 cells): the two
// partition levels then need at most 2^10 and 2^11 bins.
constexpr uint32_t kBulkMaxLog2 = 29;

struct BulkMergeArgs {
  uint32_t layout;         // 0 packed32, 1 kv64
  uint32_t op;             // 0 assign (last occurrence wins), 1 add (wrapping sum)
  const void *old_cells;   // the table's cells when merging, else null
  uint64_t old_ncells;     // cells of old_cells (0 when building)
  const void *keys;        // the batch (device), n keys
  const void *vals;        // n values, or null (every value is 1)
  uint64_t n;
  uint64_t max_items;      // upper bound of live old elements + n (sizes the staging)
  void *new_cells;         // 2^log2_new cells, need not be initialised
  uint32_t log2_new;       // 6 .. kBulkMaxLog2
  uint32_t crc_hi, crc_lo;
  uint64_t mul;            // nonzero: multiplicative hash mul * key (else the CRC-32C pair)
  DevStatus *status;       // counts zeroed by the caller; receives used = live = distinct keys
  void *scratch;           // bulk_merge_scratch_bytes(...) bytes of device memory
  uint32_t num_cus;
};

// Device-side results, at the start of the scratch block (read back by the
// host after the call).
struct BulkMergeCtl {
  unsigned long long distinct;  // distinct keys of the result
  unsigned long long wrapped;   // elements whose probe wrapped past the last cell
  unsigned int full;            // 1: more distinct keys than cells; 2: more elements than the
                                // staging holds (inconsistent counts); nothing was written
  unsigned int big_blocks;      // target blocks sorted by the global-memory path
  unsigned int mid_blocks;      // target blocks sorted by a whole workgroup
  unsigned int pad0;
  unsigned long long pad[4];
};

// Scratch for `inputs` = old_ncells + n input positions of which at most
// `max_items` are elements.
size_t bulk_merge_scratch_bytes(uint64_t inputs, uint64_t max_items, uint32_t log2_new, uint32_t layout);

// Size of the fixed device scratch used by lpht_build_noalloc.
constexpr size_t kNoAllocScratchBytes = 64ull << 20;

// The device address of that scratch on `device` (looked up once per device
// with the device current, then cached).
hipError_t noalloc_scratch(int device, void **out);

// Enqueues the whole operation on `s`.  The result (when ctl->full == 0) is
// the table obtained by inserting the distinct keys one by one in increasing
// order of (hash, key) into an empty table of 2^log2_new cells.
hipError_t launch_bulk_merge(const BulkMergeArgs &a, hipStream_t s);

}  // namespace lpht
