// Internal interface of the partitioned insert-or-add (lpht_part.hip), used
// by the host side of liblpht for large insertOrUpdate calls with the "add"
// update function.  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lpht_internal.h"

namespace lpht {

// Device scratch for a call of n operations on a table of 2^log2c cells
// (bytes); `with_vals` / `with_flags`: the call passes values / wants flags.
size_t part_scratch_bytes(uint64_t n, uint32_t log2c, uint32_t layout, bool with_vals, bool with_flags,
                          uint32_t num_cus);

// Whether the partitioned path takes a call of n operations on a table of
// 2^log2c cells (large calls on tables far beyond the caches).
bool part_applies(uint64_t n, uint32_t log2c);

// Enqueues the insert-or-add of a.keys[0..a.n) (values a.vals, or 1 each;
// flags a.flags, may be null) on `s`: the batch is partitioned by the top
// bits of its hash, i.e. by table region, equal keys of a bucket are combined
// in LDS, and one upsert per distinct key is applied.  The table must not
// run out of empty cells during the call (as for the LDS-combining kernel).
hipError_t launch_upsert_add_part(const BulkArgs &a, void *scratch, uint32_t num_cus, hipStream_t s);

}  // namespace lpht
