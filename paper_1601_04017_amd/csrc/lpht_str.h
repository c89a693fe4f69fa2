// Internal interface of the string-key table (lpht_str.hip,
// lpht_str_api.cpp).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lpht_internal.h"

namespace lpht {

enum StrKind : int { kStrInsert = 0, kStrUpsert = 1, kStrFind = 2, kStrErase = 3 };

struct alignas(128) StrCtl {      // device memory, one per table
  unsigned long long pool_used;   // bytes of the pool handed out (records start at 8)
  unsigned long long used, live;  // set by a recount
  unsigned int err;               // kErrFull: a record did not fit the pool
  unsigned int pad0;
  unsigned long long pool_start;  // pool_used when the running inserting launch began
  unsigned long long pad[11];
};

struct StrArgs {
  void *cells;                 // 2^log2c cells of two words: reference, value
  uint32_t log2c;
  uint32_t up;                 // 0 assign, 1 add (insert-or-update)
  uint8_t *pool;
  uint64_t pool_cap;
  StrCtl *ctl;
  uint32_t crc_hi, crc_lo;     // the seeds: the registers start from them
  const uint8_t *bytes;        // key i = bytes[offsets[i] .. offsets[i + 1])
  const uint64_t *offsets;
  uint64_t n;
  const uint64_t *vals;        // may be null: every value is 1
  uint64_t *vals_out;          // finds; may be null
  uint8_t *flags;              // may be null
};

struct StrMigArgs {
  const uint64_t *old_cells;
  uint32_t log2_old;
  const uint8_t *old_pool;
  uint64_t *new_cells;         // zeroed
  uint32_t log2_new;
  uint8_t *new_pool;
  uint64_t new_pool_cap;
  StrCtl *ctl;                 // pool cursor restarted at 8 for the new pool
  uint32_t crc_hi, crc_lo;
};

hipError_t launch_str_init(StrCtl *ctl, hipStream_t s);
hipError_t launch_str_op(int kind, const StrArgs &a, uint32_t num_cus, hipStream_t s);
hipError_t launch_str_migrate(const StrMigArgs &a, uint32_t num_cus, hipStream_t s);
hipError_t launch_str_recount(const void *cells, uint32_t log2c, StrCtl *ctl, uint32_t num_cus, hipStream_t s);

}  // namespace lpht
