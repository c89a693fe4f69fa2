// Internal interface of the full-key-space support (lpht_special.hip), used
// by the host side of liblpht.  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lpht_internal.h"

namespace lpht {

// The two special slots of a table with the full key space (Sec. 5.6):
// slot k holds key k (0 = empty_key, 1 = del_key) when present[k] is 1.
struct alignas(128) SpecialSlots {
  unsigned long long present[2];
  unsigned long long value[2];
  unsigned long long pad[12];
};

// Operations on keys 0 and 1 listed per call: up to kSpecialList of them go
// through a list; beyond that the batch is scanned in order.
constexpr uint32_t kSpecialList = 8192;
// Device scratch per table: a counter and the list.
constexpr size_t kSpecialScratchBytes = sizeof(uint32_t) * (kSpecialList + 64);

// Applies the operations of a batch whose key is 0 or 1 to the special
// slots, in index order, writing their flags (and values for finds) over
// what the cell kernels wrote for them.  op: OP_FIND, OP_INSERT, OP_UPSERT,
// OP_UPDATE or OP_ERASE; up: 0 assign, 1 add.  `clear` first empties the
// slots (a bulk build).
hipError_t launch_special(uint32_t layout, OpKind op, uint32_t up, const void *keys, const void *vals, uint64_t n,
                          void *vals_out, uint8_t *flags, SpecialSlots *sp, uint32_t *scratch, bool clear,
                          hipStream_t s);

}  // namespace lpht
