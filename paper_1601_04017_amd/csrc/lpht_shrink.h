// Internal interface of the shrinking migration (lpht_shrink.hip), used by
// the host side of liblpht.  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lpht_internal.h"

namespace lpht {

// Target tables of at least 2^kShrinkLocalLog2 cells are filled in two phases
// (block-local placement, then concurrent insertion of what did not fit,
// Sec. 5.3.1 "Shrinking"); smaller ones by concurrent insertion of every
// element, since they have too few target blocks to occupy the device.
constexpr uint32_t kShrinkLocalLog2 = 19;
constexpr uint32_t kShrinkBlock = 256;  // target cells per wavefront in the first phase

// Device scratch the shrink needs (one u32 per target block), 0 when none.
size_t shrink_scratch_bytes(uint32_t log2_old, uint32_t log2_new);

// Migrates the live elements of `old_cells` (2^log2_old cells) into
// `new_cells` (2^log2_new cells, log2_new < log2_old; need not be
// initialised), which must hold more cells than there are live elements.
// The cells of the old table are overwritten (it is discarded afterwards).
// `scratch` holds shrink_scratch_bytes(...) bytes of device memory (may be
// null when that is 0).  Adds the number of moved elements to the used and
// live counts (the caller zeroes them first); sets kErrFull if an element
// found no empty cell.
hipError_t launch_shrink(void *old_cells, uint32_t log2_old, void *new_cells, uint32_t log2_new,
                         uint32_t layout, uint32_t crc_hi, uint32_t crc_lo, uint64_t mul, uint32_t *scratch,
                         DevStatus *st, const LaunchCfg &cfg, hipStream_t s);

}  // namespace lpht
