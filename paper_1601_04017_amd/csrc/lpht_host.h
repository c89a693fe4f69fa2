// Host-side internals of liblpht shared by the C ABI (lpht_api.cpp) and the
// serving runtime (lpht_server.cpp).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/lpht.h"
#include "lpht_internal.h"

namespace lpht {
struct SpecialSlots;
}

struct MigTiming {
  hipEvent_t start, stop;
};

struct lpht_table {
  lpht_config cfg;
  int device;
  uint32_t log2c;
  uint32_t log2_min;  // the created capacity: the growth rule never shrinks below it
  void *cells;
  lpht::DevStatus *status;
  uint32_t crc_hi, crc_lo;  // CRC-32C of the seeds over zero key bytes (the hash's constants)
  uint64_t mul;             // nonzero: the multiplicative hash mul * key instead of the CRC pair
  // host view of the counts for the growth rule: exact at the last
  // synchronisation, plus an upper bound of insertions since then
  uint64_t known_used, known_live, pending;
  // modifying calls since known_used/known_live were last read exactly; when
  // zero the growth rule decides without reading the device counters
  uint64_t mods_since_exact;
  lpht_tuning tuning;
  lpht::LaunchCfg launch;
  lpht_stats stats;
  // full key space: the slots of keys 0 and 1, and the per-call list scratch
  lpht::SpecialSlots *special;
  uint32_t *special_scratch;
  int timing;
  std::vector<MigTiming> timed;
};

struct lpht_batch {
  static constexpr int kSlots = 16;
  int device;
  uint32_t max_ops;
  size_t slot_bytes;
  unsigned char *host[kSlots];  // pinned
  unsigned char *dev[kSlots];
  hipEvent_t ev[kSlots];
  bool used[kSlots];
  int next;
};

namespace lpht {
namespace host {

int from_hip(hipError_t e);
uint64_t cell_bytes(uint32_t layout);
// stream-ordered allocation from the library's per-device pool (or the
// table's allocator hook)
void *dev_alloc(lpht_table *t, size_t bytes, hipStream_t s);
void dev_free(lpht_table *t, void *p, size_t bytes, hipStream_t s);
void *pool_alloc(int device, size_t bytes, hipStream_t s);
void pool_free(void *p, hipStream_t s);
void fill_launch(lpht_table *t);
bool tuning_ok(const lpht_tuning *u);
bool within_fill(const lpht_table *t, uint64_t x, uint64_t c);
int read_status(lpht_table *t, hipStream_t s, DevStatus *h, uint64_t *used, uint64_t *live);
int sync_counts(lpht_table *t, hipStream_t s);
int resize_empty(lpht_table *t, uint32_t log2_new, hipStream_t s, uint32_t steps = 1);
int migrate_once(lpht_table *t, uint32_t log2_new, hipStream_t s);
int grow_before_batch(lpht_table *t, uint64_t b, hipStream_t s);
// What grow_before_batch would do before b insertions, on the host's counts
// (which must be exact: nothing pending, no modification since the last
// exact count): 0 nothing, 1 exactly one doubling of a non-empty table,
// 2 anything else (several doublings, a cleanup or shrink, the resize of an
// empty table).
int growth_kind(const lpht_table *t, uint64_t b);
BulkArgs make_args(lpht_table *t);
bool aligned(const void *p, size_t a);
int check_arrays(lpht_table *t, const void *keys, const void *vals, uint64_t n);
int run_bulk(lpht_table *t, OpKind op, const void *keys, const void *vals, uint64_t n, uint32_t up,
             void *vals_out, uint8_t *flags, void *stream);

}  // namespace host
}  // namespace lpht
