// Internal interface between the host side of liblpht (lpht_api.cpp) and its
// HIP kernels (lpht_kernels.hip).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lpht {

constexpr uint64_t kEmpty = 0;  // empty_key
constexpr uint64_t kTomb = 1;   // del_key

constexpr uint32_t kErrFull = 1u;
constexpr uint32_t kErrReserved = 2u;
constexpr uint32_t kErrMigrate = 4u;  // a block migration saw a cluster longer than its halo

// Per-table device status block: exact counts and sticky error bits.  The
// counts are spread over kCountSlots slots, one 128-byte line each, so that
// the one-atomic-per-workgroup flush of a bulk kernel does not serialise all
// workgroups on one address; the totals are the sums over the slots.
constexpr int kCountSlots = 64;

struct alignas(128) CountSlot {
  unsigned long long used;  // non-empty cells
  unsigned long long live;  // live keys
  unsigned long long pad[14];
};

struct alignas(128) DevStatus {
  unsigned int err;              // kErr* bits
  unsigned int pad0;
  unsigned long long overflow;   // set by a migration that needs the fallback
  unsigned long long pad[14];
  CountSlot slot[kCountSlots];
};

enum OpKind : int { OP_FIND = 0, OP_INSERT = 1, OP_UPSERT = 2, OP_UPDATE = 3, OP_ERASE = 4 };

// Everything a bulk kernel needs, passed by value.
struct BulkArgs {
  void *cells;          // 2^log2c cells
  uint32_t log2c;
  uint32_t layout;      // 0 packed32, 1 kv64
  uint32_t crc_hi;      // CRC-32C of the upper seed over zero data (hash constant)
  uint32_t crc_lo;      // same for the lower seed
  DevStatus *status;
  const void *keys;
  const void *vals;     // may be null: every value is 1
  uint64_t n;
  void *vals_out;       // find only; may be null
  uint8_t *flags;       // may be null
  uint32_t up;          // 0 assign, 1 add
  uint32_t aggregate;   // 1: combine equal keys in LDS (upsert with add only)
  const uint8_t *kinds; // may be null; else only operations with kinds[i] == kind_sel run
  uint32_t kind_sel;
  uint32_t pad;
  uint64_t mul;         // nonzero: multiplicative hash mul * key; 0: the CRC-32C pair
};

struct LaunchCfg {
  uint32_t block_threads;
  uint32_t group_width;
  uint32_t blocks_per_cu;
  uint32_t num_cus;
  uint32_t migrate_block;
  uint32_t aggregate;
};

// A launch wrapper reports its launches through hipGetLastError.  HIP keeps
// the error of a failed call for the calling thread until hipGetLastError
// reads it, and later successful calls leave it in place, so a wrapper first
// drops whatever an earlier call of the thread left there (another
// library's, or a failure the caller already handled): otherwise its own
// successful launch would report that error.
inline void drop_stale_error() { (void)hipGetLastError(); }

// Kernel launchers (lpht_kernels.hip).  Each returns a hipError_t.
hipError_t launch_bulk(OpKind op, const BulkArgs &a, const LaunchCfg &cfg, hipStream_t s);
// One launch over `ndesc` descriptors of the same layout, operation and
// update function (device arrays: descs[ndesc], round_start[ndesc + 1] with
// round_start[j] = sum of ceil(n_i / kRound) for i < j).
constexpr uint32_t kRound = 128;
hipError_t launch_bulk_multi(OpKind op, uint32_t up, uint32_t layout, const BulkArgs *descs,
                             const uint64_t *round_start, uint32_t ndesc, uint64_t total_rounds,
                             const LaunchCfg &cfg, hipStream_t s);
hipError_t launch_fill_zero(void *ptr, uint64_t bytes, const LaunchCfg &cfg, hipStream_t s);
hipError_t launch_set_status(DevStatus *st, uint64_t used, uint64_t live, int clear_err,
                             hipStream_t s);
// out[0..2] = used, live, error bits of one table (out may be mapped host memory)
hipError_t launch_count_totals(const DevStatus *st, uint64_t *out, hipStream_t s);
hipError_t launch_recount(const void *cells, uint32_t log2c, uint32_t layout, DevStatus *st,
                          const LaunchCfg &cfg, hipStream_t s);
// Block-parallel cluster migration of `old_cells` (2^log2_old cells) into
// `new_cells` (2^log2_new cells, log2_new >= log2_old).  `new_cells` need not
// be initialised.  Adds the number of moved elements to the used and live
// counts (the caller zeroes them first).
hipError_t launch_migrate(const void *old_cells, uint32_t log2_old, void *new_cells,
                          uint32_t log2_new, uint32_t layout, uint32_t crc_hi, uint32_t crc_lo,
                          uint64_t mul, int old_is_full, DevStatus *st, const LaunchCfg &cfg,
                          hipStream_t s);

// ---- persistent serving kernel ----
// Requests are posted by the host into a ring in pinned host memory; one
// resident kernel deals every request's 128-operation rounds to its
// wavefronts, phase by phase (finds, insert-or-increments, erases), reading
// keys and writing results directly in pinned host memory, and reports each
// completed request (with its table's exact counts) in another host ring.
constexpr uint32_t kPersistRing = 256;

struct alignas(64) PersistCtl {   // host memory, written by the host
  unsigned long long posted;      // requests posted so far
  unsigned long long stop;        // 1: every wave exits after its current round
  unsigned long long base;        // the oldest request not complete, set before each launch
  unsigned long long pad[5];
};

// A request's phases in the resident kernel: copy its keys and kinds from the
// caller's pinned host arrays into device staging, finds, insert-or-increments,
// erases, copy the values and flags back.  Rounds of the copy phases cover
// kCopyRound operations, the others kRound.
constexpr uint32_t kPersistPhases = 5;
constexpr uint32_t kCopyRound = 1024;

struct alignas(64) PersistReq {   // host memory, one per ring entry
  BulkArgs a;                     // table fields; keys, kinds, vals_out, flags: the device staging
  const void *hkeys;              // the caller's pinned host arrays
  const uint8_t *hkinds;
  void *hvals;                    // may be null
  uint8_t *hflags;                // may be null
  unsigned long long rounds[kPersistPhases];  // rounds per phase (0 for a phase without operations)
  // A migration entry (mig_cells non-null) moves the table a.cells of 2^a.log2c
  // cells into mig_cells of 2^mig_log2c cells (twice as many): its phase-0
  // rounds are blocks of kPersistMigBlock old cells (Sec. 5.3.1, Lemma 1),
  // its one copy-out round only completes it; a.n is 0 and there are no
  // host arrays.
  void *mig_cells;
  unsigned long long mig_log2c;
  unsigned long long seq;         // q + 1 once the entry holds request q (written last)
};
constexpr uint32_t kPersistMigBlock = 256;

struct alignas(64) PersistDone {  // host memory, written by the device
  unsigned long long seq;         // q + 1 when request q has completed (written last)
  unsigned long long used, live, err;
  unsigned long long pad[4];
};

struct alignas(128) PersistDev {  // device memory, one per ring entry
  unsigned long long claim;       // (generation << 32) | rounds claimed; generation = q + 1
  unsigned long long done[kPersistPhases];  // (generation << 32) | rounds finished, per phase
  unsigned long long pad[10];
};

// Serving wavefronts are split into kPersistGroups groups by workgroup index
// (consecutive workgroups go to different XCDs, so a group is one XCD's
// share); group g serves the requests q with q % kPersistGroups == g and
// polls its own copy of the control words.
constexpr uint32_t kPersistGroups = 8;

struct alignas(128) PersistGroupCtl {
  unsigned long long posted;      // requests whose descriptors are in the device ring
  unsigned long long stop;        // the host's stop flag, mirrored by the poller
  unsigned long long pad[14];
};

struct alignas(128) PersistState { // device memory
  unsigned long long error;       // nonzero: a wait exceeded its bound (a bug, reported)
  unsigned long long alive;       // serving wavefronts still running
  unsigned long long published;   // ctl->posted as last copied by the poller
  unsigned long long completed;   // requests completed
  unsigned long long base;        // this launch's first request (ctl->base, copied at arming)
  unsigned long long pad[11];
  PersistGroupCtl group[kPersistGroups];
};

// Synthetic distinct keys for timing runs (layout 0: u32, 1: u64).
hipError_t launch_gen_keys(void *out, uint64_t n, uint32_t layout, uint64_t seed, hipStream_t s);

// Arms the device ring for requests first_q .. first_q + kPersistRing - 1.
hipError_t launch_persist_init(PersistDev *dev, PersistState *st, uint64_t first_q, hipStream_t s);
// The resident kernel, after a one-wave kernel that arms st (stop flags
// cleared, serving wavefronts counted, ctl->base copied): wavefronts serve
// requests from ctl->base on until ctl->stop is set, or until one of them has
// found no work for `idle_ticks` ticks of the device's constant-rate clock
// while every published request has completed.  `ring` is the host ring,
// `dring` its device copy.  `grid` must be a positive multiple of
// kPersistGroups.  The two launches take no per-launch argument, so the pair
// can be captured once in a graph and replayed.
hipError_t launch_persist(uint32_t layout, const PersistCtl *ctl, const PersistReq *ring, PersistReq *dring,
                          PersistDone *done, PersistDev *dev, PersistState *st, uint64_t idle_ticks,
                          uint32_t grid, hipStream_t s);

}  // namespace lpht
