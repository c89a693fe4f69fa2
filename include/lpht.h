/*
 * lpht: lock-free linear-probing hash tables on AMD MI355X (gfx950).
 *
 * C ABI of the device library liblpht.so.  Every operation of the table runs
 * in hand-written HIP kernels; this header exposes plain pointers and sizes
 * only.  The method is the bounded "folklore" table of Maier, Sanders and
 * Dementiev, "Concurrent Hash Tables: Fast and General(?)!" (arXiv 1601.04017),
 * Sec. 4 and Algorithm 1, with tombstone deletion (Sec. 5.4), growth by
 * block-parallel cluster migration into a table of double size (Sec. 5.3.1,
 * Lemma 1), shrinking by two-phase migration (Sec. 5.3.1, "Shrinking"), bulk
 * insertion by pre-growing (Sec. 5.5) and the paper's hash function (two
 * CRC-32C with different seeds, Sec. 8.3).
 *
 * Conventions shared by all calls
 * -------------------------------
 * - Return value: LPHT_OK (0) or a negative LPHT_ERR_* code.  No call throws
 *   or aborts across this boundary.
 * - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *   Calls are stream-ordered: a call returns once its work is enqueued; device
 *   arrays passed in must stay valid until the stream has passed that work.
 *   A table must be used from one stream at a time.  Within one call the
 *   operations run concurrently; a call behaves as if its operations were
 *   applied one by one in some order (linearizability, Sec. 4).
 * - Keys and values: u32 for LPHT_PACKED32, u64 for LPHT_KV64.  Key 0 is
 *   empty_key and key 1 is del_key (the tombstone); both are reserved
 *   (Sec. 5.6).  An operation on a reserved key changes nothing, gets flag
 *   LPHT_FLAG_RESERVED and sets the sticky error LPHT_ERR_RESERVED_KEY.
 * - Device arrays (`keys`, `vals`, `flags`, `vals_out`, `found`) are owned by
 *   the caller and live in device memory of the table's GPU.  Key and value
 *   arrays must be aligned to their element size.  `flags`/`found` hold one
 *   byte per operation and may be NULL (not written).
 * - Per-operation flags: 1 = true, 0 = false, LPHT_FLAG_RESERVED (0xFE) for a
 *   reserved key, LPHT_FLAG_FULL (0xFF) when a bounded table had no empty cell
 *   left for an inserting operation (sticky error LPHT_ERR_FULL).
 * - The table's cells and its status block are owned by the library and
 *   allocated through the configured allocator (default: the library's own
 *   stream-ordered memory pool on the table's device, which keeps freed
 *   memory for reuse until the process ends).
 */
#ifndef LPHT_H
#define LPHT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define LPHT_OK 0
#define LPHT_ERR_INVALID (-1)      /* bad argument (NULL table, misaligned pointer, range) */
#define LPHT_ERR_OOM (-2)          /* allocation failed */
#define LPHT_ERR_FULL (-3)         /* sticky: an insertion found no empty cell */
#define LPHT_ERR_RESERVED_KEY (-4) /* sticky: an operation used key 0 or 1 */
#define LPHT_ERR_DEVICE (-5)       /* a HIP runtime call failed */
#define LPHT_ERR_UNSUPPORTED (-6)  /* valid request the library does not implement */

/* ---- per-operation flag bytes ---- */
#define LPHT_FLAG_FALSE 0
#define LPHT_FLAG_TRUE 1
#define LPHT_FLAG_RESERVED 0xFE
#define LPHT_FLAG_FULL 0xFF

/* ---- cell layouts ----
 * LPHT_PACKED32: one 8-byte word per cell, key in bits 0..31, value in bits
 *   32..63; the whole cell is claimed by one 64-bit CAS, so key and value are
 *   published together as with the paper's 2-word CAS (Sec. 4).
 * LPHT_KV64: 16-byte cell {u64 key at byte 0, u64 value at byte 8}, 16-byte
 *   aligned.  gfx950 has no 128-bit CAS: the key is claimed with a 64-bit CAS
 *   and the value is then written by a separate store (the paper's fallback
 *   "variant which does not use 2-word CAS", Sec. 4).  Therefore finds must
 *   not run concurrently with modifications of the same table, which the
 *   per-table stream order guarantees. */
#define LPHT_PACKED32 0u
#define LPHT_KV64 1u

/* ---- update functions `up` of Algorithm 1 ----
 * LPHT_ASSIGN: value := d (overwrite by a single store, Sec. 4).
 * LPHT_ADD:    value := value + d modulo 2^32 (PACKED32) or 2^64 (KV64),
 *              by fetch-and-add (Sec. 4). */
#define LPHT_ASSIGN 0u
#define LPHT_ADD 1u

/* ---- hash functions (lpht_config.hash) ----
 * LPHT_HASH_CRC32C_PAIR: h(x) = CRC(seed_hi, x) * 2^32 + CRC(seed_lo, x), the
 *   CRC-32C register update over the key's 4 (PACKED32) or 8 (KV64)
 *   little-endian bytes, as the paper computes it with two crc32 instructions
 *   (Sec. 8.3).
 * LPHT_HASH_MULSHIFT: h(x) = (mul * x) mod 2^64 with an odd `mul`
 *   (multiplicative hashing); a bijection of the 64-bit keys, one multiply per
 *   operation.  Not available for string tables. */
#define LPHT_HASH_CRC32C_PAIR 0u
#define LPHT_HASH_MULSHIFT 1u

/* Allocator hook: returns device memory of `bytes` bytes (256-byte aligned)
 * usable in stream order on `stream`, or NULL.  `free` releases it in stream
 * order.  Both NULL selects the library's pool (hipMallocFromPoolAsync /
 * hipFreeAsync on a per-device pool that never releases memory). */
typedef void *(*lpht_alloc_fn)(size_t bytes, void *stream, void *ctx);
typedef void (*lpht_free_fn)(void *ptr, size_t bytes, void *stream, void *ctx);

typedef struct lpht_config {
  uint32_t layout;        /* LPHT_PACKED32 or LPHT_KV64 */
  uint32_t log2_capacity; /* capacity c = 2^log2_capacity cells, 6..34 (Sec. 7: powers of two) */
  uint32_t seed_hi;       /* CRC-32C seed of the upper 32 hash bits (Sec. 8.3) */
  uint32_t seed_lo;       /* CRC-32C seed of the lower 32 hash bits */
  uint32_t max_fill_num;  /* growth trigger alpha = num/den, 0 < alpha <= 1 (Sec. 5.3.2) */
  uint32_t max_fill_den;
  uint32_t auto_grow;     /* 0: bounded folklore table; 1: migrate before batches (Sec. 5.5):
                           * with b the operations of a call that may insert,
                           * used + b > alpha*c triggers a migration (Sec. 5.4:
                           * triggered by non-empty cells, sized by live ones);
                           * if live + b <= alpha*c/2 it is a cleanup into the
                           * smallest c' >= the created capacity with
                           * live + b <= alpha*c'/2 (c' = c drops tombstones,
                           * c' < c shrinks), else the table doubles until
                           * live + b <= alpha*c */
  uint32_t full_keys;     /* 0: keys 0 and 1 are reserved; 1: full key space (Sec. 5.6): keys 0
                           * and 1 are stored in two special slots of the table object; the
                           * batch and serving APIs do not take such tables */
  uint32_t hash;          /* LPHT_HASH_CRC32C_PAIR (default): the paper's two CRC-32C with
                           * seed_hi / seed_lo (Sec. 8.3); LPHT_HASH_MULSHIFT: h(x) = mul * x
                           * mod 2^64.  Either way the position is the top log2 c bits of h
                           * (the scaling map of Sec. 5.3.1), so migration works unchanged */
  uint32_t reserved0;     /* must be 0 */
  uint64_t mul;           /* LPHT_HASH_MULSHIFT: the multiplier, odd; ignored otherwise */
  lpht_alloc_fn alloc;
  lpht_free_fn free;
  void *alloc_ctx;
} lpht_config;

/* Launch parameters of the kernels; see lpht_set_tuning. */
typedef struct lpht_tuning {
  uint32_t block_threads; /* workgroup size, a multiple of 64 in 64..1024 */
  uint32_t group_width;   /* lanes that probe one operation together: 1, 2, 4, 8 or 16 */
  uint32_t blocks_per_cu; /* resident workgroups per compute unit the grid is sized for, 1..32 */
  uint32_t migrate_block; /* old cells per migration workgroup, power of two 256..8192 */
  uint32_t aggregate;     /* LPHT_ADD upserts: 1 (default): combine equal keys in LDS; calls of
                           * at least 2^22 operations on tables of at least 2^20 cells are first
                           * partitioned by table region (top 12 hash bits), so that every
                           * occurrence of a key is combined and each distinct key costs one
                           * upsert (scratch: about (key width [+ value width] [+ 4 with flags])
                           * bytes per operation, from the table's allocator); 2: LDS combining
                           * of 2048-operation chunks only; 0: no combining */
  /* Group width by fill quarter, used / capacity in [0, 1/4], (1/4, 1/2],
   * (1/2, 3/4], (3/4, 1] (the host's bound on `used` after the operations):
   * for finds, and for the operations that modify the table.  0 =
   * group_width.  Long probe runs at high fill are scanned faster by wider
   * groups.  An inserting call whose operations cross a quarter boundary
   * where the width changes is launched in pieces split there (pieces of at
   * least 2^16 operations). */
  uint8_t g_find[4];
  uint8_t g_modify[4];
  uint32_t reserved;      /* must be 0 */
} lpht_tuning;

typedef struct lpht_stats {
  uint64_t migrations;     /* migrations that moved data (empty-table resizes excluded) */
  uint64_t resizes;        /* all capacity changes and gamma = 1 cleanups */
  uint64_t cells_migrated; /* sum of old capacities over data migrations */
  uint64_t host_syncs;     /* count synchronisations the growth rule needed */
  double migrate_ms;       /* device time of data migrations (when timing is on) */
  uint64_t shrinks;        /* data migrations to a smaller capacity */
  uint64_t bulk_merges;    /* completed lpht_build / lpht_merge calls */
  uint64_t async_growths;  /* migrations made inside lpht_insert_async kernels */
  uint64_t async_fallbacks; /* of those, migrations that met a cluster longer than the block
                             * migration's halo and re-inserted by compare-and-swap instead */
} lpht_stats;

typedef struct lpht_table lpht_table; /* opaque; owned by the library */

/* Fills `cfg` with: KV64, log2_capacity 12, the CRC-32C pair hash with seeds
 * 0x9E3779B9 / 0xFFFFFFFF, alpha = 1/2, auto_grow 0, default allocator. */
void lpht_config_default(lpht_config *cfg);

/* Creates an empty table on the current HIP device: every cell is set to
 * empty_key with value 0 (Sec. 4, "Initialization").  Errors: INVALID (a
 * field out of range, an unknown hash, an even MULSHIFT multiplier, reserved0
 * not 0), OOM, DEVICE.  On error *out is NULL. */
int lpht_create(const lpht_config *cfg, void *stream, lpht_table **out);

/* Empties the table in place: every cell becomes empty_key with value 0,
 * counts and sticky errors are reset, the capacity stays. */
int lpht_clear(lpht_table *t, void *stream);

/* Releases the table's memory in stream order on `stream` and frees the
 * handle.  NULL is accepted. */
int lpht_destroy(lpht_table *t, void *stream);

/* insert(k, d) (Sec. 4): flag true iff k was absent and is now stored with
 * value d; if several operations of the call carry the same absent key exactly
 * one of them succeeds and the stored value is the value of that operation.
 * `vals` NULL means every value is 1.  With auto_grow the table first grows so
 * that used + n <= alpha * c (bulk pre-growth, Sec. 5.5). */
int lpht_insert(lpht_table *t, const void *keys, const void *vals, uint64_t n, uint8_t *flags,
                void *stream);

/* find(k) (Sec. 4): found[i] = 1 and vals_out[i] = stored value, or found[i]
 * = 0 and vals_out[i] = 0.  Never writes the table.  `vals_out` may be NULL. */
int lpht_find(lpht_table *t, const void *keys, uint64_t n, void *vals_out, uint8_t *found,
              void *stream);

/* insertOrUpdate(k, d, up) (Algorithm 1): inserts (k, d) if k is absent
 * (flag true), else value := up(value, d) (flag false).  With LPHT_ADD the
 * result is exact whatever the order; with LPHT_ASSIGN and repeated keys in
 * one call the final value is the `d` of one of that key's operations.
 * `vals` NULL means d = 1 (insert-or-increment).  Grows like lpht_insert. */
int lpht_insert_or_update(lpht_table *t, const void *keys, const void *vals, uint64_t n,
                          uint32_t op, uint8_t *inserted, void *stream);

/* update(k, d, up) (Sec. 4): flag false if k is absent, else value :=
 * up(value, d) and flag true.  Never inserts, never grows. */
int lpht_update(lpht_table *t, const void *keys, const void *vals, uint64_t n, uint32_t op,
                uint8_t *flags, void *stream);

/* Deletion by tombstone (Sec. 4 and 5.4): a live key k becomes del_key (its
 * value stays, the cell is never reused); flag true iff this operation did
 * it.  Tombstones are removed only by migration. */
int lpht_erase(lpht_table *t, const void *keys, uint64_t n, uint8_t *flags, void *stream);

/* Migrates the table into a new table of 2^log2_new_capacity cells, 6..34.
 * Growing or equal sizes (gamma = 2^(log2_new - log2_old) >= 1; equal sizes
 * drop tombstones, Sec. 5.4): block-parallel cluster migration (Sec. 5.3.1);
 * the placement equals the sequential migration's exactly (Lemma 1).
 * Smaller sizes: two-phase shrinking migration (Sec. 5.3.1, "Shrinking"):
 * source blocks are placed into disjoint target blocks, then the elements
 * that did not fit are inserted concurrently; the occupied cells and each
 * cluster's key set equal the sequential migration's, the order of keys
 * inside a cluster may differ.  Errors: INVALID (range), FULL (the live
 * elements would not leave an empty cell in the smaller table; the table is
 * unchanged), OOM. */
int lpht_grow(lpht_table *t, uint32_t log2_new_capacity, void *stream);

/* Insertion that grows the table while the kernel runs (Sec. 5.3.2, the
 * (semi-)synchronized protocol, with the approximate size of Sec. 5.2): one
 * cooperative launch inserts the n keys (add = 0: insert; of equal absent
 * keys exactly one operation inserts, flag 1, and the stored value is its
 * value, the others get 0 like operations on present keys; add = 1:
 * insert-or-add, the value gets the sum of all values (vals NULL: 1 each),
 * exact).  Wavefronts keep local counts of successful insertions and add them
 * to a global counter after a random number (1..64 r, r = rounds of 64
 * operations per chunk, 1..64 growing with the table) of them; when
 * that counter reaches alpha * capacity all wavefronts stop taking work,
 * migrate the table together into one of twice the size, and go on.  The
 * capacity therefore follows the number of distinct keys actually inserted,
 * not the batch length (insert-or-add over repeated keys needs far fewer
 * cells than pre-growth by n would reserve).  The host first grows the table,
 * if needed, to a minimum that leaves room for the work in flight
 * (device-dependent, about 2^21 cells) and below alpha * capacity, and
 * reserves tables of 2, 4, ... times the capacity up to the one that holds
 * used + n (unused ones are released afterwards).  Counts are exact after
 * the call.  Reserved keys get flag LPHT_FLAG_RESERVED.  Synchronises the
 * stream.  Errors: INVALID, UNSUPPORTED (no cooperative launch, alpha = 1, or
 * more than 16 doublings), OOM, DEVICE (a wait inside the kernel exceeded its
 * two-second bound). */
int lpht_insert_async(lpht_table *t, const void *keys, const void *vals, uint64_t n, uint32_t add,
                      uint8_t *flags, void *stream);

/* Sort-based bulk build (Sec. 5.5): replaces the table's contents by the n
 * elements of the batch (keys, and vals or NULL meaning every value is 1).
 * The elements are ordered by hash value (ties by key, then by index); among
 * equal keys only the last is kept, with LPHT_ASSIGN carrying its own value
 * and with LPHT_ADD the wrapping sum of all their values; the result is laid
 * out as if inserted one by one in that order into an empty table, so the
 * cells are a function of the set of (key, value) pairs alone.  Capacity:
 * unchanged for a bounded table; with auto_grow doubled while
 * n > alpha * capacity (never shrunk).  Reserved keys are skipped and set the
 * sticky RESERVED_KEY error.  Errors: INVALID (arguments, op), FULL (more
 * distinct keys than cells; the table and its counts are unchanged, sticky
 * FULL set), UNSUPPORTED (n + live >= 2^32 or a target above 2^29 cells),
 * OOM.  Synchronises the stream (the distinct count is read back).  Scratch:
 * about 2 x (live + n) x (2 x key width + 4) bytes for the call. */
int lpht_build(lpht_table *t, const void *keys, const void *vals, uint64_t n, uint32_t op, void *stream);

/* lpht_build for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same result, flags and errors as lpht_build, but no hipMalloc, hipFree or
 * pool allocation.  The build's scratch is a fixed 64 MiB device array of
 * the library (one per GPU, held until the process ends), and the result is
 * written into the table's current cell array, so the capacity never
 * changes: an auto-growing table that would have to grow (n > alpha *
 * capacity) gets UNSUPPORTED.  Limits: the scratch the build needs for n
 * keys at the table's capacity must fit 64 MiB (about (2 x key width + 4) x
 * 2n bytes plus per-block counters: 2^20 keys into up to 2^26 cells, either
 * layout); larger calls get LPHT_ERR_INVALID and change nothing.  All calls
 * on one GPU share the array, which keeps the last call's contents (each
 * call clears what it counts with): calls that overlap on one GPU race and
 * must be ordered by the caller (one stream, or events).  On FULL the table
 * is unchanged; after a device error its contents are undefined.
 * Synchronises the stream (the distinct count is read back). */
int lpht_build_noalloc(lpht_table *t, const void *keys, const void *vals, uint64_t n, uint32_t op,
                       void *stream);

/* Sort-based batched merge (Sec. 5.5): as lpht_build over the table's live
 * elements followed by the batch, i.e. the batch applied to the table with
 * insertOrUpdate semantics in index order (LPHT_ASSIGN: the last occurrence
 * of a key wins, over the table too; LPHT_ADD: the table's value plus all the
 * batch's values of that key), tombstones dropped, cells in the canonical
 * hash order.  Capacity: with auto_grow doubled while live + n > alpha *
 * capacity.  Errors and synchronisation as lpht_build. */
int lpht_merge(lpht_table *t, const void *keys, const void *vals, uint64_t n, uint32_t op, void *stream);

/* Size (Sec. 4, "Size"; the counters of Sec. 5.2): `used` = non-empty cells
 * (live keys and tombstones, the quantity the growth trigger of Sec. 5.4
 * watches), `live` = live keys (the table's size).  Exact: every kernel adds
 * its per-wavefront deltas before it ends, so at a call boundary the counts
 * equal a sequential table's.  Synchronises `stream`.  Either pointer may be
 * NULL.  Errors: INVALID (NULL table), DEVICE. */
int lpht_count(lpht_table *t, uint64_t *used, uint64_t *live, void *stream);

/* Capacity (Sec. 7: capacities are powers of two, so the scaling map of
 * Sec. 5.3.1 is a shift): `cells` = 2^log2_capacity cells, as created or as
 * left by the last migration; either pointer may be NULL.  Host-side, no
 * synchronisation (migrations are decided on the host, so the host always
 * knows the capacity).  Errors: INVALID (NULL table). */
int lpht_capacity(const lpht_table *t, uint64_t *cells, uint32_t *log2_capacity);

/* Bytes of one cell: 8 (PACKED32) or 16 (KV64). */
uint32_t lpht_cell_bytes(uint32_t layout);

/* Copies the raw cell array (capacity * cell bytes) to device memory `dst`. */
int lpht_export_cells(lpht_table *t, void *dst_device, void *stream);

/* Replaces the table's cells by a copy of `src_device` holding
 * 2^log2_capacity cells of the table's layout, and recounts used/live on the
 * device.  Used to hand the migration a given array in tests. */
int lpht_import_cells(lpht_table *t, const void *src_device, uint32_t log2_capacity, void *stream);

/* Returns the sticky device error (LPHT_ERR_FULL before
 * LPHT_ERR_RESERVED_KEY, else LPHT_OK) and clears it.  Synchronises `stream`. */
int lpht_status(lpht_table *t, void *stream);

/* Kernel launch parameters for this table.  Values are checked; INVALID
 * leaves the previous tuning in place.  `lpht_get_tuning` reads them back. */
int lpht_set_tuning(lpht_table *t, const lpht_tuning *tuning);
int lpht_get_tuning(const lpht_table *t, lpht_tuning *tuning);

/* Autotuning.  Times candidate launch shapes on scratch tables of
 * 2^log2_capacity cells of `layout` (auto_grow off), filled with synthetic
 * distinct keys generated on the device, and returns in `out` the fastest:
 *   - per fill quarter (fill 1/8, 3/8, 5/8, 7/8): the group width for finds
 *     (half present keys, spread evenly over the insertion order, half
 *     absent keys, a quarter of the capacity) and for
 *     inserts (the last capacity/16 keys before that fill), each over
 *     {1, 2, 4, 8, 16} -> g_find, g_modify; a quarter's choice is the
 *     narrowest width within 3 % of its fastest, and a quarter keeps the
 *     fill-3/8 choice unless another width is more than 3 % faster;
 *     group_width = the fill-3/8 finds' choice;
 *   - block_threads over {256, 512, 1024} at fill 3/8 with those widths;
 *   - migrate_block over {256, 512, 1024, 2048}: doubling a table at fill 7/16
 *     (lpht_grow);
 *   - blocks_per_cu 8 and aggregate 1 as the defaults.
 * Each candidate is the fastest of `reps` (>= 1) timed runs (HIP events on
 * `stream`), each from a table rebuilt to the same state.  Needs about
 * (cell bytes + 1.5 * key bytes + 1) * 2^log2_capacity + 2 * (cell bytes) *
 * 2^log2_capacity bytes of device memory, all freed before it returns;
 * log2_capacity 16..30.  `report` (may be NULL) receives the timings (ms). */
typedef struct lpht_autotune_report {
  double find_ms[4][5];   /* [fill quarter][group width 1, 2, 4, 8, 16] */
  double insert_ms[4][5];
  double block_ms[3];     /* block_threads 256, 512, 1024 */
  double migrate_ms[4];   /* migrate_block 256, 512, 1024, 2048 */
} lpht_autotune_report;
int lpht_autotune(uint32_t layout, uint32_t log2_capacity, uint32_t reps, void *stream, lpht_tuning *out,
                  lpht_autotune_report *report);

/* Migration statistics.  With `timing` = 1 every data migration is bracketed
 * by HIP events on its stream and migrate_ms accumulates their elapsed time
 * (read at the next lpht_get_stats, which then synchronises). */
int lpht_set_timing(lpht_table *t, int timing);
int lpht_get_stats(lpht_table *t, lpht_stats *stats);

/* ---- batches: many tables and calls in few launches ----
 *
 * A batch is a list of bulk calls (descriptors), possibly on different tables
 * and of uneven lengths.  Descriptors are grouped by operation and update
 * function; the groups run in the phase order FIND, INSERT, UPSERT, UPDATE,
 * ERASE, each group as one kernel launch per cell layout in which the
 * descriptors' 128-operation rounds are dealt to the wavefronts of one grid
 * (the paper deals blocks of operations to threads, Sec. 8.3).  Descriptors of
 * one group that name the same table behave like one bulk call on it.  Before
 * an INSERT or UPSERT group, every auto-growing table of the group grows for
 * the sum of its descriptors' lengths (Sec. 5.5).  Launch parameters are those
 * of the group's first table.
 *
 * `kinds` (optional, device, n bytes): when set, the descriptor performs only
 * the operations i with kinds[i] == kind_sel and leaves the other flag bytes
 * unchanged; a FIND descriptor writes value 0 for the other operations.  This
 * runs a mixed request in phase order with one descriptor per phase. */
#define LPHT_OP_FIND 0u
#define LPHT_OP_INSERT 1u
#define LPHT_OP_UPSERT 2u
#define LPHT_OP_UPDATE 3u
#define LPHT_OP_ERASE 4u

typedef struct lpht_batch_op {
  lpht_table *table;
  uint32_t op;           /* LPHT_OP_* */
  uint32_t up;           /* LPHT_ASSIGN or LPHT_ADD (UPSERT, UPDATE) */
  const void *keys;      /* device, n keys */
  const void *vals;      /* device, n values, or NULL (value 1) */
  uint64_t n;
  void *vals_out;        /* FIND: device, n values, or NULL */
  uint8_t *flags;        /* device, n flag bytes, or NULL */
  const uint8_t *kinds;  /* device, n bytes, or NULL */
  uint32_t kind_sel;
  uint32_t count_sel;    /* with kinds: number of operations of kind kind_sel (the growth
                            rule's b); a descriptor with kinds and count_sel 0 is skipped */
} lpht_batch_op;

typedef struct lpht_batch lpht_batch; /* descriptor staging ring; owned by the caller */

/* Creates a batch context for up to `max_ops` descriptors per call on the
 * current device (pinned and device staging buffers, reused in stream order). */
int lpht_batch_create(uint32_t max_ops, lpht_batch **out);
int lpht_batch_destroy(lpht_batch *b);

/* Runs `nops` descriptors in stream order on `stream`.  Errors: INVALID
 * (NULL or foreign table, mixed devices, nops > max_ops, misaligned arrays),
 * OOM (growth), DEVICE. */
int lpht_batch_run(lpht_batch *b, const lpht_batch_op *ops, uint32_t nops, void *stream);

/* ---- serving: a request loop over resident tables ----
 *
 * A server owns `ntables` tables kept on the device and a worker thread.
 * Clients submit requests (from any thread); each request is a mixed batch of
 * operations on one table, run in phase order: all finds (they see the table
 * as it was when the request started), then all insert-or-increments (+1),
 * then all erases.  The worker admits requests while request slots and the
 * HBM budget allow, keeping per-table FIFO order (a table serves one request
 * at a time; requests for other tables proceed meanwhile), and launches the
 * admitted requests together:
 *   LPHT_SERVE_WAVES  - continuous batching: all requests admitted at the same
 *                       time form one wave, run as one multi-table launch per
 *                       phase (lpht_batch_run); new requests are admitted and
 *                       launched on another stream while earlier waves run;
 *   LPHT_SERVE_SINGLE - the plain form: every request gets its own launches;
 *   LPHT_SERVE_PERSISTENT - one resident kernel serves all requests: the
 *                       worker posts each admitted request into a ring in
 *                       pinned host memory; the kernel's wavefronts copy its
 *                       keys and kinds into a device staging arena, run its
 *                       128-operation rounds phase by phase, copy values and
 *                       flags back into the request's host arrays, and
 *                       publish the completion in host memory.  No HIP call
 *                       is made per request.  The kernel's launch is captured
 *                       once as a HIP graph and replayed: it exits when idle
 *                       and is relaunched on new work.  Growth happens inside
 *                       it (hiding the migration, Sec. 5.3.2): when the
 *                       growth rule asks for one doubling of a table of at
 *                       least 2^10 cells, the worker posts a migration entry,
 *                       whose rounds are blocks of the block-parallel cluster
 *                       migration (Sec. 5.3.1) that the serving wavefronts
 *                       run while requests on other tables go on; the
 *                       waiting request is posted once the table has its new
 *                       cells.  Other growth (several doublings, cleanups,
 *                       shrinks, small or empty tables) and a migration that
 *                       meets a cluster longer than its halo stop the
 *                       kernel, migrate on the host and relaunch it.
 *                       Request arrays must be pinned host memory (or device
 *                       memory); submit rejects others with
 *                       LPHT_ERR_INVALID.
 * Every mode stages a request's keys, kinds, values and flags in a device
 * arena the server allocates once: 1 GiB, or what hbm_budget leaves beside the
 * initial tables (at least 1 MiB).  A request needs about (2 * key bytes + 2)
 * * n bytes of it while in flight; the budget counts tables, the staging in
 * use and the memory a request's growth would allocate.  A request that could
 * never be admitted (larger than the arena or the budget with nothing in
 * flight) completes with LPHT_ERR_OOM.
 * Tables grow before a request's increments by the growth rule (bulk
 * pre-growth, Sec. 5.5), which also removes tombstones (Sec. 5.4); the counts
 * the rule needs are read back after every request without synchronising.
 * Host buffers of a request should be pinned (hipHostMalloc); they must stay
 * valid until the request completes. */
#define LPHT_SERVE_WAVES 0u
#define LPHT_SERVE_SINGLE 1u
#define LPHT_SERVE_PERSISTENT 2u

#define LPHT_KIND_FIND 0u
#define LPHT_KIND_INCREMENT 1u
#define LPHT_KIND_ERASE 2u

typedef struct lpht_server_config {
  uint32_t ntables;
  uint32_t layout;                 /* LPHT_KV64 or LPHT_PACKED32 */
  const uint32_t *log2_capacity;   /* host, ntables initial capacities (auto-growing tables) */
  uint32_t mode;                   /* LPHT_SERVE_WAVES, _SINGLE or _PERSISTENT */
  uint32_t max_inflight;           /* request slots, 1..4096 */
  uint32_t streams;                /* device streams for launches, 1..8 */
  uint32_t reserved;               /* must be 0 */
  uint64_t hbm_budget;             /* bytes for tables, staging in use and growth; 0 = no limit */
} lpht_server_config;

typedef struct lpht_request {
  uint32_t table;        /* 0..ntables-1 */
  uint32_t reserved;     /* must be 0 */
  uint64_t n;            /* operations, 1..2^31 */
  const void *keys;      /* host, n keys */
  const uint8_t *kinds;  /* host, n LPHT_KIND_* bytes */
  void *vals_out;        /* host, n values: the found value for finds, else 0; may be NULL */
  uint8_t *flags;        /* host, n flags (find: found; increment: inserted; erase: erased) */
} lpht_request;

typedef struct lpht_completion {
  uint64_t ticket;
  int status;            /* LPHT_OK, or LPHT_ERR_OOM when the request can never fit the budget */
  uint32_t wave;         /* sequence number of the launch group that ran it */
  double submit_us;      /* host steady clock, microseconds */
  double admit_us;
  double done_us;
} lpht_completion;

typedef struct lpht_server_stats {
  uint64_t completed;
  uint64_t waves;
  uint64_t launches_phases;  /* phase launch groups issued */
  uint64_t peak_hbm_bytes;   /* peak of tables + staging as accounted by admission */
  uint64_t admission_waits;  /* times the head request waited for budget */
  double busy_us;            /* time with at least one request on the device */
  uint64_t kernel_growths;   /* resident mode: doublings migrated by the running kernel */
  uint64_t kernel_growth_fallbacks; /* of those, moves redone by the host (a cluster longer
                                     * than the migration's halo) */
} lpht_server_stats;

typedef struct lpht_server lpht_server;

int lpht_server_create(const lpht_server_config *cfg, lpht_server **out);
/* Thread-safe, non-blocking.  Errors: INVALID. */
int lpht_server_submit(lpht_server *srv, const lpht_request *req, uint64_t *ticket);
/* LPHT_OK and *out filled when the request is done (the record is then
 * released), 1 when it is still pending, INVALID for an unknown ticket. */
int lpht_server_poll(lpht_server *srv, uint64_t ticket, lpht_completion *out);
/* Blocks until the request is done. */
int lpht_server_wait(lpht_server *srv, uint64_t ticket, lpht_completion *out);
/* Blocks until every submitted request is done. */
int lpht_server_drain(lpht_server *srv);
/* The server's table `index` (use it only while the server is drained). */
int lpht_server_table(lpht_server *srv, uint32_t index, lpht_table **out);
int lpht_server_stats_get(lpht_server *srv, lpht_server_stats *out);
/* Drains, stops the worker and destroys the tables. */
int lpht_server_destroy(lpht_server *srv);

/* Closed-loop driver: `nclients` clients, each submitting its next request
 * when its previous one completes, walk through reqs[0..nreq) in order.
 * Writes each request's completion to done[i] (latency = done_us -
 * submit_us) and the wall time to *wall_us. */
int lpht_server_run_closed_loop(lpht_server *srv, const lpht_request *reqs, uint32_t nreq,
                                uint32_t nclients, lpht_completion *done, double *wall_us);

/* Static description of an error code. */
const char *lpht_strerror(int code);

/* Library version string. */
const char *lpht_version(void);

/* Orderly shutdown: waits for every device that has a library memory pool,
 * returns the pools' memory and destroys them, so that nothing of the
 * library is left for the HIP runtime's own teardown at process exit.  Call
 * it after every table, string table and server has been destroyed (their
 * memory comes from the pools); a table created afterwards makes a new pool.
 * Errors: INVALID (pool memory still in use: some object is alive; nothing is
 * released), DEVICE. */
int lpht_release_pools(void);

/* ---- string keys (Sec. 5.7, "Complex Keys") ----
 *
 * A table whose keys are byte strings (any length, the empty string
 * included) and whose values are u64.  The table manages a byte pool for the
 * keys: a cell holds a reference word, (signature << 48) | pool offset, and
 * the value; the signature is the low 16 bits of the key's 64-bit hash (bits
 * the position does not use), so a probe compares signatures before it
 * follows a reference.  The hash is the pair of CRC-32C register updates
 * over the key's bytes with the two seeds (Sec. 8.3) -- an 8-byte key hashes
 * like the same word in a KV64 table.  A batch of n keys is a byte array and
 * n + 1 u64 offsets (key i = bytes[offsets[i] .. offsets[i + 1])), both
 * device memory; offsets must be non-decreasing.  Within a call operations
 * run concurrently (as for word keys).  Erased keys' bytes stay in the pool
 * until a migration, which copies only live keys into a new pool; a
 * migration also happens when an inserting call might not fit the pool
 * (records take length + 4 bytes rounded up to 8).  Inserting calls read
 * offsets[0] and offsets[n] back (one synchronisation). */
typedef struct lpht_str_table lpht_str_table;

typedef struct lpht_str_config {
  uint32_t log2_capacity; /* 6..34 */
  uint32_t auto_grow;     /* the word tables' growth rule (including cleanup and shrink) */
  uint32_t seed_hi, seed_lo;
  uint32_t max_fill_num, max_fill_den;
  uint32_t reserved[2];   /* must be 0 */
  uint64_t pool_bytes;    /* initial key pool (>= 64) */
} lpht_str_config;

/* log2_capacity 12, seeds as lpht_config_default, alpha = 1/2, no growth,
 * a 1 MiB pool. */
void lpht_str_config_default(lpht_str_config *cfg);
int lpht_str_create(const lpht_str_config *cfg, void *stream, lpht_str_table **out);
int lpht_str_destroy(lpht_str_table *t, void *stream);
/* insert: flag 1 = inserted, 0 = present (its value unchanged), 0xFF = no
 * room (sticky FULL, lpht_str_status); vals may be NULL (1 each). */
int lpht_str_insert(lpht_str_table *t, const uint8_t *bytes, const uint64_t *offsets, uint64_t n,
                    const uint64_t *vals, uint8_t *flags, void *stream);
/* insertOrUpdate with up = LPHT_ASSIGN or LPHT_ADD (value + d mod 2^64). */
int lpht_str_insert_or_update(lpht_str_table *t, const uint8_t *bytes, const uint64_t *offsets, uint64_t n,
                              const uint64_t *vals, uint32_t up, uint8_t *flags, void *stream);
/* find: found[i] 1/0, vals_out[i] the value or 0 (either may be NULL). */
int lpht_str_find(lpht_str_table *t, const uint8_t *bytes, const uint64_t *offsets, uint64_t n,
                  uint64_t *vals_out, uint8_t *found, void *stream);
/* erase by tombstone: flag 1 for the operation that erased the key. */
int lpht_str_erase(lpht_str_table *t, const uint8_t *bytes, const uint64_t *offsets, uint64_t n, uint8_t *flags,
                   void *stream);
/* Exact counts (non-empty cells, live keys); synchronises. */
int lpht_str_count(lpht_str_table *t, uint64_t *used, uint64_t *live, void *stream);
int lpht_str_capacity(lpht_str_table *t, uint64_t *cells, uint64_t *pool_used, uint64_t *pool_cap, void *stream);
/* Migration into 2^log2 cells (larger, equal or smaller), compacting the
 * pool.  Errors: INVALID, FULL (live keys would not leave an empty cell). */
int lpht_str_grow(lpht_str_table *t, uint32_t log2_new_capacity, void *stream);
/* Copies the cells (16 bytes each) and up to pool_dst_bytes of the pool
 * (device destinations). */
int lpht_str_export(lpht_str_table *t, void *cells_dst, void *pool_dst, uint64_t pool_dst_bytes, void *stream);
/* Sticky error (LPHT_ERR_FULL after an insertion found no room), cleared. */
int lpht_str_status(lpht_str_table *t, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* LPHT_H */
