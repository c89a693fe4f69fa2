// Host side of liblpht: table objects, the growth rule, allocation and the C
// ABI declared in include/lpht.h.  Every table operation is executed by the
// HIP kernels of lpht_kernels.hip; this file only validates arguments, sizes
// launches and decides when to migrate.

#include <hip/hip_runtime.h>

#include <algorithm>

#include <atomic>
#include <mutex>
#include <new>
#include <vector>

#include "lpht_host.h"
#include "lpht_async.h"
#include "lpht_bulk.h"
#include "lpht_part.h"
#include "lpht_shrink.h"
#include "lpht_special.h"

using namespace lpht;

namespace {

// CRC-32C register update (reflected Castagnoli polynomial, no inversion)
// from register 0 over the `nbytes` little-endian bytes of `x`, bit by bit.
// Used once per table for the two hash constants CRC(0, seed).
uint32_t crc0_bytes(uint64_t x, int nbytes) {
  uint32_t r = 0;
  for (int i = 0; i < nbytes; ++i) {
    r ^= (uint32_t)((x >> (8 * i)) & 0xFFu);
    for (int b = 0; b < 8; ++b) r = (r >> 1) ^ (0x82F63B78u & (0u - (r & 1u)));
  }
  return r;
}



}  // namespace



namespace lpht {
namespace host {

int from_hip(hipError_t e) {
  if (e == hipSuccess) return LPHT_OK;
  if (e == hipErrorOutOfMemory) return LPHT_ERR_OOM;
  if (e == hipErrorInvalidValue) return LPHT_ERR_INVALID;
  return LPHT_ERR_DEVICE;
}

uint64_t cell_bytes(uint32_t layout) { return layout == LPHT_PACKED32 ? 8u : 16u; }

// The library's own stream-ordered memory pool per device.  It keeps freed
// memory mapped (release threshold: never), so that the repeated growth of
// a table reuses pages instead of mapping new ones; the paper uses a
// user-space memory pool for the same reason (Sec. 7).
constexpr int kMaxDevices = 64;
std::mutex g_pool_mu;
hipMemPool_t g_pools[kMaxDevices];
// blocks handed out by pool_alloc and not yet given back to pool_free
std::atomic<long long> g_pool_blocks{0};

// Frees the pool has not been told of yet.  A block freed on stream s is
// often still to be read by work queued on s (the old table of a migration
// just enqueued); handed to another stream's allocation at once, it was seen
// overwritten before that work ran, although the stream-ordered allocator
// should have kept it back.  So pool_free records an event on s and returns
// the block to the pool only once the event has completed; allocations and
// frees reap the completed ones.
struct PendingFree {
  void *p;
  hipEvent_t ev;
  int device;
};
std::mutex g_pending_mu;
std::vector<PendingFree> g_pending;
std::vector<hipEvent_t> g_spare_events;
// blocks whose event cannot be waited on: returned when the pools are released
std::vector<PendingFree> g_stuck;

// Returns to the pool every pending block of `device` whose event has
// completed (all of them, waiting, when `wait`), ordered on stream s.
void reap_pending(int device, hipStream_t s, bool wait) {
  std::lock_guard<std::mutex> lk(g_pending_mu);
  size_t k = 0;
  for (size_t i = 0; i < g_pending.size(); ++i) {
    PendingFree &f = g_pending[i];
    hipError_t q = hipErrorNotReady;
    if (f.device == device) q = wait ? hipEventSynchronize(f.ev) : hipEventQuery(f.ev);
    const bool done = q == hipSuccess;
    if (q != hipSuccess && q != hipErrorNotReady) {
      // The event cannot be waited on (HIP has reported events recorded into
      // a stream capture this way): the error is the pool's, not the
      // caller's, and the block stays out of the pool until the pools are
      // released after a device synchronisation.
      (void)hipGetLastError();
      g_stuck.push_back(f);
      continue;
    }
    if (done) {
      // a failed free leaves the block to the pool; its error is not the
      // caller's to read
      if (hipFreeAsync(f.p, s) != hipSuccess) (void)hipGetLastError();
      g_spare_events.push_back(f.ev);
    } else {
      g_pending[k++] = f;
    }
  }
  g_pending.resize(k);
}

hipMemPool_t device_pool(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_pool_mu);
  if (!g_pools[dev]) {
    hipMemPoolProps props{};
    props.allocType = hipMemAllocationTypePinned;
    props.handleTypes = hipMemHandleTypeNone;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = dev;
    hipMemPool_t pool = nullptr;
    if (hipMemPoolCreate(&pool, &props) != hipSuccess) return nullptr;
    uint64_t keep = ~0ull;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    g_pools[dev] = pool;
  }
  return g_pools[dev];
}

void *pool_alloc(int device, size_t bytes, hipStream_t s) {
  hipMemPool_t pool = device_pool(device);
  if (!pool) return nullptr;
  reap_pending(device, s, false);
  void *p = nullptr;
  if (hipMallocFromPoolAsync(&p, bytes, pool, s) != hipSuccess) return nullptr;
  g_pool_blocks.fetch_add(1);
  return p;
}

void pool_free(void *p, hipStream_t s) {
  if (!p) return;
  int device = 0;
  hipEvent_t ev = nullptr;
  bool queued = false;
  if (hipGetDevice(&device) == hipSuccess) {
    {
      std::lock_guard<std::mutex> lk(g_pending_mu);
      if (!g_spare_events.empty()) {
        ev = g_spare_events.back();
        g_spare_events.pop_back();
      }
    }
    if (ev || hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess) {
      if (hipEventRecord(ev, s) == hipSuccess) {
        std::lock_guard<std::mutex> lk(g_pending_mu);
        g_pending.push_back({p, ev, device});
        queued = true;
      } else {
        (void)hipGetLastError();  // handled below: the free waits for the stream instead
        (void)hipEventDestroy(ev);
      }
    }
  }
  if (!queued) {
    // no event: wait for the stream, then free
    if (hipStreamSynchronize(s) != hipSuccess) (void)hipGetLastError();
    if (hipFreeAsync(p, s) != hipSuccess) (void)hipGetLastError();
  }
  g_pool_blocks.fetch_sub(1);
  reap_pending(device, s, false);
}

int release_pools() {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  if (g_pool_blocks.load() != 0) return LPHT_ERR_INVALID;
  int cur = 0;
  bool have_cur = false;
  int rc = LPHT_OK;
  for (int d = 0; d < kMaxDevices; ++d) {
    if (!g_pools[d]) continue;
    if (!have_cur) {
      if (hipGetDevice(&cur) != hipSuccess) return LPHT_ERR_DEVICE;
      have_cur = true;
    }
    // the frees of destroyed tables complete in stream order: wait for them
    if (hipSetDevice(d) == hipSuccess) {
      reap_pending(d, nullptr, true);
      if (hipDeviceSynchronize() == hipSuccess) {
        std::lock_guard<std::mutex> lk(g_pending_mu);
        size_t k = 0;
        for (const PendingFree &f : g_stuck) {
          if (f.device == d) {
            if (hipFreeAsync(f.p, nullptr) != hipSuccess) (void)hipGetLastError();
            if (hipEventDestroy(f.ev) != hipSuccess) (void)hipGetLastError();
          } else {
            g_stuck[k++] = f;
          }
        }
        g_stuck.resize(k);
      }
    }
    if (hipSetDevice(d) != hipSuccess || hipDeviceSynchronize() != hipSuccess ||
        hipMemPoolTrimTo(g_pools[d], 0) != hipSuccess || hipMemPoolDestroy(g_pools[d]) != hipSuccess)
      rc = LPHT_ERR_DEVICE;
    g_pools[d] = nullptr;
  }
  {
    std::lock_guard<std::mutex> lk(g_pending_mu);
    for (hipEvent_t ev : g_spare_events) (void)hipEventDestroy(ev);
    g_spare_events.clear();
  }
  if (have_cur) (void)hipSetDevice(cur);
  return rc;
}

void *dev_alloc(lpht_table *t, size_t bytes, hipStream_t s) {
  if (t->cfg.alloc) return t->cfg.alloc(bytes, (void *)s, t->cfg.alloc_ctx);
  return pool_alloc(t->device, bytes, s);
}

void dev_free(lpht_table *t, void *p, size_t bytes, hipStream_t s) {
  if (!p) return;
  if (t->cfg.free) {
    t->cfg.free(p, bytes, (void *)s, t->cfg.alloc_ctx);
    return;
  }
  pool_free(p, s);
}

void fill_launch(lpht_table *t) {
  t->launch.block_threads = t->tuning.block_threads;
  t->launch.group_width = t->tuning.group_width;
  t->launch.blocks_per_cu = t->tuning.blocks_per_cu;
  t->launch.migrate_block = t->tuning.migrate_block;
  t->launch.aggregate = t->tuning.aggregate;
}

bool tuning_ok(const lpht_tuning *u) {
  if (u->block_threads < 64 || u->block_threads > 1024 || (u->block_threads % 64)) return false;
  switch (u->group_width) {
    case 1: case 2: case 4: case 8: case 16: break;
    default: return false;
  }
  if (u->blocks_per_cu < 1 || u->blocks_per_cu > 32) return false;
  if (u->migrate_block < 256 || u->migrate_block > 8192 ||
      (u->migrate_block & (u->migrate_block - 1)))
    return false;
  if (u->aggregate > 2) return false;
  for (int i = 0; i < 4; ++i)
    for (uint8_t g : {u->g_find[i], u->g_modify[i]})
      if (g != 0 && g != 1 && g != 2 && g != 4 && g != 8 && g != 16) return false;
  if (u->reserved) return false;
  return true;
}

// The group width for an operation on `t` when `used` is the host's bound on
// the table's non-empty cells after it: by the fill quarter (0, c/4],
// (c/4, c/2], (c/2, 3c/4], (3c/4, c] that holds `used`, else the default.
uint32_t pick_group_width(const lpht_table *t, OpKind op, uint64_t used) {
  const uint64_t c = 1ull << t->log2c;
  used = std::min<uint64_t>(c, used);
  const uint32_t qi = used == 0 ? 0 : (uint32_t)std::min<uint64_t>(3, (unsigned __int128)(used - 1) * 4 / c);
  const uint8_t g = op == OP_FIND ? t->tuning.g_find[qi] : t->tuning.g_modify[qi];
  return g ? g : t->tuning.group_width;
}

// Inserting calls with fill-dependent widths are launched in pieces that end
// at the fill-quarter boundaries the call may cross where the width changes
// (pieces of at least this many operations), each with its quarter's width.  Consecutive pieces
// are the call's operations in order, so the results are those of one launch.
constexpr uint64_t kMinPiece = 1ull << 16;

bool within_fill(const lpht_table *t, uint64_t x, uint64_t c) {
  return (unsigned __int128)x * t->cfg.max_fill_den <= (unsigned __int128)c * t->cfg.max_fill_num;
}

// Reads the status block (synchronises the stream) and the count totals.
int read_status(lpht_table *t, hipStream_t s, DevStatus *h, uint64_t *used, uint64_t *live) {
  hipError_t e = hipMemcpyAsync(h, t->status, sizeof(DevStatus), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return from_hip(e);
  uint64_t u = 0, l = 0;
  for (int i = 0; i < kCountSlots; ++i) {
    u += h->slot[i].used;
    l += h->slot[i].live;
  }
  *used = u;
  *live = l;
  return LPHT_OK;
}

int sync_counts(lpht_table *t, hipStream_t s) {
  DevStatus h;
  uint64_t u, l;
  int rc = read_status(t, s, &h, &u, &l);
  if (rc) return rc;
  t->known_used = u;
  t->known_live = l;
  t->pending = 0;
  t->mods_since_exact = 0;
  return LPHT_OK;
}

// Replaces the cells by an all-empty table of 2^log2_new cells; `steps` is
// the number of migrations of the growth rule this resize stands for.
int resize_empty(lpht_table *t, uint32_t log2_new, hipStream_t s, uint32_t steps) {
  const size_t nb = (size_t)cell_bytes(t->cfg.layout) << log2_new;
  void *nc = dev_alloc(t, nb, s);
  if (!nc) return LPHT_ERR_OOM;
  hipError_t e = launch_fill_zero(nc, nb, t->launch, s);
  if (e == hipSuccess) e = launch_set_status(t->status, 0, 0, 0, s);
  if (e != hipSuccess) {
    dev_free(t, nc, nb, s);
    return from_hip(e);
  }
  dev_free(t, t->cells, (size_t)cell_bytes(t->cfg.layout) << t->log2c, s);
  t->cells = nc;
  t->log2c = log2_new;
  t->known_used = t->known_live = 0;
  t->pending = 0;
  t->mods_since_exact = 0;
  t->stats.resizes += steps;
  return LPHT_OK;
}

// One migration into 2^log2_new cells.  The host must know the exact live
// count (`known_live`); afterwards used = live = that count.  A smaller
// target must have more cells than live elements (else LPHT_ERR_FULL, the
// table unchanged).
int migrate_once(lpht_table *t, uint32_t log2_new, hipStream_t s) {
  if (log2_new < t->log2c && t->known_live >= (1ull << log2_new)) return LPHT_ERR_FULL;
  if (t->known_live == 0) return resize_empty(t, log2_new, s);
  const size_t ob = (size_t)cell_bytes(t->cfg.layout) << t->log2c;
  const size_t nb = (size_t)cell_bytes(t->cfg.layout) << log2_new;
  void *nc = dev_alloc(t, nb, s);
  if (!nc) return LPHT_ERR_OOM;
  MigTiming tm{};
  if (t->timing) {
    if (hipEventCreate(&tm.start) != hipSuccess || hipEventCreate(&tm.stop) != hipSuccess)
      return LPHT_ERR_DEVICE;
    (void)hipEventRecord(tm.start, s);
  }
  const int old_full = (t->known_used == (1ull << t->log2c)) ? 1 : 0;
  const bool shrink = log2_new < t->log2c;
  const size_t sb = shrink ? shrink_scratch_bytes(t->log2c, log2_new) : 0;
  uint32_t *scratch = nullptr;
  if (sb && !(scratch = (uint32_t *)dev_alloc(t, sb, s))) {
    dev_free(t, nc, nb, s);
    return LPHT_ERR_OOM;
  }
  hipError_t e = launch_set_status(t->status, 0, 0, 0, s);
  if (e == hipSuccess && shrink)
    e = launch_shrink(t->cells, t->log2c, nc, log2_new, t->cfg.layout, t->crc_hi, t->crc_lo, t->mul, scratch,
                      t->status, t->launch, s);
  else if (e == hipSuccess)
    e = launch_migrate(t->cells, t->log2c, nc, log2_new, t->cfg.layout, t->crc_hi, t->crc_lo, t->mul,
                       old_full, t->status, t->launch, s);
  if (scratch) dev_free(t, scratch, sb, s);
  if (e != hipSuccess) {
    dev_free(t, nc, nb, s);
    return from_hip(e);
  }
  if (t->timing) {
    (void)hipEventRecord(tm.stop, s);
    t->timed.push_back(tm);
  }
  dev_free(t, t->cells, ob, s);
  t->stats.migrations++;
  t->stats.resizes++;
  if (shrink) t->stats.shrinks++;
  t->stats.cells_migrated += 1ull << t->log2c;
  t->cells = nc;
  t->log2c = log2_new;
  t->known_used = t->known_live;
  t->pending = 0;
  t->mods_since_exact = 0;
  return LPHT_OK;
}

// The growth rule before a batch of b operations that may insert (bulk
// insertion by pre-growing, Sec. 5.5; trigger at fill factor alpha and
// doubling, Sec. 5.3.2 and Sec. 7; the migration triggered by non-empty
// cells and sized by live elements, Sec. 5.4):
//   used + b <= alpha*c     -> nothing
//   live + b <= alpha*c/2   -> one migration into c' = c / 2^k, the largest
//                              k >= 0 with c' >= the created capacity and
//                              live + b <= alpha*c'/2 (k = 0 drops
//                              tombstones, k > 0 shrinks)
//   otherwise               -> migrate with gamma = 2, repeated while
//                              live + b > alpha*c.
// Decisions use exact counts.  The host keeps an upper bound of `used` and
// reads the device counters only when the bound does not already rule a
// migration out.
int grow_before_batch(lpht_table *t, uint64_t b, hipStream_t s) {
  if (b == 0) return LPHT_OK;
  if (!t->cfg.auto_grow) {
    t->pending += b;
    return LPHT_OK;
  }
  const uint64_t c = 1ull << t->log2c;
  if (within_fill(t, t->known_used + t->pending + b, c)) {
    t->pending += b;
    return LPHT_OK;
  }
  if (t->mods_since_exact != 0 || t->pending != 0) {
    int rc = sync_counts(t, s);
    if (rc) return rc;
    t->stats.host_syncs++;
  }
  int rc = LPHT_OK;
  if (within_fill(t, t->known_used + b, c)) {
    t->pending = b;
    return LPHT_OK;
  }
  if ((unsigned __int128)(t->known_live + b) * 2 * t->cfg.max_fill_den <=
      (unsigned __int128)c * t->cfg.max_fill_num) {
    // halve while live + b <= alpha * c_target / 4
    uint32_t target = t->log2c;
    while (target > t->log2_min && (unsigned __int128)(t->known_live + b) * 4 * t->cfg.max_fill_den <=
                                       ((unsigned __int128)1 << target) * t->cfg.max_fill_num)
      --target;
    rc = migrate_once(t, target, s);
  } else {
    uint32_t target = t->log2c;
    do {
      if (target >= 34) return LPHT_ERR_OOM;
      ++target;
    } while (!within_fill(t, t->known_live + b, 1ull << target));
    if (t->known_live == 0) {
      // migrations of an empty table are resizes; jump to the final size
      rc = resize_empty(t, target, s, target - t->log2c);
    } else {
      while (!rc && t->log2c < target) rc = migrate_once(t, t->log2c + 1, s);
    }
  }
  if (rc) return rc;
  t->pending = b;
  return LPHT_OK;
}

int growth_kind(const lpht_table *t, uint64_t b) {
  const uint64_t c = 1ull << t->log2c;
  if (b == 0 || !t->cfg.auto_grow || within_fill(t, t->known_used + b, c)) return 0;
  if ((unsigned __int128)(t->known_live + b) * 2 * t->cfg.max_fill_den <=
      (unsigned __int128)c * t->cfg.max_fill_num)
    return 2;  // cleanup or shrink
  if (t->known_live == 0 || t->log2c >= 34) return 2;
  return within_fill(t, t->known_live + b, 2 * c) ? 1 : 2;
}

BulkArgs make_args(lpht_table *t) {
  BulkArgs a{};
  a.cells = t->cells;
  a.log2c = t->log2c;
  a.layout = t->cfg.layout;
  a.crc_hi = t->crc_hi;
  a.crc_lo = t->crc_lo;
  a.mul = t->mul;
  a.status = t->status;
  return a;
}

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

int check_arrays(lpht_table *t, const void *keys, const void *vals, uint64_t n) {
  if (!t) return LPHT_ERR_INVALID;
  if (n && !keys) return LPHT_ERR_INVALID;
  const size_t w = t->cfg.layout == LPHT_PACKED32 ? 4 : 8;
  if (!aligned(keys, w) || !aligned(vals, w)) return LPHT_ERR_INVALID;
  return LPHT_OK;
}

int run_bulk(lpht_table *t, OpKind op, const void *keys, const void *vals, uint64_t n, uint32_t up,
             void *vals_out, uint8_t *flags, void *stream) {
  int rc = check_arrays(t, keys, vals, n);
  if (rc) return rc;
  if (up > LPHT_ADD) return LPHT_ERR_INVALID;
  if (vals_out && !aligned(vals_out, t->cfg.layout == LPHT_PACKED32 ? 4 : 8))
    return LPHT_ERR_INVALID;
  if (n == 0) return LPHT_OK;
  hipStream_t s = (hipStream_t)stream;
  if (hipSetDevice(t->device) != hipSuccess) return LPHT_ERR_DEVICE;
  if (op == OP_INSERT || op == OP_UPSERT) {
    rc = grow_before_batch(t, n, s);
    if (rc) return rc;
  }
  if (op != OP_FIND) t->mods_since_exact++;
  BulkArgs a = make_args(t);
  a.keys = keys;
  a.vals = vals;
  a.n = n;
  a.vals_out = vals_out;
  a.flags = flags;
  a.up = up;
  // Combining equal keys is exact for "add" as long as no insertion can find
  // the table full: used + (insertions since the last count) <= c.
  a.aggregate = (op == OP_UPSERT && up == LPHT_ADD && t->tuning.aggregate &&
                 t->known_used + t->pending <= (1ull << t->log2c))
                    ? 1u
                    : 0u;
  if (a.aggregate && t->tuning.aggregate == 1 && part_applies(n, t->log2c)) {
    // large insert-or-add on a large table: partition by table region first
    const size_t sb = part_scratch_bytes(n, t->log2c, t->cfg.layout, vals != nullptr, flags != nullptr,
                                         t->launch.num_cus);
    void *scratch = dev_alloc(t, sb, s);
    if (scratch) {
      const hipError_t e = launch_upsert_add_part(a, scratch, t->launch.num_cus, s);
      dev_free(t, scratch, sb, s);
      if (e != hipSuccess) return from_hip(e);
      if (t->special)
        return from_hip(launch_special(t->cfg.layout, op, up, keys, vals, n, vals_out, flags, t->special,
                                       t->special_scratch, false, s));
      return LPHT_OK;
    }
    // no memory for the partition: combine chunk by chunk instead
  }
  const bool inserting = op == OP_INSERT || op == OP_UPSERT;
  const uint64_t c = 1ull << t->log2c;
  // bound on used before this call (the growth rule already counted it)
  const uint64_t used0 = t->known_used + t->pending - (inserting ? n : 0);
  bool by_fill = false;
  for (uint8_t g : t->tuning.g_modify) by_fill |= g != 0;
  const uint32_t kb = t->cfg.layout == LPHT_PACKED32 ? 4 : 8;
  uint64_t done = 0;
  while (done < n) {
    uint64_t len = n - done;
    if (inserting && by_fill) {
      for (uint64_t q = 1; q < 4; ++q) {
        const uint64_t b = q * c / 4;
        if (used0 + done < b && b < used0 + done + len && b - (used0 + done) >= kMinPiece &&
            used0 + done + len - b >= kMinPiece &&
            pick_group_width(t, op, b) != pick_group_width(t, op, b + 1))
          len = b - (used0 + done);
      }
    }
    BulkArgs p = a;
    p.keys = (const unsigned char *)keys + done * kb;
    p.vals = vals ? (const unsigned char *)vals + done * kb : nullptr;
    p.vals_out = vals_out ? (unsigned char *)vals_out + done * kb : nullptr;
    p.flags = flags ? flags + done : nullptr;
    p.n = len;
    LaunchCfg cfg = t->launch;
    cfg.group_width = pick_group_width(t, op, inserting ? used0 + done + len : t->known_used + t->pending);
    const hipError_t e = launch_bulk(op, p, cfg, s);
    if (e != hipSuccess) return from_hip(e);
    done += len;
  }
  if (t->special)
    return from_hip(launch_special(t->cfg.layout, op, up, keys, vals, n, vals_out, flags, t->special,
                                   t->special_scratch, false, s));
  return LPHT_OK;
}

}  // namespace host
}  // namespace lpht

using namespace lpht::host;



namespace {

const OpKind kPhaseOrder[] = {OP_FIND, OP_INSERT, OP_UPSERT, OP_UPDATE, OP_ERASE};

void batch_free(lpht_batch *b) {
  for (int i = 0; i < lpht_batch::kSlots; ++i) {
    if (b->ev[i]) (void)hipEventDestroy(b->ev[i]);
    if (b->host[i]) (void)hipHostFree(b->host[i]);
    if (b->dev[i]) (void)hipFree(b->dev[i]);
  }
  delete b;
}

// Uploads one group's descriptors and round offsets through a ring slot and
// launches it.
int batch_launch(lpht_batch *b, OpKind op, uint32_t up, uint32_t layout, const BulkArgs *args,
                 uint32_t nd, const LaunchCfg &cfg, hipStream_t s) {
  const int slot = b->next;
  b->next = (b->next + 1) % lpht_batch::kSlots;
  if (b->used[slot] && hipEventSynchronize(b->ev[slot]) != hipSuccess) return LPHT_ERR_DEVICE;
  BulkArgs *ha = (BulkArgs *)b->host[slot];
  uint64_t *hr = (uint64_t *)(b->host[slot] + sizeof(BulkArgs) * b->max_ops);
  uint64_t total = 0;
  for (uint32_t j = 0; j < nd; ++j) {
    ha[j] = args[j];
    hr[j] = total;
    total += (args[j].n + kRound - 1) / kRound;
  }
  hr[nd] = total;
  if (total == 0) return LPHT_OK;
  hipError_t e = hipMemcpyAsync(b->dev[slot], b->host[slot], b->slot_bytes, hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = launch_bulk_multi(op, up, layout, (const BulkArgs *)b->dev[slot],
                          (const uint64_t *)(b->dev[slot] + sizeof(BulkArgs) * b->max_ops), nd, total,
                          cfg, s);
  if (e == hipSuccess) e = hipEventRecord(b->ev[slot], s);
  if (e != hipSuccess) return from_hip(e);
  b->used[slot] = true;
  return LPHT_OK;
}

}  // namespace

extern "C" {

int lpht_batch_create(uint32_t max_ops, lpht_batch **out) {
  if (!out) return LPHT_ERR_INVALID;
  *out = nullptr;
  if (max_ops == 0 || max_ops > (1u << 20)) return LPHT_ERR_INVALID;
  lpht_batch *b = new (std::nothrow) lpht_batch();
  if (!b) return LPHT_ERR_OOM;
  if (hipGetDevice(&b->device) != hipSuccess) {
    delete b;
    return LPHT_ERR_DEVICE;
  }
  b->max_ops = max_ops;
  b->slot_bytes = sizeof(BulkArgs) * max_ops + sizeof(uint64_t) * (max_ops + 1);
  for (int i = 0; i < lpht_batch::kSlots; ++i) {
    if (hipHostMalloc((void **)&b->host[i], b->slot_bytes, hipHostMallocDefault) != hipSuccess ||
        hipMalloc((void **)&b->dev[i], b->slot_bytes) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev[i], hipEventDisableTiming) != hipSuccess) {
      batch_free(b);
      return LPHT_ERR_OOM;
    }
  }
  *out = b;
  return LPHT_OK;
}

int lpht_batch_destroy(lpht_batch *b) {
  if (!b) return LPHT_OK;
  (void)hipSetDevice(b->device);
  for (int i = 0; i < lpht_batch::kSlots; ++i)
    if (b->used[i]) (void)hipEventSynchronize(b->ev[i]);
  batch_free(b);
  return LPHT_OK;
}

int lpht_batch_run(lpht_batch *b, const lpht_batch_op *ops, uint32_t nops, void *stream) {
  if (!b || (nops && !ops) || nops > b->max_ops) return LPHT_ERR_INVALID;
  for (uint32_t j = 0; j < nops; ++j) {
    const lpht_batch_op &o = ops[j];
    if (!o.table || o.op > LPHT_OP_ERASE || o.up > LPHT_ADD) return LPHT_ERR_INVALID;
    if (o.table->special) return LPHT_ERR_UNSUPPORTED;
    if (o.count_sel > o.n) return LPHT_ERR_INVALID;
    if (o.table->device != b->device) return LPHT_ERR_INVALID;
    int rc = check_arrays(o.table, o.keys, o.vals, o.n);
    if (rc) return rc;
    if (o.vals_out && !aligned(o.vals_out, o.table->cfg.layout == LPHT_PACKED32 ? 4 : 8))
      return LPHT_ERR_INVALID;
  }
  hipStream_t s = (hipStream_t)stream;
  if (hipSetDevice(b->device) != hipSuccess) return LPHT_ERR_DEVICE;
  std::vector<BulkArgs> group;
  group.reserve(nops);
  for (OpKind op : kPhaseOrder) {
    for (uint32_t up = 0; up <= 1; ++up) {
      if (up == 1 && op != OP_UPSERT && op != OP_UPDATE) continue;
      for (uint32_t layout = 0; layout <= 1; ++layout) {
        // growth first: each table grows once for all of its descriptors
        if (op == OP_INSERT || op == OP_UPSERT) {
          std::vector<std::pair<lpht_table *, uint64_t>> need;
          for (uint32_t j = 0; j < nops; ++j) {
            const lpht_batch_op &o = ops[j];
            if ((OpKind)o.op != op || o.table->cfg.layout != layout || o.n == 0) continue;
            if (op == OP_UPSERT && o.up != up) continue;
            if (o.kinds && o.count_sel == 0) continue;
            const uint64_t b_ops = o.kinds ? o.count_sel : o.n;
            bool found = false;
            for (auto &pr : need)
              if (pr.first == o.table) {
                pr.second += b_ops;
                found = true;
              }
            if (!found) need.emplace_back(o.table, b_ops);
          }
          for (auto &pr : need) {
            int rc = grow_before_batch(pr.first, pr.second, s);
            if (rc) return rc;
          }
        }
        group.clear();
        const lpht_table *first = nullptr;
        for (uint32_t j = 0; j < nops; ++j) {
          const lpht_batch_op &o = ops[j];
          if ((OpKind)o.op != op || o.table->cfg.layout != layout || o.n == 0) continue;
          if ((op == OP_UPSERT || op == OP_UPDATE) && o.up != up) continue;
          if (o.kinds && o.count_sel == 0) continue;
          if (op != OP_FIND) o.table->mods_since_exact++;
          BulkArgs a = make_args(o.table);
          a.keys = o.keys;
          a.vals = o.vals;
          a.n = o.n;
          a.vals_out = o.vals_out;
          a.flags = o.flags;
          a.up = up;
          a.kinds = o.kinds;
          a.kind_sel = o.kind_sel;
          group.push_back(a);
          if (!first) first = o.table;
        }
        if (group.empty()) continue;
        int rc = batch_launch(b, op, up, layout, group.data(), (uint32_t)group.size(), first->launch, s);
        if (rc) return rc;
      }
    }
  }
  return LPHT_OK;
}


void lpht_config_default(lpht_config *cfg) {
  if (!cfg) return;
  *cfg = lpht_config{};
  cfg->layout = LPHT_KV64;
  cfg->log2_capacity = 12;
  cfg->seed_hi = 0x9E3779B9u;
  cfg->seed_lo = 0xFFFFFFFFu;
  cfg->max_fill_num = 1;
  cfg->max_fill_den = 2;
  cfg->auto_grow = 0;
}

int lpht_create(const lpht_config *cfg, void *stream, lpht_table **out) {
  if (!out) return LPHT_ERR_INVALID;
  *out = nullptr;
  if (!cfg) return LPHT_ERR_INVALID;
  if (cfg->layout != LPHT_PACKED32 && cfg->layout != LPHT_KV64) return LPHT_ERR_INVALID;
  if (cfg->log2_capacity < 6 || cfg->log2_capacity > 34) return LPHT_ERR_INVALID;
  if (cfg->max_fill_num == 0 || cfg->max_fill_den == 0 || cfg->max_fill_num > cfg->max_fill_den)
    return LPHT_ERR_INVALID;
  if (cfg->full_keys > 1) return LPHT_ERR_INVALID;
  if (cfg->reserved0 != 0) return LPHT_ERR_INVALID;
  if (cfg->hash != LPHT_HASH_CRC32C_PAIR && cfg->hash != LPHT_HASH_MULSHIFT) return LPHT_ERR_INVALID;
  if (cfg->hash == LPHT_HASH_MULSHIFT && (cfg->mul & 1u) == 0) return LPHT_ERR_INVALID;
  if ((cfg->alloc == nullptr) != (cfg->free == nullptr)) return LPHT_ERR_INVALID;
  lpht_table *t = new (std::nothrow) lpht_table();
  if (!t) return LPHT_ERR_OOM;
  t->cfg = *cfg;
  if (hipGetDevice(&t->device) != hipSuccess) {
    delete t;
    return LPHT_ERR_DEVICE;
  }
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, t->device) != hipSuccess ||
      ncu <= 0) {
    delete t;
    return LPHT_ERR_DEVICE;
  }
  t->launch.num_cus = (uint32_t)ncu;
  t->tuning.block_threads = 256;
  t->tuning.group_width = 1;
  t->tuning.blocks_per_cu = 8;
  t->tuning.migrate_block = 512;
  t->tuning.aggregate = 1;
  fill_launch(t);
  const int kb = cfg->layout == LPHT_PACKED32 ? 4 : 8;
  t->crc_hi = crc0_bytes(cfg->seed_hi, kb);
  t->crc_lo = crc0_bytes(cfg->seed_lo, kb);
  t->mul = cfg->hash == LPHT_HASH_MULSHIFT ? cfg->mul : 0;
  hipStream_t s = (hipStream_t)stream;
  t->status = (DevStatus *)dev_alloc(t, sizeof(DevStatus), s);
  if (!t->status) {
    delete t;
    return LPHT_ERR_OOM;
  }
  hipError_t e = launch_set_status(t->status, 0, 0, 1, s);
  if (e != hipSuccess) {
    dev_free(t, t->status, sizeof(DevStatus), s);
    delete t;
    return from_hip(e);
  }
  const size_t nb = (size_t)cell_bytes(cfg->layout) << cfg->log2_capacity;
  t->cells = dev_alloc(t, nb, s);
  if (!t->cells) {
    dev_free(t, t->status, sizeof(DevStatus), s);
    delete t;
    return LPHT_ERR_OOM;
  }
  t->log2c = cfg->log2_capacity;
  t->log2_min = cfg->log2_capacity;
  e = launch_fill_zero(t->cells, nb, t->launch, s);
  if (e == hipSuccess && cfg->full_keys) {
    t->special = (SpecialSlots *)dev_alloc(t, sizeof(SpecialSlots), s);
    t->special_scratch = (uint32_t *)dev_alloc(t, kSpecialScratchBytes, s);
    if (!t->special || !t->special_scratch) e = hipErrorOutOfMemory;
    if (e == hipSuccess) e = launch_fill_zero(t->special, sizeof(SpecialSlots), t->launch, s);
    if (e == hipSuccess) e = launch_fill_zero(t->special_scratch, kSpecialScratchBytes, t->launch, s);
  }
  if (e != hipSuccess) {
    if (t->special) dev_free(t, t->special, sizeof(SpecialSlots), s);
    if (t->special_scratch) dev_free(t, t->special_scratch, kSpecialScratchBytes, s);
    dev_free(t, t->cells, nb, s);
    dev_free(t, t->status, sizeof(DevStatus), s);
    delete t;
    return from_hip(e);
  }
  *out = t;
  return LPHT_OK;
}

int lpht_clear(lpht_table *t, void *stream) {
  if (!t) return LPHT_ERR_INVALID;
  hipStream_t s = (hipStream_t)stream;
  if (hipSetDevice(t->device) != hipSuccess) return LPHT_ERR_DEVICE;
  hipError_t e = launch_fill_zero(t->cells, (size_t)cell_bytes(t->cfg.layout) << t->log2c, t->launch, s);
  if (e == hipSuccess) e = launch_set_status(t->status, 0, 0, 1, s);
  if (e == hipSuccess && t->special) e = launch_fill_zero(t->special, sizeof(SpecialSlots), t->launch, s);
  if (e != hipSuccess) return from_hip(e);
  t->known_used = t->known_live = 0;
  t->pending = 0;
  t->mods_since_exact = 0;
  return LPHT_OK;
}

int lpht_destroy(lpht_table *t, void *stream) {
  if (!t) return LPHT_OK;
  hipStream_t s = (hipStream_t)stream;
  (void)hipSetDevice(t->device);
  dev_free(t, t->cells, (size_t)cell_bytes(t->cfg.layout) << t->log2c, s);
  dev_free(t, t->status, sizeof(DevStatus), s);
  if (t->special) dev_free(t, t->special, sizeof(SpecialSlots), s);
  if (t->special_scratch) dev_free(t, t->special_scratch, kSpecialScratchBytes, s);
  for (auto &tm : t->timed) {
    (void)hipEventDestroy(tm.start);
    (void)hipEventDestroy(tm.stop);
  }
  delete t;
  return LPHT_OK;
}

int lpht_insert(lpht_table *t, const void *keys, const void *vals, uint64_t n, uint8_t *flags,
                void *stream) {
  return run_bulk(t, OP_INSERT, keys, vals, n, 0, nullptr, flags, stream);
}

int lpht_find(lpht_table *t, const void *keys, uint64_t n, void *vals_out, uint8_t *found,
              void *stream) {
  return run_bulk(t, OP_FIND, keys, nullptr, n, 0, vals_out, found, stream);
}

int lpht_insert_or_update(lpht_table *t, const void *keys, const void *vals, uint64_t n,
                          uint32_t op, uint8_t *inserted, void *stream) {
  return run_bulk(t, OP_UPSERT, keys, vals, n, op, nullptr, inserted, stream);
}

int lpht_update(lpht_table *t, const void *keys, const void *vals, uint64_t n, uint32_t op,
                uint8_t *flags, void *stream) {
  return run_bulk(t, OP_UPDATE, keys, vals, n, op, nullptr, flags, stream);
}

int lpht_erase(lpht_table *t, const void *keys, uint64_t n, uint8_t *flags, void *stream) {
  return run_bulk(t, OP_ERASE, keys, nullptr, n, 0, nullptr, flags, stream);
}

namespace {

// The sort-based bulk build (keep_old = false) and batched merge (Sec. 5.5):
// the result replaces the table's cells; the host learns the distinct count
// from the device (one synchronisation after the launches, one before to
// know the live elements exactly).
int bulk_merge(lpht_table *t, const void *keys, const void *vals, uint64_t n, uint32_t op, bool keep_old,
               void *stream) {
  int rc = check_arrays(t, keys, vals, n);
  if (rc) return rc;
  if (op > LPHT_ADD) return LPHT_ERR_INVALID;
  if (n >= (1ull << 32) - 1) return LPHT_ERR_UNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  if (hipSetDevice(t->device) != hipSuccess) return LPHT_ERR_DEVICE;
  rc = sync_counts(t, s);
  if (rc) return rc;
  const uint64_t old_live = keep_old ? t->known_live : 0;
  uint32_t log2_new = t->log2c;
  if (t->cfg.auto_grow)
    while (!within_fill(t, old_live + n, 1ull << log2_new)) {
      if (log2_new >= 34) return LPHT_ERR_OOM;
      ++log2_new;
    }
  if (log2_new > kBulkMaxLog2) return LPHT_ERR_UNSUPPORTED;
  const uint64_t max_items = old_live + n;
  if (max_items >= (1ull << 32)) return LPHT_ERR_UNSUPPORTED;
  const uint64_t old_ncells = keep_old ? (1ull << t->log2c) : 0;
  const size_t nb = (size_t)cell_bytes(t->cfg.layout) << log2_new;
  const size_t sb = bulk_merge_scratch_bytes(old_ncells + n, max_items, log2_new, t->cfg.layout);
  void *nc = dev_alloc(t, nb, s);
  if (!nc) return LPHT_ERR_OOM;
  void *scratch = dev_alloc(t, sb, s);
  if (!scratch) {
    dev_free(t, nc, nb, s);
    return LPHT_ERR_OOM;
  }
  BulkMergeArgs a{};
  a.layout = t->cfg.layout;
  a.op = op;
  a.old_cells = keep_old ? t->cells : nullptr;
  a.old_ncells = old_ncells;
  a.keys = keys;
  a.vals = vals;
  a.n = n;
  a.max_items = max_items;
  a.new_cells = nc;
  a.log2_new = log2_new;
  a.crc_hi = t->crc_hi;
  a.crc_lo = t->crc_lo;
  a.mul = t->mul;
  a.status = t->status;
  a.scratch = scratch;
  a.num_cus = t->launch.num_cus;
  BulkMergeCtl ctl{};
  hipError_t e = launch_set_status(t->status, 0, 0, 0, s);
  if (e == hipSuccess) e = launch_bulk_merge(a, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&ctl, scratch, sizeof(ctl), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  dev_free(t, scratch, sb, s);
  if (e != hipSuccess || ctl.full) {
    dev_free(t, nc, nb, s);
    // the table is unchanged: restore its counts
    (void)launch_set_status(t->status, t->known_used, t->known_live, 0, s);
    return e != hipSuccess ? from_hip(e) : ctl.full == 1 ? LPHT_ERR_FULL : LPHT_ERR_DEVICE;
  }
  dev_free(t, t->cells, (size_t)cell_bytes(t->cfg.layout) << t->log2c, s);
  t->cells = nc;
  t->log2c = log2_new;
  t->known_used = t->known_live = ctl.distinct;
  t->pending = 0;
  t->mods_since_exact = 0;
  t->stats.bulk_merges++;
  if (t->special) {
    // the batch's keys 0 and 1, in index order, on the special slots (a
    // build starts them empty)
    e = launch_special(t->cfg.layout, OP_UPSERT, op, keys, vals, n, nullptr, nullptr, t->special,
                       t->special_scratch, !keep_old, s);
    if (e != hipSuccess) return from_hip(e);
  }
  return LPHT_OK;
}

}  // namespace

int lpht_build(lpht_table *t, const void *keys, const void *vals, uint64_t n, uint32_t op, void *stream) {
  return bulk_merge(t, keys, vals, n, op, false, stream);
}

int lpht_build_noalloc(lpht_table *t, const void *keys, const void *vals, uint64_t n, uint32_t op,
                       void *stream) {
  int rc = check_arrays(t, keys, vals, n);
  if (rc) return rc;
  if (op > LPHT_ADD) return LPHT_ERR_INVALID;
  if (n >= (1ull << 32) - 1) return LPHT_ERR_UNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  if (hipSetDevice(t->device) != hipSuccess) return LPHT_ERR_DEVICE;
  void *scratch = nullptr;
  hipError_t e = noalloc_scratch(t->device, &scratch);
  if (e != hipSuccess) return from_hip(e);
  // the capacity cannot change (a new cell array would be an allocation)
  if (t->log2c > kBulkMaxLog2) return LPHT_ERR_UNSUPPORTED;
  if (t->cfg.auto_grow && !within_fill(t, n, 1ull << t->log2c)) return LPHT_ERR_UNSUPPORTED;
  if (bulk_merge_scratch_bytes(n, n, t->log2c, t->cfg.layout) > kNoAllocScratchBytes) return LPHT_ERR_INVALID;
  rc = sync_counts(t, s);
  if (rc) return rc;
  BulkMergeArgs a{};
  a.layout = t->cfg.layout;
  a.op = op;
  a.keys = keys;
  a.vals = vals;
  a.n = n;
  a.max_items = n;
  // a build never reads the old cells, and when it does not fail for lack
  // of room it writes every cell, so the result goes to the table's own array
  a.new_cells = t->cells;
  a.log2_new = t->log2c;
  a.crc_hi = t->crc_hi;
  a.crc_lo = t->crc_lo;
  a.mul = t->mul;
  a.status = t->status;
  a.scratch = scratch;
  a.num_cus = t->launch.num_cus;
  BulkMergeCtl ctl{};
  e = launch_set_status(t->status, 0, 0, 0, s);
  if (e == hipSuccess) e = launch_bulk_merge(a, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&ctl, scratch, sizeof(ctl), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess || ctl.full) {
    (void)launch_set_status(t->status, t->known_used, t->known_live, 0, s);
    return e != hipSuccess ? from_hip(e) : ctl.full == 1 ? LPHT_ERR_FULL : LPHT_ERR_DEVICE;
  }
  t->known_used = t->known_live = ctl.distinct;
  t->pending = 0;
  t->mods_since_exact = 0;
  t->stats.bulk_merges++;
  if (t->special) {
    e = launch_special(t->cfg.layout, OP_UPSERT, op, keys, vals, n, nullptr, nullptr, t->special,
                       t->special_scratch, 1, s);
    if (e != hipSuccess) return from_hip(e);
  }
  return LPHT_OK;
}

int lpht_merge(lpht_table *t, const void *keys, const void *vals, uint64_t n, uint32_t op, void *stream) {
  return bulk_merge(t, keys, vals, n, op, true, stream);
}

int lpht_insert_async(lpht_table *t, const void *keys, const void *vals, uint64_t n, uint32_t add,
                      uint8_t *flags, void *stream) {
  int rc = check_arrays(t, keys, vals, n);
  if (rc) return rc;
  if (add > 1) return LPHT_ERR_INVALID;
  if (n == 0) return LPHT_OK;
  hipStream_t s = (hipStream_t)stream;
  if (hipSetDevice(t->device) != hipSuccess) return LPHT_ERR_DEVICE;
  const uint32_t grid = async_grid(t->device);
  if (!grid || t->cfg.max_fill_den - t->cfg.max_fill_num < 1) return LPHT_ERR_UNSUPPORTED;
  rc = sync_counts(t, s);
  if (rc) return rc;
  // the kernel needs room for the work in flight, and starts below the trigger
  uint32_t lg = std::max(t->log2c, async_min_log2(grid, t->cfg.max_fill_num, t->cfg.max_fill_den));
  while (!within_fill(t, t->known_used, 1ull << lg)) ++lg;
  if (lg > 34) return LPHT_ERR_OOM;
  if (lg != t->log2c) {
    rc = migrate_once(t, lg, s);
    if (rc) return rc;
  }
  // the ladder of doubled tables, up to the capacity that holds used + n
  uint32_t K = 0;
  while (!within_fill(t, t->known_used + n, 1ull << (t->log2c + K))) ++K;
  if (K > kAsyncLadder || t->log2c + K > 34) return LPHT_ERR_UNSUPPORTED;
  AsyncArgs a{};
  a.layout = t->cfg.layout;
  a.add = add;
  a.keys = keys;
  a.vals = vals;
  a.n = n;
  a.flags = flags;
  a.ladder[0] = t->cells;
  a.nladder = K + 1;
  a.log2c = t->log2c;
  a.used0 = t->known_used;
  a.alpha_num = t->cfg.max_fill_num;
  a.alpha_den = t->cfg.max_fill_den;
  a.crc_hi = t->crc_hi;
  a.crc_lo = t->crc_lo;
  a.mul = t->mul;
  a.status = t->status;
  a.grid = grid;
  const size_t cb = cell_bytes(t->cfg.layout);
  auto release = [&](uint32_t keep) {
    for (uint32_t i = 1; i <= K; ++i)
      if (i != keep && a.ladder[i]) dev_free(t, a.ladder[i], cb << (t->log2c + i), s);
  };
  for (uint32_t i = 1; i <= K; ++i) {
    a.ladder[i] = dev_alloc(t, cb << (t->log2c + i), s);
    if (!a.ladder[i]) {
      release(0);
      return LPHT_ERR_OOM;
    }
    // no clearing: the kernel's block migration writes every cell of the
    // target (its rare fallback clears the target itself)
  }
  AsyncCtl *ctl = (AsyncCtl *)dev_alloc(t, sizeof(AsyncCtl), s);
  if (!ctl) {
    release(0);
    return LPHT_ERR_OOM;
  }
  a.ctl = ctl;
  AsyncCtl h{};
  hipError_t e = launch_async_insert(a, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&h, ctl, sizeof(h), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  dev_free(t, ctl, sizeof(AsyncCtl), s);
  if (e != hipSuccess) {
    release(0);
    return from_hip(e);
  }
  const uint32_t fin = h.epoch;
  if (fin > K) {
    release(0);
    return LPHT_ERR_DEVICE;
  }
  release(fin);
  if (fin > 0) {
    dev_free(t, t->cells, cb << t->log2c, s);
    t->stats.migrations += fin;
    t->stats.resizes += fin;
    for (uint32_t i = 0; i < fin; ++i) t->stats.cells_migrated += 1ull << (t->log2c + i);
    t->cells = a.ladder[fin];
    t->log2c += fin;
  }
  t->stats.async_growths += fin;
  t->stats.async_fallbacks += h.fallbacks;
  if (t->special) {
    e = launch_special(t->cfg.layout, add ? OP_UPSERT : OP_INSERT, add ? LPHT_ADD : LPHT_ASSIGN, keys, vals, n,
                       nullptr, flags, t->special, t->special_scratch, false, s);
    if (e != hipSuccess) return from_hip(e);
  }
  // exact counts of the result
  e = launch_set_status(t->status, 0, 0, 0, s);
  if (e == hipSuccess) e = launch_recount(t->cells, t->log2c, t->cfg.layout, t->status, t->launch, s);
  if (e != hipSuccess) return from_hip(e);
  rc = sync_counts(t, s);
  if (rc) return rc;
  return (h.err & 3) ? LPHT_ERR_DEVICE : LPHT_OK;
}

int lpht_grow(lpht_table *t, uint32_t log2_new_capacity, void *stream) {
  if (!t) return LPHT_ERR_INVALID;
  if (log2_new_capacity < 6 || log2_new_capacity > 34) return LPHT_ERR_INVALID;
  hipStream_t s = (hipStream_t)stream;
  if (hipSetDevice(t->device) != hipSuccess) return LPHT_ERR_DEVICE;
  int rc = sync_counts(t, s);
  if (rc) return rc;
  return migrate_once(t, log2_new_capacity, s);
}

int lpht_count(lpht_table *t, uint64_t *used, uint64_t *live, void *stream) {
  if (!t) return LPHT_ERR_INVALID;
  if (hipSetDevice(t->device) != hipSuccess) return LPHT_ERR_DEVICE;
  int rc = sync_counts(t, (hipStream_t)stream);
  if (rc) return rc;
  uint64_t sp = 0;
  if (t->special) {
    unsigned long long pr[2] = {0, 0};
    hipError_t e = hipMemcpyAsync(pr, t->special, sizeof(pr), hipMemcpyDeviceToHost, (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return from_hip(e);
    sp = pr[0] + pr[1];
  }
  if (used) *used = t->known_used + sp;
  if (live) *live = t->known_live + sp;
  return LPHT_OK;
}

int lpht_capacity(const lpht_table *t, uint64_t *cells, uint32_t *log2_capacity) {
  if (!t) return LPHT_ERR_INVALID;
  if (cells) *cells = 1ull << t->log2c;
  if (log2_capacity) *log2_capacity = t->log2c;
  return LPHT_OK;
}

uint32_t lpht_cell_bytes(uint32_t layout) { return (uint32_t)cell_bytes(layout); }

int lpht_export_cells(lpht_table *t, void *dst_device, void *stream) {
  if (!t || !dst_device) return LPHT_ERR_INVALID;
  if (hipSetDevice(t->device) != hipSuccess) return LPHT_ERR_DEVICE;
  const size_t nb = (size_t)cell_bytes(t->cfg.layout) << t->log2c;
  return from_hip(hipMemcpyAsync(dst_device, t->cells, nb, hipMemcpyDeviceToDevice,
                                 (hipStream_t)stream));
}

int lpht_import_cells(lpht_table *t, const void *src_device, uint32_t log2_capacity, void *stream) {
  if (!t || !src_device) return LPHT_ERR_INVALID;
  if (log2_capacity < 6 || log2_capacity > 34) return LPHT_ERR_INVALID;
  if (!aligned(src_device, 16)) return LPHT_ERR_INVALID;
  hipStream_t s = (hipStream_t)stream;
  if (hipSetDevice(t->device) != hipSuccess) return LPHT_ERR_DEVICE;
  const size_t nb = (size_t)cell_bytes(t->cfg.layout) << log2_capacity;
  void *nc = t->cells;
  if (log2_capacity != t->log2c) {
    nc = dev_alloc(t, nb, s);
    if (!nc) return LPHT_ERR_OOM;
  }
  hipError_t e = hipMemcpyAsync(nc, src_device, nb, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) {
    if (nc != t->cells) dev_free(t, nc, nb, s);
    return from_hip(e);
  }
  if (nc != t->cells) {
    dev_free(t, t->cells, (size_t)cell_bytes(t->cfg.layout) << t->log2c, s);
    t->cells = nc;
    t->log2c = log2_capacity;
  }
  e = launch_set_status(t->status, 0, 0, 0, s);
  if (e == hipSuccess) e = launch_recount(t->cells, t->log2c, t->cfg.layout, t->status, t->launch, s);
  if (e != hipSuccess) return from_hip(e);
  return sync_counts(t, s);
}

int lpht_status(lpht_table *t, void *stream) {
  if (!t) return LPHT_ERR_INVALID;
  hipStream_t s = (hipStream_t)stream;
  if (hipSetDevice(t->device) != hipSuccess) return LPHT_ERR_DEVICE;
  DevStatus h;
  uint64_t u, l;
  int rc = read_status(t, s, &h, &u, &l);
  if (rc) return rc;
  t->known_used = u;
  t->known_live = l;
  t->pending = 0;
  t->mods_since_exact = 0;
  if (h.err) {
    hipError_t e = launch_set_status(t->status, u, l, 1, s);
    if (e != hipSuccess) return from_hip(e);
  }
  if (h.err & kErrFull) return LPHT_ERR_FULL;
  if ((h.err & kErrReserved) && !t->special) return LPHT_ERR_RESERVED_KEY;
  return LPHT_OK;
}

int lpht_set_tuning(lpht_table *t, const lpht_tuning *tuning) {
  if (!t || !tuning || !tuning_ok(tuning)) return LPHT_ERR_INVALID;
  t->tuning = *tuning;
  fill_launch(t);
  return LPHT_OK;
}

int lpht_get_tuning(const lpht_table *t, lpht_tuning *tuning) {
  if (!t || !tuning) return LPHT_ERR_INVALID;
  *tuning = t->tuning;
  return LPHT_OK;
}

int lpht_set_timing(lpht_table *t, int timing) {
  if (!t) return LPHT_ERR_INVALID;
  t->timing = timing ? 1 : 0;
  return LPHT_OK;
}

int lpht_get_stats(lpht_table *t, lpht_stats *stats) {
  if (!t || !stats) return LPHT_ERR_INVALID;
  for (auto &tm : t->timed) {
    if (hipEventSynchronize(tm.stop) != hipSuccess) return LPHT_ERR_DEVICE;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, tm.start, tm.stop) == hipSuccess) t->stats.migrate_ms += ms;
    (void)hipEventDestroy(tm.start);
    (void)hipEventDestroy(tm.stop);
  }
  t->timed.clear();
  *stats = t->stats;
  return LPHT_OK;
}

const char *lpht_strerror(int code) {
  switch (code) {
    case LPHT_OK: return "ok";
    case LPHT_ERR_INVALID: return "invalid argument";
    case LPHT_ERR_OOM: return "out of device memory";
    case LPHT_ERR_FULL: return "bounded table full: an insertion found no empty cell";
    case LPHT_ERR_RESERVED_KEY: return "reserved key (0 = empty, 1 = tombstone) used";
    case LPHT_ERR_DEVICE: return "HIP runtime error";
    case LPHT_ERR_UNSUPPORTED: return "unsupported";
    default: return "unknown error";
  }
}

const char *lpht_version(void) { return "lpht 0.1 gfx950"; }

int lpht_release_pools(void) { return release_pools(); }

}  // extern "C"
