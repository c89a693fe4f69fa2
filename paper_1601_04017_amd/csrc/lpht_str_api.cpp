// C ABI of the string-key table (see include/lpht.h, "String keys").

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "lpht_host.h"
#include "lpht_str.h"

using namespace lpht;
using namespace lpht::host;

struct lpht_str_table {
  lpht_str_config cfg;
  int device;
  uint32_t num_cus;
  uint32_t log2c, log2_min;
  uint64_t *cells;
  uint8_t *pool;
  uint64_t pool_cap;
  StrCtl *ctl;
  // exact at the last recount, plus an upper bound of insertions since
  uint64_t known_used, known_live, pending;
};

namespace {

void *alloc(lpht_str_table *t, size_t bytes, hipStream_t s) { return pool_alloc(t->device, bytes, s); }
void release(void *p, hipStream_t s) { pool_free(p, s); }

LaunchCfg fill_cfg(const lpht_str_table *t) {
  LaunchCfg c{};
  c.block_threads = 256;
  c.group_width = 1;
  c.blocks_per_cu = 8;
  c.num_cus = t->num_cus;
  c.migrate_block = 512;
  return c;
}

bool fits(const lpht_str_table *t, uint64_t x, uint64_t c) {
  return (unsigned __int128)x * t->cfg.max_fill_den <= (unsigned __int128)c * t->cfg.max_fill_num;
}

// Exact used/live and pool cursor (synchronises the stream).
int recount(lpht_str_table *t, hipStream_t s) {
  hipError_t e = launch_str_recount(t->cells, t->log2c, t->ctl, t->num_cus, s);
  StrCtl h{};
  if (e == hipSuccess) e = hipMemcpyAsync(&h, t->ctl, sizeof(h), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return from_hip(e);
  t->known_used = h.used;
  t->known_live = h.live;
  t->pending = 0;
  return LPHT_OK;
}

uint64_t pool_cursor(lpht_str_table *t, hipStream_t s, int *rc) {
  unsigned long long v = 0;
  hipError_t e = hipMemcpyAsync(&v, &t->ctl->pool_used, sizeof(v), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  *rc = from_hip(e);
  return v;
}

// Migrates into 2^log2_new cells and a new pool of new_pool_cap bytes,
// copying only live keys.  known_live must be exact.
int migrate(lpht_str_table *t, uint32_t log2_new, uint64_t new_pool_cap, hipStream_t s) {
  if (t->known_live >= (1ull << log2_new)) return LPHT_ERR_FULL;
  const size_t nb = (size_t)16 << log2_new;
  uint64_t *nc = (uint64_t *)alloc(t, nb, s);
  uint8_t *np = (uint8_t *)alloc(t, new_pool_cap, s);
  if (!nc || !np) {
    release(nc, s);
    release(np, s);
    return LPHT_ERR_OOM;
  }
  hipError_t e = launch_fill_zero(nc, nb, fill_cfg(t), s);
  StrMigArgs a{};
  a.old_cells = t->cells;
  a.log2_old = t->log2c;
  a.old_pool = t->pool;
  a.new_cells = nc;
  a.log2_new = log2_new;
  a.new_pool = np;
  a.new_pool_cap = new_pool_cap;
  a.ctl = t->ctl;
  a.crc_hi = t->cfg.seed_hi;
  a.crc_lo = t->cfg.seed_lo;
  if (e == hipSuccess) e = launch_str_migrate(a, t->num_cus, s);
  if (e != hipSuccess) {
    release(nc, s);
    release(np, s);
    return from_hip(e);
  }
  release(t->cells, s);
  release(t->pool, s);
  t->cells = nc;
  t->pool = np;
  t->pool_cap = new_pool_cap;
  t->log2c = log2_new;
  t->known_used = t->known_live;
  t->pending = 0;
  return LPHT_OK;
}

// The word tables' growth rule (trigger at alpha on non-empty cells; cleanup
// that may shrink when live + b <= alpha c / 2; else doubling), plus room in
// the pool for `bytes` more record bytes.
int grow_before(lpht_str_table *t, uint64_t b, uint64_t bytes, hipStream_t s) {
  int rc = LPHT_OK;
  const uint64_t pused = pool_cursor(t, s, &rc);
  if (rc) return rc;
  const bool pool_ok = pused + bytes <= t->pool_cap;
  const uint64_t c = 1ull << t->log2c;
  if (pool_ok && (!t->cfg.auto_grow || fits(t, t->known_used + t->pending + b, c))) {
    t->pending += b;
    return LPHT_OK;
  }
  rc = recount(t, s);
  if (rc) return rc;
  uint32_t target = t->log2c;
  bool move = !pool_ok;
  if (t->cfg.auto_grow && !fits(t, t->known_used + b, c)) {
    move = true;
    if ((unsigned __int128)(t->known_live + b) * 2 * t->cfg.max_fill_den <= (unsigned __int128)c * t->cfg.max_fill_num) {
      while (target > t->log2_min && (unsigned __int128)(t->known_live + b) * 4 * t->cfg.max_fill_den <=
                                         ((unsigned __int128)1 << target) * t->cfg.max_fill_num)
        --target;
    } else {
      do {
        ++target;
      } while (target < 34 && !fits(t, t->known_live + b, 1ull << target));
    }
  }
  if (move) {
    // live records fit in what the pool holds now; keep slack for growth
    const uint64_t cap = std::max<uint64_t>(t->pool_cap, 2 * (pused + bytes));
    if (target > t->log2c + 1 && t->known_live > 0) {
      // a chain of doublings, like the word tables
      while (t->log2c < target) {
        rc = migrate(t, t->log2c + 1, cap, s);
        if (rc) return rc;
      }
    } else {
      rc = migrate(t, target, cap, s);
      if (rc) return rc;
    }
  }
  t->pending = b;
  return LPHT_OK;
}

int run(lpht_str_table *t, int kind, const uint8_t *bytes, const uint64_t *offsets, uint64_t n, const uint64_t *vals,
        uint32_t up, uint64_t *vals_out, uint8_t *flags, void *stream) {
  if (!t || up > 1) return LPHT_ERR_INVALID;
  if (n == 0) return LPHT_OK;
  if (!offsets || !bytes || ((uintptr_t)offsets % 8) || (vals && ((uintptr_t)vals % 8)) ||
      (vals_out && ((uintptr_t)vals_out % 8)))
    return LPHT_ERR_INVALID;
  hipStream_t s = (hipStream_t)stream;
  if (hipSetDevice(t->device) != hipSuccess) return LPHT_ERR_DEVICE;
  if (kind == kStrInsert || kind == kStrUpsert) {
    uint64_t o[2];
    hipError_t e = hipMemcpyAsync(&o[0], offsets, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&o[1], offsets + n, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return from_hip(e);
    if (o[1] < o[0]) return LPHT_ERR_INVALID;
    // each record takes at most its length + 11 bytes
    const int rc = grow_before(t, n, (o[1] - o[0]) + 12 * n, s);
    if (rc) return rc;
  }
  StrArgs a{};
  a.cells = t->cells;
  a.log2c = t->log2c;
  a.up = up;
  a.pool = t->pool;
  a.pool_cap = t->pool_cap;
  a.ctl = t->ctl;
  a.crc_hi = t->cfg.seed_hi;
  a.crc_lo = t->cfg.seed_lo;
  a.bytes = bytes;
  a.offsets = offsets;
  a.n = n;
  a.vals = vals;
  a.vals_out = vals_out;
  a.flags = flags;
  return from_hip(launch_str_op(kind, a, t->num_cus, s));
}

}  // namespace

extern "C" {

void lpht_str_config_default(lpht_str_config *cfg) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->log2_capacity = 12;
  cfg->seed_hi = 0x9E3779B9u;
  cfg->seed_lo = 0xFFFFFFFFu;
  cfg->max_fill_num = 1;
  cfg->max_fill_den = 2;
  cfg->pool_bytes = 1 << 20;
}

int lpht_str_create(const lpht_str_config *cfg, void *stream, lpht_str_table **out) {
  if (!cfg || !out) return LPHT_ERR_INVALID;
  *out = nullptr;
  if (cfg->log2_capacity < 6 || cfg->log2_capacity > 34 || cfg->max_fill_num == 0 ||
      cfg->max_fill_num > cfg->max_fill_den || cfg->pool_bytes < 64 || cfg->auto_grow > 1 || cfg->reserved[0] ||
      cfg->reserved[1])
    return LPHT_ERR_INVALID;
  lpht_str_table *t = new (std::nothrow) lpht_str_table();
  if (!t) return LPHT_ERR_OOM;
  t->cfg = *cfg;
  hipStream_t s = (hipStream_t)stream;
  int ncu = 0;
  if (hipGetDevice(&t->device) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, t->device) != hipSuccess) {
    delete t;
    return LPHT_ERR_DEVICE;
  }
  t->num_cus = (uint32_t)ncu;
  t->log2c = t->log2_min = cfg->log2_capacity;
  t->pool_cap = (cfg->pool_bytes + 7) & ~7ull;
  const size_t nb = (size_t)16 << t->log2c;
  t->cells = (uint64_t *)alloc(t, nb, s);
  t->pool = (uint8_t *)alloc(t, t->pool_cap, s);
  t->ctl = (StrCtl *)alloc(t, sizeof(StrCtl), s);
  hipError_t e = (t->cells && t->pool && t->ctl) ? hipSuccess : hipErrorOutOfMemory;
  if (e == hipSuccess) e = launch_fill_zero(t->cells, nb, fill_cfg(t), s);
  if (e == hipSuccess) e = launch_fill_zero(t->ctl, sizeof(StrCtl), fill_cfg(t), s);
  if (e == hipSuccess) e = launch_str_init(t->ctl, s);
  if (e != hipSuccess) {
    release(t->cells, s);
    release(t->pool, s);
    release(t->ctl, s);
    delete t;
    return e == hipErrorOutOfMemory ? LPHT_ERR_OOM : from_hip(e);
  }
  *out = t;
  return LPHT_OK;
}

int lpht_str_destroy(lpht_str_table *t, void *stream) {
  if (!t) return LPHT_OK;
  hipStream_t s = (hipStream_t)stream;
  (void)hipSetDevice(t->device);
  release(t->cells, s);
  release(t->pool, s);
  release(t->ctl, s);
  delete t;
  return LPHT_OK;
}

int lpht_str_insert(lpht_str_table *t, const uint8_t *bytes, const uint64_t *offsets, uint64_t n,
                    const uint64_t *vals, uint8_t *flags, void *stream) {
  return run(t, kStrInsert, bytes, offsets, n, vals, 0, nullptr, flags, stream);
}

int lpht_str_insert_or_update(lpht_str_table *t, const uint8_t *bytes, const uint64_t *offsets, uint64_t n,
                              const uint64_t *vals, uint32_t up, uint8_t *flags, void *stream) {
  return run(t, kStrUpsert, bytes, offsets, n, vals, up, nullptr, flags, stream);
}

int lpht_str_find(lpht_str_table *t, const uint8_t *bytes, const uint64_t *offsets, uint64_t n,
                  uint64_t *vals_out, uint8_t *found, void *stream) {
  return run(t, kStrFind, bytes, offsets, n, nullptr, 0, vals_out, found, stream);
}

int lpht_str_erase(lpht_str_table *t, const uint8_t *bytes, const uint64_t *offsets, uint64_t n, uint8_t *flags,
                   void *stream) {
  return run(t, kStrErase, bytes, offsets, n, nullptr, 0, nullptr, flags, stream);
}

int lpht_str_count(lpht_str_table *t, uint64_t *used, uint64_t *live, void *stream) {
  if (!t) return LPHT_ERR_INVALID;
  if (hipSetDevice(t->device) != hipSuccess) return LPHT_ERR_DEVICE;
  const int rc = recount(t, (hipStream_t)stream);
  if (rc) return rc;
  if (used) *used = t->known_used;
  if (live) *live = t->known_live;
  return LPHT_OK;
}

int lpht_str_capacity(lpht_str_table *t, uint64_t *cells, uint64_t *pool_used, uint64_t *pool_cap, void *stream) {
  if (!t) return LPHT_ERR_INVALID;
  if (hipSetDevice(t->device) != hipSuccess) return LPHT_ERR_DEVICE;
  int rc = LPHT_OK;
  const uint64_t pu = pool_cursor(t, (hipStream_t)stream, &rc);
  if (rc) return rc;
  if (cells) *cells = 1ull << t->log2c;
  if (pool_used) *pool_used = pu;
  if (pool_cap) *pool_cap = t->pool_cap;
  return LPHT_OK;
}

int lpht_str_grow(lpht_str_table *t, uint32_t log2_new_capacity, void *stream) {
  if (!t || log2_new_capacity < 6 || log2_new_capacity > 34) return LPHT_ERR_INVALID;
  hipStream_t s = (hipStream_t)stream;
  if (hipSetDevice(t->device) != hipSuccess) return LPHT_ERR_DEVICE;
  int rc = recount(t, s);
  if (rc) return rc;
  const uint64_t pu = pool_cursor(t, s, &rc);
  if (rc) return rc;
  return migrate(t, log2_new_capacity, std::max<uint64_t>(t->pool_cap, pu), s);
}

int lpht_str_export(lpht_str_table *t, void *cells_dst, void *pool_dst, uint64_t pool_dst_bytes, void *stream) {
  if (!t || !cells_dst) return LPHT_ERR_INVALID;
  hipStream_t s = (hipStream_t)stream;
  if (hipSetDevice(t->device) != hipSuccess) return LPHT_ERR_DEVICE;
  hipError_t e = hipMemcpyAsync(cells_dst, t->cells, (size_t)16 << t->log2c, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess && pool_dst && pool_dst_bytes)
    e = hipMemcpyAsync(pool_dst, t->pool, std::min<uint64_t>(pool_dst_bytes, t->pool_cap), hipMemcpyDeviceToDevice,
                       s);
  return from_hip(e);
}

int lpht_str_status(lpht_str_table *t, void *stream) {
  if (!t) return LPHT_ERR_INVALID;
  hipStream_t s = (hipStream_t)stream;
  if (hipSetDevice(t->device) != hipSuccess) return LPHT_ERR_DEVICE;
  unsigned int err = 0;
  hipError_t e = hipMemcpyAsync(&err, &t->ctl->err, sizeof(err), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return from_hip(e);
  if (err) {
    const unsigned int zero = 0;
    e = hipMemcpyAsync(&t->ctl->err, &zero, sizeof(zero), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return from_hip(e);
  }
  return (err & kErrFull) ? LPHT_ERR_FULL : LPHT_OK;
}

}  // extern "C"
