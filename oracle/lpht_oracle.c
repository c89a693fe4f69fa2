/*
 * Sequential CPU oracle for the linear-probing hash table of Maier, Sanders and
 * Dementiev, "Concurrent Hash Tables: Fast and General(?)!" (arXiv 1601.04017).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg do.  It shares no source, header or table with the HIP path.
 *
 * It is deliberately plain: one table, no atomics, no blocking, every bulk call
 * applies its operations one after another in index order.  The paper's own
 * "sequential variants" are tables of exactly this kind (Sec. 8.1), and since
 * the concurrent table is linearizable (Sec. 4) a bulk call of the concurrent
 * table has the same outcome as this one up to the order of operations.
 *
 * Cell layouts (same bytes as the device table so exported arrays compare
 * directly):
 *   PACKED32 (layout 0): one u64 word per cell, key in bits 0..31, value in
 *                        bits 32..63; the all-zero word is an empty cell.
 *   KV64     (layout 1): two u64 words per cell, key then value.
 * Reserved keys: 0 = empty_key, 1 = del_key (tombstone) (Sec. 4 "Deletions",
 * Sec. 5.6 names the two special keys).
 *
 * Per-operation result codes: 1 = true, 0 = false, 0xFE = reserved key,
 * 0xFF = bounded table full.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PACKED32 0
#define ORC_KV64 1

#define ORC_EMPTY 0ull
#define ORC_TOMB 1ull

#define ORC_ASSIGN 0
#define ORC_ADD 1

#define ORC_FLAG_RESERVED 0xFE
#define ORC_FLAG_FULL 0xFF

#define ORC_HASH_CRC32C_PAIR 0
#define ORC_HASH_MULSHIFT 1

#define ORC_STICKY_FULL 1
#define ORC_STICKY_RESERVED 2

/* ------------------------------------------------------------------------- */
/* Hash (Sec. 8.3): two CRC-32C computations with different seeds give the    */
/* upper and lower 32 bits of the 64-bit hash value.                          */
/* ------------------------------------------------------------------------- */

/* CRC-32C register update over a byte string, bit by bit from the
 * Castagnoli polynomial in reflected form (0x82F63B78).  No initial or final
 * inversion: this is the register update that the x86 crc32 instruction the
 * paper uses performs, starting from the register value `reg`. */
uint32_t orc_crc32c_bytes(uint32_t reg, const uint8_t *buf, uint64_t len) {
  for (uint64_t i = 0; i < len; ++i) {
    reg ^= (uint32_t)buf[i];
    for (int bit = 0; bit < 8; ++bit) {
      if (reg & 1u)
        reg = (reg >> 1) ^ 0x82F63B78u;
      else
        reg = reg >> 1;
    }
  }
  return reg;
}

/* CRC-32C update over the `nbytes` little-endian bytes of a key word. */
uint32_t orc_crc32c_word(uint32_t reg, uint64_t x, int nbytes) {
  uint8_t b[8];
  for (int i = 0; i < nbytes; ++i) b[i] = (uint8_t)(x >> (8 * i));
  return orc_crc32c_bytes(reg, b, (uint64_t)nbytes);
}

/* h(x) = CRC(seed_hi, x) * 2^32 + CRC(seed_lo, x). */
uint64_t orc_hash(uint64_t key, int key_bytes, uint32_t seed_hi, uint32_t seed_lo) {
  uint64_t hi = orc_crc32c_word(seed_hi, key, key_bytes);
  uint64_t lo = orc_crc32c_word(seed_lo, key, key_bytes);
  return (hi << 32) | lo;
}

/* Multiplicative hashing, the alternative hash function of a table created
 * with ORC_HASH_MULSHIFT: h(x) = (a * x) mod 2^64 for an odd multiplier a
 * (the textbook multiply-shift scheme of Dietzfelbinger et al., 1997, whose
 * "shift" is the scaling map below: the position keeps the top bits).  The
 * paper leaves the hash function open apart from its CRC-32C choice
 * (Sec. 8.3).  With an odd multiplier the map is a bijection of the 64-bit
 * keys. */
uint64_t orc_mulshift(uint64_t key, uint64_t mul) { return key * mul; }

/* Scaling map of Sec. 5.3.1: h_c(x) = floor(h(x) * c / U) with U = 2^64 and
 * c = 2^log2c, i.e. the top log2c bits of h. */
uint64_t orc_home(uint64_t h, uint32_t log2c) {
  if (log2c == 0) return 0;
  return h >> (64 - log2c);
}

/* ------------------------------------------------------------------------- */
/* The table                                                                  */
/* ------------------------------------------------------------------------- */

typedef struct orc_table {
  int layout;
  uint32_t log2c;
  uint32_t log2_min; /* the capacity it was created with: no automatic shrink below */
  uint64_t cap;
  uint64_t *cells;
  uint32_t seed_hi, seed_lo;
  int hash_kind; /* ORC_HASH_CRC32C_PAIR (default) or ORC_HASH_MULSHIFT */
  uint64_t mul;  /* odd multiplier of ORC_HASH_MULSHIFT */
  uint32_t alpha_num, alpha_den;
  int auto_grow;
  uint64_t used; /* non-empty cells (live keys and tombstones) */
  uint64_t live; /* live keys */
  int sticky;
  uint64_t migrations;
  /* Full key space (Sec. 5.6): keys empty_key and del_key live in two
   * special slots outside the cell array instead of being reserved. */
  int full_keys;
  int sp_present[2];
  uint64_t sp_val[2];
} orc_table;

static int key_bytes(const orc_table *t) { return t->layout == ORC_PACKED32 ? 4 : 8; }

static uint64_t key_at(const orc_table *t, const uint64_t *cells, uint64_t i) {
  if (t->layout == ORC_PACKED32) return cells[i] & 0xFFFFFFFFull;
  return cells[2 * i];
}

static uint64_t val_at(const orc_table *t, const uint64_t *cells, uint64_t i) {
  if (t->layout == ORC_PACKED32) return cells[i] >> 32;
  return cells[2 * i + 1];
}

static void set_cell(const orc_table *t, uint64_t *cells, uint64_t i, uint64_t k, uint64_t v) {
  if (t->layout == ORC_PACKED32) {
    cells[i] = (k & 0xFFFFFFFFull) | ((v & 0xFFFFFFFFull) << 32);
  } else {
    cells[2 * i] = k;
    cells[2 * i + 1] = v;
  }
}

static uint64_t words_per_cell(const orc_table *t) { return t->layout == ORC_PACKED32 ? 1 : 2; }

/* The table's 64-bit hash of key k. */
static uint64_t table_hash(const orc_table *t, uint64_t k) {
  if (t->hash_kind == ORC_HASH_MULSHIFT) return orc_mulshift(k, t->mul);
  return orc_hash(k, key_bytes(t), t->seed_hi, t->seed_lo);
}

static uint64_t home_of(const orc_table *t, uint64_t k, uint32_t log2c) {
  return orc_home(table_hash(t, k), log2c);
}

/* Wrapping update function `up` of Algorithm 1: overwrite or add (modulo the
 * value width). */
static uint64_t apply_up(const orc_table *t, uint64_t cur, uint64_t d, int op) {
  uint64_t r = (op == ORC_ADD) ? cur + d : d;
  if (t->layout == ORC_PACKED32) r &= 0xFFFFFFFFull;
  return r;
}

orc_table *orc_create(int layout, uint32_t log2c, uint32_t seed_hi, uint32_t seed_lo,
                      uint32_t alpha_num, uint32_t alpha_den, int auto_grow) {
  if (layout != ORC_PACKED32 && layout != ORC_KV64) return NULL;
  if (log2c < 1 || log2c > 40) return NULL;
  if (alpha_num == 0 || alpha_den == 0 || alpha_num > alpha_den) return NULL;
  orc_table *t = (orc_table *)calloc(1, sizeof(orc_table));
  if (!t) return NULL;
  t->layout = layout;
  t->log2c = log2c;
  t->log2_min = log2c;
  t->cap = 1ull << log2c;
  t->seed_hi = seed_hi;
  t->seed_lo = seed_lo;
  t->alpha_num = alpha_num;
  t->alpha_den = alpha_den;
  t->auto_grow = auto_grow;
  /* Sec. 4 "Initialization": every key starts as empty_key; values start 0. */
  t->cells = (uint64_t *)calloc(t->cap * words_per_cell(t), sizeof(uint64_t));
  if (!t->cells) {
    free(t);
    return NULL;
  }
  return t;
}

void orc_destroy(orc_table *t) {
  if (!t) return;
  free(t->cells);
  free(t);
}

uint64_t orc_capacity(const orc_table *t) { return t->cap; }
uint32_t orc_log2_capacity(const orc_table *t) { return t->log2c; }
uint64_t orc_migrations(const orc_table *t) { return t->migrations; }

/* Counts include the special slots that hold a key. */
void orc_counts(const orc_table *t, uint64_t *used, uint64_t *live) {
  uint64_t sp = (uint64_t)t->sp_present[0] + (uint64_t)t->sp_present[1];
  *used = t->used + sp;
  *live = t->live + sp;
}

/* Switches the full key space on or off (a table with no special key). */
int orc_set_full_keys(orc_table *t, int on) {
  if (t->sp_present[0] || t->sp_present[1]) return -1;
  t->full_keys = on ? 1 : 0;
  return 0;
}

/* Selects the hash function of an empty table: ORC_HASH_CRC32C_PAIR (the
 * seeds given at creation) or ORC_HASH_MULSHIFT with the odd multiplier
 * `mul`.  Returns -1 for a table that holds elements, an unknown kind or an
 * even multiplier. */
int orc_set_hash(orc_table *t, int kind, uint64_t mul) {
  if (t->used || t->sp_present[0] || t->sp_present[1]) return -1;
  if (kind == ORC_HASH_CRC32C_PAIR) {
    t->hash_kind = kind;
    t->mul = 0;
    return 0;
  }
  if (kind != ORC_HASH_MULSHIFT || (mul & 1u) == 0) return -1;
  t->hash_kind = kind;
  t->mul = mul;
  return 0;
}

/* Operations on a special slot (k is 0 or 1), with the same results as the
 * cell operations: a slot is one cell that only key k can use. */
static uint8_t sp_insert(orc_table *t, uint64_t k, uint64_t v, int is_upsert, int op) {
  if (!t->sp_present[k]) {
    t->sp_present[k] = 1;
    t->sp_val[k] = apply_up(t, 0, v, ORC_ASSIGN);
    return 1;
  }
  if (is_upsert) t->sp_val[k] = apply_up(t, t->sp_val[k], v, op);
  return 0;
}

/* Returns the sticky error bits and clears them. */
int orc_status(orc_table *t) {
  int s = t->sticky;
  t->sticky = 0;
  return s;
}

void orc_export(const orc_table *t, uint64_t *dst) {
  memcpy(dst, t->cells, t->cap * words_per_cell(t) * sizeof(uint64_t));
}

/* Replaces the cell array by a copy of `src` (2^log2c cells) and recounts. */
int orc_import(orc_table *t, const uint64_t *src, uint32_t log2c) {
  if (log2c < 1 || log2c > 40) return -1;
  uint64_t cap = 1ull << log2c;
  uint64_t *cells = (uint64_t *)malloc(cap * words_per_cell(t) * sizeof(uint64_t));
  if (!cells) return -2;
  memcpy(cells, src, cap * words_per_cell(t) * sizeof(uint64_t));
  free(t->cells);
  t->cells = cells;
  t->log2c = log2c;
  t->cap = cap;
  t->used = 0;
  t->live = 0;
  for (uint64_t i = 0; i < cap; ++i) {
    uint64_t k = key_at(t, cells, i);
    if (k != ORC_EMPTY) t->used++;
    if (k != ORC_EMPTY && k != ORC_TOMB) t->live++;
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Single operations (Sec. 4; Algorithm 1 and its insert/update variants;    */
/* tombstone deletion of Sec. 5.4).                                           */
/* ------------------------------------------------------------------------- */

/* insert(k,d): scan from h_c(k); an empty cell receives the element (true);
 * an equal key means the key is present (false).  Tombstones and other keys
 * are skipped, so tombstones are never reused. */
static uint8_t op_insert(orc_table *t, uint64_t k, uint64_t v) {
  if (t->full_keys && k <= ORC_TOMB) return sp_insert(t, k, v, 0, ORC_ASSIGN);
  if (k == ORC_EMPTY || k == ORC_TOMB) {
    t->sticky |= ORC_STICKY_RESERVED;
    return ORC_FLAG_RESERVED;
  }
  uint64_t i = home_of(t, k, t->log2c);
  for (uint64_t probes = 0; probes < t->cap; ++probes) {
    uint64_t cur = key_at(t, t->cells, i);
    if (cur == ORC_EMPTY) {
      set_cell(t, t->cells, i, k, v);
      t->used++;
      t->live++;
      return 1;
    }
    if (cur == k) return 0;
    i = (i + 1) & (t->cap - 1);
  }
  t->sticky |= ORC_STICKY_FULL;
  return ORC_FLAG_FULL;
}

/* insertOrUpdate(k,d,up): as insert, but an equal key gets
 * value := up(value, d); returns true iff a new key was inserted. */
static uint8_t op_insert_or_update(orc_table *t, uint64_t k, uint64_t d, int op) {
  if (t->full_keys && k <= ORC_TOMB) return sp_insert(t, k, d, 1, op);
  if (k == ORC_EMPTY || k == ORC_TOMB) {
    t->sticky |= ORC_STICKY_RESERVED;
    return ORC_FLAG_RESERVED;
  }
  uint64_t i = home_of(t, k, t->log2c);
  for (uint64_t probes = 0; probes < t->cap; ++probes) {
    uint64_t cur = key_at(t, t->cells, i);
    if (cur == ORC_EMPTY) {
      set_cell(t, t->cells, i, k, apply_up(t, 0, d, ORC_ASSIGN));
      t->used++;
      t->live++;
      return 1;
    }
    if (cur == k) {
      set_cell(t, t->cells, i, k, apply_up(t, val_at(t, t->cells, i), d, op));
      return 0;
    }
    i = (i + 1) & (t->cap - 1);
  }
  t->sticky |= ORC_STICKY_FULL;
  return ORC_FLAG_FULL;
}

/* update(k,d,up): false if the key is absent, else value := up(value, d). */
static uint8_t op_update(orc_table *t, uint64_t k, uint64_t d, int op) {
  if (t->full_keys && k <= ORC_TOMB) {
    if (!t->sp_present[k]) return 0;
    t->sp_val[k] = apply_up(t, t->sp_val[k], d, op);
    return 1;
  }
  if (k == ORC_EMPTY || k == ORC_TOMB) {
    t->sticky |= ORC_STICKY_RESERVED;
    return ORC_FLAG_RESERVED;
  }
  uint64_t i = home_of(t, k, t->log2c);
  for (uint64_t probes = 0; probes < t->cap; ++probes) {
    uint64_t cur = key_at(t, t->cells, i);
    if (cur == ORC_EMPTY) return 0;
    if (cur == k) {
      set_cell(t, t->cells, i, k, apply_up(t, val_at(t, t->cells, i), d, op));
      return 1;
    }
    i = (i + 1) & (t->cap - 1);
  }
  return 0;
}

/* find(k): a copy of the stored value if the key is present. */
static uint8_t op_find(orc_table *t, uint64_t k, uint64_t *val) {
  *val = 0;
  if (t->full_keys && k <= ORC_TOMB) {
    if (!t->sp_present[k]) return 0;
    *val = t->sp_val[k];
    return 1;
  }
  if (k == ORC_EMPTY || k == ORC_TOMB) {
    t->sticky |= ORC_STICKY_RESERVED;
    return ORC_FLAG_RESERVED;
  }
  uint64_t i = home_of(t, k, t->log2c);
  for (uint64_t probes = 0; probes < t->cap; ++probes) {
    uint64_t cur = key_at(t, t->cells, i);
    if (cur == ORC_EMPTY) return 0;
    if (cur == k) {
      *val = val_at(t, t->cells, i);
      return 1;
    }
    i = (i + 1) & (t->cap - 1);
  }
  return 0;
}

/* Tombstone delete: the key becomes del_key, the value stays. */
static uint8_t op_erase(orc_table *t, uint64_t k) {
  if (t->full_keys && k <= ORC_TOMB) {
    if (!t->sp_present[k]) return 0;
    t->sp_present[k] = 0;
    t->sp_val[k] = 0;
    return 1;
  }
  if (k == ORC_EMPTY || k == ORC_TOMB) {
    t->sticky |= ORC_STICKY_RESERVED;
    return ORC_FLAG_RESERVED;
  }
  uint64_t i = home_of(t, k, t->log2c);
  for (uint64_t probes = 0; probes < t->cap; ++probes) {
    uint64_t cur = key_at(t, t->cells, i);
    if (cur == ORC_EMPTY) return 0;
    if (cur == k) {
      set_cell(t, t->cells, i, ORC_TOMB, val_at(t, t->cells, i));
      t->live--;
      return 1;
    }
    i = (i + 1) & (t->cap - 1);
  }
  return 0;
}

/* Number of cells a find for k inspects, the terminating cell included. */
uint64_t orc_probe_count(const orc_table *t, uint64_t k) {
  uint64_t i = home_of(t, k, t->log2c);
  uint64_t probes = 0;
  while (probes < t->cap) {
    uint64_t cur = key_at(t, t->cells, i);
    probes++;
    if (cur == ORC_EMPTY || cur == k) break;
    i = (i + 1) & (t->cap - 1);
  }
  return probes;
}

/* ------------------------------------------------------------------------- */
/* Migration (Sec. 5.3.1: growing with factor gamma = new/old >= 1, and      */
/* shrinking, gamma < 1) and cleanup of tombstones by migration (Sec. 5.4).  */
/* ------------------------------------------------------------------------- */

/* The sequential migration: scan the old table once, starting just after an
 * empty cell so that every cluster (the one that wraps from the last cell to
 * cell 0 included) is visited contiguously in old-array order, and insert
 * every live element into the new table with the ordinary linear-probing
 * rule.  Tombstones are dropped.  A table without any empty cell is scanned
 * from cell 0.  This is the sequential order whose placement the
 * block-parallel migration reproduces (Lemma 1). */
int orc_migrate(orc_table *t, uint32_t log2_new) {
  if (log2_new < 1 || log2_new > 40) return -1;
  uint64_t newcap = 1ull << log2_new;
  /* a smaller target must keep an empty cell; a table of the same or a
   * larger size holds its live elements as they are */
  if (log2_new < t->log2c && t->live >= newcap) return -3;
  uint64_t *nc = (uint64_t *)calloc(newcap * words_per_cell(t), sizeof(uint64_t));
  if (!nc) return -2;
  uint64_t e = t->cap - 1;
  for (uint64_t i = 0; i < t->cap; ++i) {
    if (key_at(t, t->cells, i) == ORC_EMPTY) {
      e = i;
      break;
    }
  }
  uint64_t moved = 0;
  for (uint64_t j = 1; j <= t->cap; ++j) {
    uint64_t i = (e + j) & (t->cap - 1);
    uint64_t k = key_at(t, t->cells, i);
    if (k == ORC_EMPTY || k == ORC_TOMB) continue;
    uint64_t v = val_at(t, t->cells, i);
    uint64_t p = home_of(t, k, log2_new);
    while (key_at(t, nc, p) != ORC_EMPTY) p = (p + 1) & (newcap - 1);
    set_cell(t, nc, p, k, v);
    moved++;
  }
  free(t->cells);
  t->cells = nc;
  t->log2c = log2_new;
  t->cap = newcap;
  t->used = moved;
  t->live = moved;
  t->migrations++;
  return 0;
}

/* x <= alpha * c, with alpha = num/den, in exact integer arithmetic. */
static int within_fill(const orc_table *t, uint64_t x, uint64_t c) {
  return (unsigned __int128)x * t->alpha_den <= (unsigned __int128)c * t->alpha_num;
}

/* Growth rule applied before a batch of b operations that may insert
 * (bulk insertion by pre-growing, Sec. 5.5; trigger at fill factor alpha,
 * doubling, Sec. 5.3.2 and Sec. 7; the migration is triggered by the
 * non-empty cells I and its size chosen from the live elements I - D,
 * Sec. 5.4):
 *   used + b <= alpha*c            -> nothing;
 *   live + b <= alpha*c/2          -> migrate once to c' = c / 2^s, the
 *                                     smallest s >= 0 with c' >= the created
 *                                     capacity such that halving once more
 *                                     would give live + b > alpha*c'/2
 *                                     (s = 0: gamma = 1, tombstones dropped;
 *                                     s > 0: a shrink);
 *   otherwise                      -> migrate with gamma = 2, repeated while
 *                                     live + b > alpha*c. */
static int fits_quarter(const orc_table *t, uint64_t x, uint64_t c) {
  /* x <= alpha * c / 4 */
  return (unsigned __int128)x * 4 * t->alpha_den <= (unsigned __int128)c * t->alpha_num;
}

static int grow_before_batch(orc_table *t, uint64_t b) {
  if (!t->auto_grow || b == 0) return 0;
  if (within_fill(t, t->used + b, t->cap)) return 0;
  if ((unsigned __int128)(t->live + b) * 2 * t->alpha_den <= (unsigned __int128)t->cap * t->alpha_num) {
    uint32_t target = t->log2c;
    while (target > t->log2_min && fits_quarter(t, t->live + b, 1ull << target)) --target;
    return orc_migrate(t, target);
  }
  do {
    if (t->log2c >= 40) return -1;
    int rc = orc_migrate(t, t->log2c + 1);
    if (rc) return rc;
  } while (!within_fill(t, t->live + b, t->cap));
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Bulk calls: index order.  Keys and values are u32 for PACKED32 and u64    */
/* for KV64.  `vals` may be NULL, meaning every operation carries value 1.   */
/* `flags` may be NULL.                                                       */
/* ------------------------------------------------------------------------- */

static uint64_t load_word(const orc_table *t, const void *a, uint64_t i) {
  if (t->layout == ORC_PACKED32) return ((const uint32_t *)a)[i];
  return ((const uint64_t *)a)[i];
}

static void store_word(const orc_table *t, void *a, uint64_t i, uint64_t v) {
  if (t->layout == ORC_PACKED32)
    ((uint32_t *)a)[i] = (uint32_t)v;
  else
    ((uint64_t *)a)[i] = v;
}

int orc_insert(orc_table *t, const void *keys, const void *vals, uint64_t n, uint8_t *flags) {
  int rc = grow_before_batch(t, n);
  if (rc) return rc;
  for (uint64_t i = 0; i < n; ++i) {
    uint64_t v = vals ? load_word(t, vals, i) : 1;
    uint8_t f = op_insert(t, load_word(t, keys, i), v);
    if (flags) flags[i] = f;
  }
  return 0;
}

int orc_insert_or_update(orc_table *t, const void *keys, const void *vals, uint64_t n, int op,
                         uint8_t *flags) {
  int rc = grow_before_batch(t, n);
  if (rc) return rc;
  for (uint64_t i = 0; i < n; ++i) {
    uint64_t d = vals ? load_word(t, vals, i) : 1;
    uint8_t f = op_insert_or_update(t, load_word(t, keys, i), d, op);
    if (flags) flags[i] = f;
  }
  return 0;
}

int orc_update(orc_table *t, const void *keys, const void *vals, uint64_t n, int op, uint8_t *flags) {
  for (uint64_t i = 0; i < n; ++i) {
    uint64_t d = vals ? load_word(t, vals, i) : 1;
    uint8_t f = op_update(t, load_word(t, keys, i), d, op);
    if (flags) flags[i] = f;
  }
  return 0;
}

int orc_find(orc_table *t, const void *keys, uint64_t n, void *vals_out, uint8_t *found) {
  for (uint64_t i = 0; i < n; ++i) {
    uint64_t v;
    uint8_t f = op_find(t, load_word(t, keys, i), &v);
    if (vals_out) store_word(t, vals_out, i, v);
    if (found) found[i] = f;
  }
  return 0;
}

int orc_erase(orc_table *t, const void *keys, uint64_t n, uint8_t *flags) {
  for (uint64_t i = 0; i < n; ++i) {
    uint8_t f = op_erase(t, load_word(t, keys, i));
    if (flags) flags[i] = f;
  }
  return 0;
}

/* Explicit resize entry: gamma = 2^(log2_new - log2c); equal size is the
 * tombstone cleanup with gamma = 1, a smaller size a shrink (-3 when the live
 * elements would not leave an empty cell). */
int orc_grow(orc_table *t, uint32_t log2_new) { return orc_migrate(t, log2_new); }

/* ------------------------------------------------------------------------- */
/* Bulk build and batched merge by sorting (Sec. 5.5).                        */
/* ------------------------------------------------------------------------- */

/* An element of a sorted batch: its 64-bit hash, key, value and sequence
 * number (0 for an element already in the table, i + 1 for batch entry i). */
typedef struct orc_item {
  uint64_t h, k, v, seq;
} orc_item;

/* The order of Sec. 5.5's sort: by the upper 32 hash bits (they hold every
 * position bit of a table of up to 2^32 cells), then by key, then by sequence
 * number.  For the CRC-32C pair equal upper halves mean equal CRC values and
 * therefore equal lower halves, so this is the order of the whole 64-bit
 * hash; for the multiplicative hash it breaks ties of the upper bits by key. */
static int item_cmp(const void *a, const void *b) {
  const orc_item *x = (const orc_item *)a, *y = (const orc_item *)b;
  if ((x->h >> 32) != (y->h >> 32)) return (x->h >> 32) < (y->h >> 32) ? -1 : 1;
  if (x->k != y->k) return x->k < y->k ? -1 : 1;
  if (x->seq != y->seq) return x->seq < y->seq ? -1 : 1;
  return 0;
}

/* Builds the table from a batch (keep_old = 0: the old contents are dropped)
 * or merges the batch into it (keep_old = 1), following the sort-based bulk
 * operation of Sec. 5.5:
 *   1. the elements (the table's live elements first, then the batch in index
 *      order) are sorted by their hash value (its upper 32 bits, see
 *      item_cmp); equal hashes by key, equal keys by sequence number;
 *   2. among equal keys all but the last are removed; with ORC_ADD the kept
 *      element carries the wrapping sum of all their values, with ORC_ASSIGN
 *      its own value (the batch's last occurrence overrides the table);
 *   3. the result is inserted into an empty table in that sorted order by
 *      ordinary linear probing, so each element starts its search for a free
 *      cell at the larger of its home and the previous element's position.
 * vals NULL means every value is 1.  Reserved keys are skipped (sticky
 * RESERVED).  The capacity: unchanged for a bounded table; with auto growth
 * doubled while (kept live elements + n) exceeds alpha * capacity (a + b is
 * an upper bound of the new size, Sec. 5.5), never shrunk.  Returns -3
 * (sticky FULL, table unchanged) when the distinct keys exceed the capacity,
 * -2 when out of memory. */
int orc_bulk_merge(orc_table *t, const void *keys, const void *vals, uint64_t n, int op, int keep_old) {
  uint64_t old_n = keep_old ? t->live : 0;
  orc_item *it = (orc_item *)malloc((old_n + n + 1) * sizeof(orc_item));
  if (!it) return -2;
  uint64_t m = 0;
  if (keep_old)
    for (uint64_t i = 0; i < t->cap; ++i) {
      uint64_t k = key_at(t, t->cells, i);
      if (k == ORC_EMPTY || k == ORC_TOMB) continue;
      it[m].h = table_hash(t, k);
      it[m].k = k;
      it[m].v = val_at(t, t->cells, i);
      it[m].seq = 0;
      ++m;
    }
  /* full key space: the special slots take the batch's keys 0 and 1 in
   * index order (a build starts them empty); decided after the capacity
   * check below, so a refused call changes nothing */
  int spp[2] = {keep_old ? t->sp_present[0] : 0, keep_old ? t->sp_present[1] : 0};
  uint64_t spv[2] = {keep_old ? t->sp_val[0] : 0, keep_old ? t->sp_val[1] : 0};
  for (uint64_t i = 0; i < n; ++i) {
    uint64_t k = load_word(t, keys, i);
    if (k == ORC_EMPTY || k == ORC_TOMB) {
      if (t->full_keys) {
        uint64_t v = vals ? load_word(t, vals, i) : 1;
        spv[k] = (op == ORC_ADD) ? apply_up(t, spp[k] ? spv[k] : 0, v, ORC_ADD) : apply_up(t, 0, v, ORC_ASSIGN);
        spp[k] = 1;
        continue;
      }
      t->sticky |= ORC_STICKY_RESERVED;
      continue;
    }
    it[m].h = table_hash(t, k);
    it[m].k = k;
    it[m].v = vals ? load_word(t, vals, i) : 1;
    it[m].seq = i + 1;
    ++m;
  }
  qsort(it, m, sizeof(orc_item), item_cmp);
  uint64_t d = 0;
  for (uint64_t i = 0; i < m; ++i) {
    if (d > 0 && it[d - 1].k == it[i].k) {
      it[d - 1].v = (op == ORC_ADD) ? apply_up(t, it[d - 1].v, it[i].v, ORC_ADD) : it[i].v;
      it[d - 1].seq = it[i].seq;
    } else {
      it[d++] = it[i];
    }
  }
  uint32_t log2c = t->log2c;
  if (t->auto_grow)
    while (!within_fill(t, old_n + n, 1ull << log2c)) {
      if (log2c >= 40) {
        free(it);
        return -1;
      }
      ++log2c;
    }
  uint64_t cap = 1ull << log2c;
  if (d > cap) {
    free(it);
    t->sticky |= ORC_STICKY_FULL;
    return -3;
  }
  uint64_t *cells = (uint64_t *)calloc(cap * words_per_cell(t), sizeof(uint64_t));
  if (!cells) {
    free(it);
    return -2;
  }
  for (uint64_t j = 0; j < d; ++j) {
    uint64_t i = orc_home(it[j].h, log2c);
    while (key_at(t, cells, i) != ORC_EMPTY) i = (i + 1) & (cap - 1);
    set_cell(t, cells, i, it[j].k, it[j].v);
  }
  free(it);
  free(t->cells);
  t->cells = cells;
  t->log2c = log2c;
  t->cap = cap;
  t->used = t->live = d;
  for (int q = 0; q < 2; ++q) {
    t->sp_present[q] = spp[q];
    t->sp_val[q] = spv[q];
  }
  return 0;
}

/* Hash of many keys at once (for test comparisons). */
void orc_hash_bulk(const void *keys, uint64_t n, int key_bytes, uint32_t seed_hi, uint32_t seed_lo,
                   uint64_t *out) {
  for (uint64_t i = 0; i < n; ++i) {
    uint64_t k = key_bytes == 4 ? ((const uint32_t *)keys)[i] : ((const uint64_t *)keys)[i];
    out[i] = orc_hash(k, key_bytes, seed_hi, seed_lo);
  }
}

/* ------------------------------------------------------------------------- */
/* String keys (Sec. 5.7, "Complex Keys"): the same linear-probing table     */
/* whose keys are byte strings.  The oracle keeps its own copies of the       */
/* strings; a cell holds 0 (empty), 1 (tombstone) or 2 + the index of the     */
/* string, and a value.  The hash of a string is the pair of CRC-32C register */
/* updates over its bytes with the two seeds (Sec. 8.3), as for word keys.    */
/* ------------------------------------------------------------------------- */

typedef struct orc_str_table {
  uint32_t log2c, log2_min;
  uint64_t cap;
  uint64_t *ref; /* per cell */
  uint64_t *val;
  uint32_t seed_hi, seed_lo;
  uint32_t alpha_num, alpha_den;
  int auto_grow;
  uint64_t used, live;
  uint8_t **str;
  uint64_t *len;
  uint64_t nstr, strcap;
} orc_str_table;

uint64_t orc_str_hash(const uint8_t *s, uint64_t len, uint32_t seed_hi, uint32_t seed_lo) {
  return ((uint64_t)orc_crc32c_bytes(seed_hi, s, len) << 32) | orc_crc32c_bytes(seed_lo, s, len);
}

orc_str_table *orc_str_create(uint32_t log2c, uint32_t seed_hi, uint32_t seed_lo, uint32_t alpha_num,
                              uint32_t alpha_den, int auto_grow) {
  if (log2c < 1 || log2c > 40 || alpha_num == 0 || alpha_den == 0 || alpha_num > alpha_den) return NULL;
  orc_str_table *t = (orc_str_table *)calloc(1, sizeof(orc_str_table));
  if (!t) return NULL;
  t->log2c = t->log2_min = log2c;
  t->cap = 1ull << log2c;
  t->ref = (uint64_t *)calloc(t->cap, sizeof(uint64_t));
  t->val = (uint64_t *)calloc(t->cap, sizeof(uint64_t));
  t->seed_hi = seed_hi;
  t->seed_lo = seed_lo;
  t->alpha_num = alpha_num;
  t->alpha_den = alpha_den;
  t->auto_grow = auto_grow;
  return t;
}

void orc_str_destroy(orc_str_table *t) {
  if (!t) return;
  for (uint64_t i = 0; i < t->nstr; ++i) free(t->str[i]);
  free(t->str);
  free(t->len);
  free(t->ref);
  free(t->val);
  free(t);
}

uint64_t orc_str_capacity(const orc_str_table *t) { return t->cap; }
void orc_str_counts(const orc_str_table *t, uint64_t *used, uint64_t *live) {
  *used = t->used;
  *live = t->live;
}

static uint64_t str_home(const orc_str_table *t, const uint8_t *s, uint64_t len, uint32_t log2c) {
  return orc_home(orc_str_hash(s, len, t->seed_hi, t->seed_lo), log2c);
}

static int str_eq(const orc_str_table *t, uint64_t r, const uint8_t *s, uint64_t len) {
  uint64_t i = r - 2;
  return t->len[i] == len && (len == 0 || memcmp(t->str[i], s, len) == 0);
}

static int64_t str_keep(orc_str_table *t, const uint8_t *s, uint64_t len) {
  if (t->nstr == t->strcap) {
    uint64_t nc = t->strcap ? 2 * t->strcap : 64;
    uint8_t **ns = (uint8_t **)realloc(t->str, nc * sizeof(uint8_t *));
    if (!ns) return -1;
    t->str = ns;
    uint64_t *nl = (uint64_t *)realloc(t->len, nc * sizeof(uint64_t));
    if (!nl) return -1;
    t->len = nl;
    t->strcap = nc;
  }
  uint8_t *c = (uint8_t *)malloc(len ? len : 1);
  if (!c) return -1;
  if (len) memcpy(c, s, len);
  t->str[t->nstr] = c;
  t->len[t->nstr] = len;
  return (int64_t)(t->nstr++);
}

/* One operation: kind 0 insert, 1 insert-or-update (op), 2 find, 3 erase. */
static uint8_t str_op(orc_str_table *t, int kind, const uint8_t *s, uint64_t len, uint64_t d, int op,
                      uint64_t *out) {
  uint64_t i = str_home(t, s, len, t->log2c);
  if (out) *out = 0;
  for (uint64_t probes = 0; probes < t->cap; ++probes) {
    uint64_t r = t->ref[i];
    if (r == 0) {
      if (kind >= 2) return 0;
      int64_t x = str_keep(t, s, len);
      if (x < 0) return ORC_FLAG_FULL;
      t->ref[i] = (uint64_t)x + 2;
      t->val[i] = d;
      t->used++;
      t->live++;
      return 1;
    }
    if (r != 1 && str_eq(t, r, s, len)) {
      if (kind == 1) t->val[i] = (op == ORC_ADD) ? t->val[i] + d : d;
      if (kind == 2 && out) *out = t->val[i];
      if (kind == 3) {
        t->ref[i] = 1;
        t->live--;
        return 1;
      }
      return kind == 2 ? 1 : 0;
    }
    i = (i + 1) & (t->cap - 1);
  }
  return kind >= 2 ? 0 : ORC_FLAG_FULL;
}

/* The sequential migration of the word table, for string keys. */
static int str_migrate(orc_str_table *t, uint32_t log2_new) {
  uint64_t nc = 1ull << log2_new;
  if (t->live >= nc) return -3;
  uint64_t *nr = (uint64_t *)calloc(nc, sizeof(uint64_t));
  uint64_t *nv = (uint64_t *)calloc(nc, sizeof(uint64_t));
  if (!nr || !nv) {
    free(nr);
    free(nv);
    return -2;
  }
  uint64_t start = 0;
  for (uint64_t i = 0; i < t->cap; ++i)
    if (t->ref[i] == 0) {
      start = (i + 1) & (t->cap - 1);
      break;
    }
  uint64_t moved = 0;
  for (uint64_t q = 0; q < t->cap; ++q) {
    uint64_t i = (start + q) & (t->cap - 1);
    uint64_t r = t->ref[i];
    if (r < 2) continue;
    uint64_t p = str_home(t, t->str[r - 2], t->len[r - 2], log2_new);
    while (nr[p] != 0) p = (p + 1) & (nc - 1);
    nr[p] = r;
    nv[p] = t->val[i];
    ++moved;
  }
  free(t->ref);
  free(t->val);
  t->ref = nr;
  t->val = nv;
  t->cap = nc;
  t->log2c = log2_new;
  t->used = t->live = moved;
  return 0;
}

/* The word table's growth rule before a batch of b insertions. */
static int str_grow_before(orc_str_table *t, uint64_t b) {
  if (!t->auto_grow || b == 0) return 0;
  if ((unsigned __int128)(t->used + b) * t->alpha_den <= (unsigned __int128)t->cap * t->alpha_num) return 0;
  if ((unsigned __int128)(t->live + b) * 2 * t->alpha_den <= (unsigned __int128)t->cap * t->alpha_num) {
    uint32_t target = t->log2c;
    while (target > t->log2_min &&
           (unsigned __int128)(t->live + b) * 4 * t->alpha_den <= ((unsigned __int128)1 << target) * t->alpha_num)
      --target;
    return str_migrate(t, target);
  }
  uint32_t target = t->log2c;
  do {
    ++target;
  } while ((unsigned __int128)(t->live + b) * t->alpha_den > ((unsigned __int128)1 << target) * t->alpha_num);
  while (t->log2c < target) {
    int rc = str_migrate(t, t->log2c + 1);
    if (rc) return rc;
  }
  return 0;
}

/* Bulk calls: string i is bytes[offsets[i] .. offsets[i+1]); vals may be
 * NULL (every value 1).  kind: 0 insert, 1 insert-or-update with op, 2 find
 * (vals_out), 3 erase. */
int orc_str_bulk(orc_str_table *t, int kind, const uint8_t *bytes, const uint64_t *offsets, uint64_t n,
                 const uint64_t *vals, int op, uint64_t *vals_out, uint8_t *flags) {
  if (kind <= 1) {
    int rc = str_grow_before(t, n);
    if (rc) return rc;
  }
  for (uint64_t i = 0; i < n; ++i) {
    uint64_t v = 0;
    uint8_t f = str_op(t, kind, bytes + offsets[i], offsets[i + 1] - offsets[i], vals ? vals[i] : 1, op, &v);
    if (flags) flags[i] = f;
    if (vals_out) vals_out[i] = v;
  }
  return 0;
}

int orc_str_grow(orc_str_table *t, uint32_t log2_new) { return str_migrate(t, log2_new); }

/* Cell i: -1 empty, -2 tombstone, else the stored string's length, copied to
 * buf (up to cap bytes), and its value. */
int64_t orc_str_cell(const orc_str_table *t, uint64_t i, uint8_t *buf, uint64_t cap, uint64_t *val) {
  uint64_t r = t->ref[i];
  *val = t->val[i];
  if (r == 0) return -1;
  if (r == 1) return -2;
  uint64_t len = t->len[r - 2];
  if (buf && len) memcpy(buf, t->str[r - 2], len < cap ? len : cap);
  return (int64_t)len;
}
