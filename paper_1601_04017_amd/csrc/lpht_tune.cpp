// Autotuner of liblpht: times candidate launch shapes on scratch tables and
// returns the fastest (see lpht_autotune in include/lpht.h).
//
// Everything runs through the library's own C ABI on one stream, timed with
// HIP events; each candidate is measured from a table rebuilt to the same
// state with the default shape, so only the timed call differs.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <limits>

#include "lpht_host.h"

using namespace lpht;

namespace {

constexpr uint32_t kWidths[5] = {1, 2, 4, 8, 16};
constexpr uint32_t kBlocks[3] = {256, 512, 1024};
constexpr uint32_t kMigrateBlocks[4] = {256, 512, 1024, 2048};
constexpr double kTie = 0.03;  // relative time difference treated as noise

lpht_tuning default_tuning() {
  lpht_tuning u;
  std::memset(&u, 0, sizeof(u));
  u.block_threads = 256;
  u.group_width = 1;
  u.blocks_per_cu = 8;
  u.migrate_block = 512;
  u.aggregate = 1;
  return u;
}

struct Scratch {
  hipStream_t s = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  void *keys = nullptr, *absent = nullptr, *present = nullptr, *vals = nullptr;
  uint8_t *found = nullptr;
  lpht_table *t = nullptr;
  ~Scratch() {
    if (t) lpht_destroy(t, (void *)s);
    (void)hipStreamSynchronize(s);
    for (void *p : {keys, absent, present, vals, (void *)found})
      if (p) (void)hipFree(p);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

// Runs `f` between two events on the scratch stream; returns the elapsed ms
// (or +inf when a call failed).
template <typename F>
double timed(Scratch &x, F f) {
  if (hipEventRecord(x.ev[0], x.s) != hipSuccess) return std::numeric_limits<double>::infinity();
  const int rc = f();
  if (hipEventRecord(x.ev[1], x.s) != hipSuccess || hipEventSynchronize(x.ev[1]) != hipSuccess || rc)
    return std::numeric_limits<double>::infinity();
  float ms = 0;
  if (hipEventElapsedTime(&ms, x.ev[0], x.ev[1]) != hipSuccess) return std::numeric_limits<double>::infinity();
  return ms;
}

int make_table(Scratch &x, uint32_t layout, uint32_t log2c) {
  if (x.t) {
    lpht_destroy(x.t, (void *)x.s);
    x.t = nullptr;
  }
  lpht_config cfg;
  lpht_config_default(&cfg);
  cfg.layout = layout;
  cfg.log2_capacity = log2c;
  cfg.auto_grow = 0;
  return lpht_create(&cfg, (void *)x.s, &x.t);
}

}  // namespace

extern "C" int lpht_autotune(uint32_t layout, uint32_t log2c, uint32_t reps, void *stream, lpht_tuning *out,
                             lpht_autotune_report *report) {
  if (!out || reps < 1 || log2c < 16 || log2c > 30) return LPHT_ERR_INVALID;
  if (layout != LPHT_KV64 && layout != LPHT_PACKED32) return LPHT_ERR_INVALID;
  Scratch x;
  x.s = (hipStream_t)stream;
  const uint64_t c = 1ull << log2c;
  const uint64_t kb = layout == LPHT_PACKED32 ? 4 : 8;
  const uint64_t m_ins = c / 16, m_half = c / 8;  // timed inserts; finds: m_half present + m_half absent
  if (hipEventCreate(&x.ev[0]) != hipSuccess || hipEventCreate(&x.ev[1]) != hipSuccess ||
      hipMalloc(&x.keys, c * kb) != hipSuccess || hipMalloc(&x.absent, m_half * kb) != hipSuccess ||
      hipMalloc(&x.present, m_half * kb) != hipSuccess ||
      hipMalloc(&x.vals, m_half * kb) != hipSuccess || hipMalloc((void **)&x.found, m_half) != hipSuccess)
    return LPHT_ERR_OOM;
  if (launch_gen_keys(x.keys, c, layout, 1, x.s) != hipSuccess ||
      launch_gen_keys(x.absent, m_half, layout, 2, x.s) != hipSuccess)
    return LPHT_ERR_DEVICE;
  int rc = make_table(x, layout, log2c);
  if (rc) return rc;
  const lpht_tuning base = default_tuning();
  const unsigned char *K = (const unsigned char *)x.keys;
  lpht_autotune_report rep;
  std::memset(&rep, 0, sizeof(rep));

  // Builds the table to fill end - m_ins with the default shape, then times
  // the last m_ins inserts and the finds with shape `u`.  The present keys
  // of the finds are every (end / m_half)-th inserted key (end is an odd
  // multiple of m_half), so their probe lengths average the table's
  // successful search rather than those of the earliest insertions.
  auto measure = [&](uint64_t end, const lpht_tuning &u, double &ins_ms, double &find_ms) -> int {
    ins_ms = find_ms = std::numeric_limits<double>::infinity();
    if (hipMemcpy2DAsync(x.present, kb, K, kb * (end / m_half), kb, m_half, hipMemcpyDeviceToDevice, x.s) !=
        hipSuccess)
      return LPHT_ERR_DEVICE;
    for (uint32_t r = 0; r < reps; ++r) {
      int e = lpht_set_tuning(x.t, &base);
      if (!e) e = lpht_clear(x.t, (void *)x.s);
      if (!e) e = lpht_insert(x.t, K, nullptr, end - m_ins, nullptr, (void *)x.s);
      if (!e) e = lpht_set_tuning(x.t, &u);
      if (e) return e;
      ins_ms = std::min(ins_ms, timed(x, [&] {
                          return lpht_insert(x.t, K + (end - m_ins) * kb, nullptr, m_ins, nullptr, (void *)x.s);
                        }));
      find_ms = std::min(find_ms, timed(x, [&] {
                           int f = lpht_find(x.t, x.present, m_half, x.vals, x.found, (void *)x.s);
                           if (!f) f = lpht_find(x.t, x.absent, m_half, x.vals, x.found, (void *)x.s);
                           return f;
                         }));
    }
    return LPHT_OK;
  };

  lpht_tuning best = base;
  for (int qi = 0; qi < 4; ++qi) {
    const uint64_t end = (2 * (uint64_t)qi + 1) * c / 8;
    for (int gi = 0; gi < 5; ++gi) {
      lpht_tuning u = base;
      u.group_width = kWidths[gi];
      rc = measure(end, u, rep.insert_ms[qi][gi], rep.find_ms[qi][gi]);
      if (rc) return rc;
    }
  }
  // Per quarter the narrowest width within kTie of the fastest (fewer lanes
  // per operation; near-ties then resolve the same way on every run); a
  // quarter keeps the width chosen for fill 3/8 unless another is more than
  // kTie faster, so that timing noise does not split calls into launches of
  // different widths.
  auto choose = [&](const double (*ms)[5], uint8_t *g) {
    auto argmin = [&](int q) {
      int b = 0;
      for (int gi = 1; gi < 5; ++gi)
        if (ms[q][gi] < ms[q][b]) b = gi;
      for (int gi = 0; gi < b; ++gi)
        if (ms[q][gi] <= ms[q][b] * (1.0 + kTie)) return gi;
      return b;
    };
    const int ref = argmin(1);
    g[1] = (uint8_t)kWidths[ref];
    for (int q : {0, 2, 3}) {
      const int b = argmin(q);
      g[q] = (uint8_t)kWidths[ms[q][ref] <= ms[q][b] * (1.0 + kTie) ? ref : b];
    }
  };
  choose(rep.find_ms, best.g_find);
  choose(rep.insert_ms, best.g_modify);
  best.group_width = best.g_find[1];

  // workgroup size at fill 3/8 with the chosen widths
  uint32_t bb = 0;
  for (int bi = 0; bi < 3; ++bi) {
    lpht_tuning u = best;
    u.block_threads = kBlocks[bi];
    double ins, fnd;
    rc = measure(3 * c / 8, u, ins, fnd);
    if (rc) return rc;
    rep.block_ms[bi] = ins + fnd;
    if (rep.block_ms[bi] < rep.block_ms[bb]) bb = bi;
  }
  best.block_threads = kBlocks[bb];

  // migration block: doubling a table at fill 7/16
  uint32_t bm = 0;
  for (int mi = 0; mi < 4; ++mi) {
    rep.migrate_ms[mi] = std::numeric_limits<double>::infinity();
    for (uint32_t r = 0; r < reps; ++r) {
      lpht_tuning u = best;
      u.migrate_block = kMigrateBlocks[mi];
      rc = make_table(x, layout, log2c);
      if (!rc) rc = lpht_set_tuning(x.t, &u);
      if (!rc) rc = lpht_insert(x.t, K, nullptr, 7 * c / 16, nullptr, (void *)x.s);
      if (rc) return rc;
      rep.migrate_ms[mi] =
          std::min(rep.migrate_ms[mi], timed(x, [&] { return lpht_grow(x.t, log2c + 1, (void *)x.s); }));
    }
    if (rep.migrate_ms[mi] < rep.migrate_ms[bm]) bm = mi;
  }
  best.migrate_block = kMigrateBlocks[bm];
  *out = best;
  if (report) *report = rep;
  return LPHT_OK;
}
