// Serving runtime of liblpht: a request loop over tables kept resident on
// one device.  See the "serving" part of include/lpht.h for the contract.
//
// One worker thread owns every HIP call of the server that touches a stream.  It admits requests
// (request slots, one request per table at a time in submission order, HBM
// budget), launches them (as one multi-table wave per admission round, or one
// request at a time), and retires launch groups whose completion event has
// fired.  After each group a one-wave kernel writes every touched table's
// exact counts into pinned host memory, so the growth rule that runs before
// the next request on that table decides on exact counts with no stream
// synchronisation.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "lpht_host.h"

using namespace lpht;
using namespace lpht::host;

namespace {

double now_us() {
  return std::chrono::duration<double, std::micro>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

size_t round256(size_t x) { return (x + 255) & ~(size_t)255; }

// True when the first and the last byte of [p, p + bytes) lie in pinned host
// memory or in device memory (memory a kernel can address).
bool gpu_accessible(const void *p, size_t bytes) {
  for (const void *x : {p, (const void *)((const char *)p + bytes - 1)}) {
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, x) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    if (at.type != hipMemoryTypeHost && at.type != hipMemoryTypeDevice) return false;
  }
  return true;
}

struct Req {
  lpht_request r;
  uint32_t count[3];  // operations per kind
  lpht_completion c;
  bool done = false;
  uint64_t need = 0;  // bytes accounted by admission (staging and growth)
  uint64_t grow = 0;  // the growth part of `need`
  uint64_t arena_off = ~0ull;  // resident mode: the request's staging in the arena
  // resident mode, a migration entry of the server's own: its table grows
  // into mig_cells before `waiting` is posted
  bool mig = false;
  Req *waiting = nullptr;
  void *mig_cells = nullptr;
};

struct Group {
  std::vector<Req *> reqs;
  std::vector<uint32_t> tables;
  hipEvent_t ev;
  uint32_t stream;
};

}  // namespace

struct lpht_server {
  lpht_server_config cfg;
  int device = 0;
  uint32_t kb = 8;
  std::vector<lpht_table *> tables;
  // count readback areas, one per stream (a stream's groups copy its whole
  // area; a table's entry is only read back after the group that wrote it):
  // [stream][table][used, live, err, pad]
  uint64_t *totals = nullptr;    // pinned
  uint64_t *d_totals = nullptr;  // device, written by the count kernel
  std::vector<uint8_t> busy;
  std::vector<std::deque<Req *>> fifo;
  std::deque<Req *> incoming;
  std::unordered_map<uint64_t, Req *> reqs;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::vector<hipStream_t> streams;
  std::vector<lpht_batch *> batches;
  std::vector<Group> inflight;
  std::vector<hipEvent_t> spare_events;
  uint64_t next_ticket = 1;
  uint64_t outstanding = 0;  // submitted, not done (under mu)
  uint32_t inflight_reqs = 0;
  uint64_t staging_bytes = 0;
  lpht_server_stats st{};
  double busy_since = 0;
  bool stop = false;
  uint32_t next_stream = 0;
  uint32_t group_seq = 0;
  std::thread worker;
  // persistent mode
  PersistCtl *pctl = nullptr;      // pinned
  PersistReq *pring = nullptr;     // pinned
  PersistDone *pdone = nullptr;    // pinned
  PersistReq *pdring = nullptr;   // device copy of the ring
  PersistDev *pdev = nullptr;      // device
  PersistState *pst = nullptr;     // device
  Req *pentry[kPersistRing] = {};  // request held by each ring entry
  uint64_t next_q = 0;             // requests posted
  uint64_t oldest_q = 0;           // oldest request not yet retired
  bool running = false;
  hipEvent_t persist_ev = nullptr;
  hipGraph_t persist_graph = nullptr;     // {arm, resident kernel}, captured once
  hipGraphExec_t persist_exec = nullptr;
  std::vector<Req *> grow_wait;    // admitted, waiting for their table to grow
  uint32_t persist_grid = 0;
  unsigned char *arena = nullptr;  // resident mode: device staging of requests in flight
  uint64_t arena_bytes = 0;
  std::map<uint64_t, uint64_t> arena_free;  // offset -> length of free ranges
  uint64_t idle_ticks = 0;         // kIdleExitMs in ticks of the device's constant clock
  uint64_t persist_launches = 0;
  bool persist_failed = false;     // a bounded wait in the kernel expired

};

namespace {

uint64_t table_bytes_of(const lpht_table *t) { return cell_bytes(t->cfg.layout) << t->log2c; }

uint64_t table_bytes(const lpht_server *S) {
  uint64_t b = 0;
  for (auto *t : S->tables) b += cell_bytes(t->cfg.layout) << t->log2c;
  return b;
}

// A table that grew for request q is counted at its new size from then on;
// until q retires, its reservation stands for the old cells instead (freed
// once the work queued before the growth is done), not for the new ones a
// second time.
void growth_done(lpht_server *S, Req *q, uint64_t before) {
  if (!q->grow || table_bytes_of(S->tables[q->r.table]) == before) return;
  const uint64_t keep = std::min<uint64_t>(q->grow, before);
  S->staging_bytes -= q->grow - keep;
  q->need -= q->grow - keep;
  q->grow = keep;
}

// Bytes a growth before `b` insertions would allocate for the new table: an
// upper bound, as the growth rule decides on exact counts, and insertions
// made on the table since its counts were last exact (`pending`) may each
// have added a live key.
uint64_t growth_bytes(const lpht_table *t, uint64_t b) {
  const uint64_t c = 1ull << t->log2c;
  if (b == 0 || within_fill(t, t->known_used + t->pending + b, c)) return 0;
  const uint64_t live = t->known_live + t->pending + b;
  uint32_t target = t->log2c;
  if ((unsigned __int128)live * 2 * t->cfg.max_fill_den > (unsigned __int128)c * t->cfg.max_fill_num) {
    do {
      ++target;
    } while (target < 34 && !within_fill(t, live, 1ull << target));
  }
  // the old and the new table coexist during a migration; a chain of
  // doublings peaks at the last one
  return cell_bytes(t->cfg.layout) << target;
}

size_t staging_size(const lpht_server *S, const Req *q) {
  const size_t n = q->r.n;
  return 2 * round256(n * S->kb) + 2 * round256(n);
}

// Resident mode: best fit in the staging arena (256-byte granules).
uint64_t arena_alloc(lpht_server *S, uint64_t bytes) {
  bytes = round256(bytes);
  auto best = S->arena_free.end();
  for (auto it = S->arena_free.begin(); it != S->arena_free.end(); ++it)
    if (it->second >= bytes && (best == S->arena_free.end() || it->second < best->second)) best = it;
  if (best == S->arena_free.end()) return ~0ull;
  const uint64_t off = best->first, len = best->second;
  S->arena_free.erase(best);
  if (len > bytes) S->arena_free[off + bytes] = len - bytes;
  return off;
}

void arena_release(lpht_server *S, uint64_t off, uint64_t bytes) {
  bytes = round256(bytes);
  auto next = S->arena_free.lower_bound(off);
  if (next != S->arena_free.end() && off + bytes == next->first) {
    bytes += next->second;
    next = S->arena_free.erase(next);
  }
  if (next != S->arena_free.begin()) {
    auto prev = std::prev(next);
    if (prev->first + prev->second == off) {
      prev->second += bytes;
      return;
    }
  }
  S->arena_free[off] = bytes;
}

void finish_locked(lpht_server *S, Req *q) {
  q->done = true;
  S->outstanding--;
  S->st.completed++;
}

hipEvent_t get_event(lpht_server *S) {
  if (!S->spare_events.empty()) {
    hipEvent_t e = S->spare_events.back();
    S->spare_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
  return e;
}

// Launches one group of admitted requests on the next stream.
void launch_group(lpht_server *S, std::vector<Req *> &group) {
  const uint32_t si = S->next_stream++ % (uint32_t)S->streams.size();
  hipStream_t s = S->streams[si];
  Group g;
  g.ev = get_event(S);
  std::vector<lpht_batch_op> ops;
  ops.reserve(3 * group.size());
  const double t_admit = now_us();
  for (Req *q : group) {
    q->c.admit_us = t_admit;
    q->c.wave = S->group_seq;
    const size_t n = q->r.n;
    unsigned char *base = S->arena + q->arena_off;  // the request's staging
    void *dkeys = base;
    void *dvals = base + round256(n * S->kb);
    uint8_t *dkinds = base + 2 * round256(n * S->kb);
    uint8_t *dflags = dkinds + round256(n);
    lpht_table *t = S->tables[q->r.table];
    g.tables.push_back(q->r.table);
    g.reqs.push_back(q);
    (void)hipMemcpyAsync(dkeys, q->r.keys, n * S->kb, hipMemcpyHostToDevice, s);
    (void)hipMemcpyAsync(dkinds, q->r.kinds, n, hipMemcpyHostToDevice, s);
    const uint32_t kind_op[3] = {LPHT_OP_FIND, LPHT_OP_UPSERT, LPHT_OP_ERASE};
    for (uint32_t k = 0; k < 3; ++k) {
      if (q->count[k] == 0) continue;
      lpht_batch_op o{};
      o.table = t;
      o.op = kind_op[k];
      o.up = LPHT_ADD;
      o.keys = dkeys;
      o.vals = nullptr;  // increments by one
      o.n = n;
      o.vals_out = k == 0 ? dvals : nullptr;
      o.flags = dflags;
      o.kinds = dkinds;
      o.kind_sel = k;
      o.count_sel = q->count[k];
      ops.push_back(o);
    }
  }
  std::vector<uint64_t> before(group.size());
  for (size_t i = 0; i < group.size(); ++i) before[i] = table_bytes_of(S->tables[group[i]->r.table]);
  if (!ops.empty()) {
    const int rc = lpht_batch_run(S->batches[si], ops.data(), (uint32_t)ops.size(), (void *)s);
    S->st.launches_phases += 1;
    if (rc != LPHT_OK)
      for (Req *q : group)
        if (q->c.status == LPHT_OK) q->c.status = rc;
  }
  for (size_t i = 0; i < group.size(); ++i) growth_done(S, group[i], before[i]);
  const size_t area = 4 * S->tables.size();
  for (uint32_t ti : g.tables)
    (void)launch_count_totals(S->tables[ti]->status, S->d_totals + si * area + 4 * ti, s);
  (void)hipMemcpyAsync(S->totals + si * area, S->d_totals + si * area, sizeof(uint64_t) * area,
                       hipMemcpyDeviceToHost, s);
  g.stream = si;
  for (Req *q : group) {
    const size_t n = q->r.n;
    unsigned char *base = S->arena + q->arena_off;
    if (q->r.vals_out && q->count[0])
      (void)hipMemcpyAsync(q->r.vals_out, base + round256(n * S->kb), n * S->kb,
                           hipMemcpyDeviceToHost, s);
    if (q->r.flags)
      (void)hipMemcpyAsync(q->r.flags, base + 2 * round256(n * S->kb) + round256(n), n,
                           hipMemcpyDeviceToHost, s);
  }
  (void)hipEventRecord(g.ev, s);
  if (S->inflight.empty()) S->busy_since = now_us();
  S->inflight_reqs += (uint32_t)group.size();
  S->group_seq++;
  S->st.waves++;
  S->inflight.push_back(std::move(g));
}

void retire_group(lpht_server *S, Group &g) {
  const double t = now_us();
  for (uint32_t ti : g.tables) {
    lpht_table *T = S->tables[ti];
    const uint64_t *tot = S->totals + g.stream * 4 * S->tables.size() + 4 * ti;
    T->known_used = tot[0];
    T->known_live = tot[1];
    T->pending = 0;
    T->mods_since_exact = 0;
    S->busy[ti] = 0;
  }
  for (Req *q : g.reqs) {
    if (q->r.vals_out && q->count[0] == 0) std::memset(q->r.vals_out, 0, q->r.n * S->kb);
    q->c.done_us = t;
    S->staging_bytes -= q->need;
    arena_release(S, q->arena_off, staging_size(S, q));
  }
  S->inflight_reqs -= (uint32_t)g.reqs.size();
  S->spare_events.push_back(g.ev);
  if (S->inflight.size() == 1) S->st.busy_us += t - S->busy_since;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    for (Req *q : g.reqs) finish_locked(S, q);
  }
  S->cv_done.notify_all();
}

// Operations of one wave: enough for the batch kernels to fill the device,
// few enough that several waves are in flight on the server's streams (their
// copies, kernels and completions overlap, and a table's next request does
// not wait for every other table's).  On the 300-request config-5 trace,
// admitting every ready request into one wave gave 180-250 Mops/s and this
// cap 220-380 (runs spread widely; 2^19 and 2^20 were no better); a tight
// HBM budget, which admits fewer requests at once, gives 410-530.
constexpr uint64_t kWaveMaxOps = 1ull << 21;

// Picks requests to start now: oldest first among tables that are idle, while
// slots and the HBM budget allow, up to max_ops operations (0: no limit; a
// request larger than that is admitted alone).
void admit(lpht_server *S, std::vector<Req *> &out, uint64_t max_ops = 0) {
  uint64_t ops = 0;
  std::vector<uint32_t> cand;
  for (uint32_t t = 0; t < S->fifo.size(); ++t)
    if (!S->busy[t] && !S->fifo[t].empty()) cand.push_back(t);
  std::sort(cand.begin(), cand.end(), [&](uint32_t a, uint32_t b) {
    return S->fifo[a].front()->c.ticket < S->fifo[b].front()->c.ticket;
  });
  uint64_t hbm = table_bytes(S) + S->staging_bytes;
  const uint32_t slots = S->cfg.mode == LPHT_SERVE_PERSISTENT
                            ? std::min<uint32_t>(S->cfg.max_inflight, kPersistRing)
                            : S->cfg.max_inflight;
  for (uint32_t t : cand) {
    if (S->inflight_reqs + S->grow_wait.size() + out.size() >= slots) break;
    if (S->cfg.mode == LPHT_SERVE_PERSISTENT &&
        S->next_q + S->grow_wait.size() + out.size() >= S->oldest_q + kPersistRing)
      break;  // the ring entry of the oldest request is still in use
    Req *q = S->fifo[t].front();
    if (max_ops && !out.empty() && ops + q->r.n > max_ops) break;
    // the staging comes from the arena; the budget counts it while in use
    const uint64_t staging = staging_size(S, q);
    const uint64_t grow = growth_bytes(S->tables[t], q->count[1]);
    const uint64_t need = round256(staging) + grow;
    uint64_t off = ~0ull;
    const bool over = S->cfg.hbm_budget && hbm + need > S->cfg.hbm_budget;
    if (over || (off = arena_alloc(S, staging)) == ~0ull) {
      if (S->inflight_reqs == 0 && S->grow_wait.empty() && out.empty()) {
        // nothing will free memory: this request can never run
        S->fifo[t].pop_front();
        q->c.status = LPHT_ERR_OOM;
        q->c.admit_us = q->c.done_us = now_us();
        {
          std::lock_guard<std::mutex> lk(S->mu);
          finish_locked(S, q);
        }
        S->cv_done.notify_all();
        continue;
      }
      S->st.admission_waits++;
      break;  // keep the order: the oldest waiting request goes first
    }
    S->fifo[t].pop_front();
    S->busy[t] = 1;
    q->need = need;
    q->grow = grow;
    q->arena_off = off;
    hbm += need;
    S->staging_bytes += need;
    ops += q->r.n;
    out.push_back(q);
  }
  if (hbm > S->st.peak_hbm_bytes) S->st.peak_hbm_bytes = hbm;
}

// ---- persistent mode ----

// The resident kernel exits after this long without work (a new request then
// relaunches it).
constexpr double kIdleExitMs = 20.0;

// Captures the resident kernel's launch (arming kernel + resident kernel,
// which read the first request to serve from ctl->base) into a graph.
hipError_t persist_capture(lpht_server *S) {
  hipStream_t s = S->streams[0];
  hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  const hipError_t le = launch_persist(S->cfg.layout, S->pctl, S->pring, S->pdring, S->pdone, S->pdev,
                                       S->pst, S->idle_ticks, S->persist_grid, s);
  e = hipStreamEndCapture(s, &S->persist_graph);
  if (le != hipSuccess) return le;
  if (e != hipSuccess) return e;
  return hipGraphInstantiate(&S->persist_exec, S->persist_graph, nullptr, nullptr, 0);
}

void persist_launch(lpht_server *S) {
  hipStream_t s = S->streams[0];
  __atomic_store_n(&S->pctl->base, S->oldest_q, __ATOMIC_RELAXED);
  __atomic_store_n(&S->pctl->stop, 0ull, __ATOMIC_RELEASE);
  if (hipGraphLaunch(S->persist_exec, s) == hipSuccess) {
    (void)hipEventRecord(S->persist_ev, s);
    S->running = true;
    S->persist_launches++;
    S->st.waves++;
    S->st.launches_phases++;
  } else {
    S->persist_failed = true;
  }
}

// Called once the resident kernel has ended: reads its error word.
void persist_ended(lpht_server *S) {
  S->running = false;
  uint64_t err = 0;
  if (hipMemcpyAsync(&err, &S->pst->error, sizeof(err), hipMemcpyDeviceToHost, S->streams[0]) !=
          hipSuccess ||
      hipStreamSynchronize(S->streams[0]) != hipSuccess || err)
    S->persist_failed = true;
}

// Posts an admitted request into the device ring.
void persist_post(lpht_server *S, Req *q) {
  const uint64_t qn = S->next_q;
  const uint32_t e = (uint32_t)(qn % kPersistRing);
  lpht_table *t = S->tables[q->r.table];
  PersistReq &R = S->pring[e];
  const size_t n = q->r.n;
  unsigned char *base = S->arena + q->arena_off;
  BulkArgs a = make_args(t);
  a.keys = base;
  a.vals = nullptr;  // increments by one
  a.n = n;
  a.vals_out = base + round256(n * S->kb);
  a.flags = base + 2 * round256(n * S->kb) + round256(n);
  a.up = LPHT_ADD;
  a.kinds = base + 2 * round256(n * S->kb);
  a.kind_sel = 0;
  R.a = a;
  R.hkeys = q->r.keys;
  R.hkinds = q->r.kinds;
  R.hvals = q->r.vals_out;
  R.hflags = q->r.flags;
  const unsigned long long copy_rounds = (n + kCopyRound - 1) / kCopyRound;
  R.rounds[0] = copy_rounds;
  for (int k = 0; k < 3; ++k) R.rounds[k + 1] = q->count[k] ? (n + kRound - 1) / kRound : 0;
  R.rounds[4] = copy_rounds;
  R.mig_cells = nullptr;
  R.mig_log2c = 0;
  __atomic_store_n(&R.seq, qn + 1, __ATOMIC_RELEASE);
  t->mods_since_exact++;
  S->pentry[e] = q;
  q->c.admit_us = now_us();
  q->c.wave = (uint32_t)S->persist_launches;
  S->next_q = qn + 1;
  if (S->inflight_reqs++ == 0) S->busy_since = now_us();
  __atomic_store_n(&S->pctl->posted, qn + 1, __ATOMIC_RELEASE);
}

// Smallest capacity the resident kernel migrates itself (its migration
// window spans 512 old cells).
constexpr uint32_t kPersistMigMinLog2 = 10;

// Posts a migration entry that doubles table `ti` inside the running resident
// kernel (Sec. 5.3.2: the serving wavefronts are the helpers, and requests on
// other tables keep being served meanwhile); `q` is posted once it is done.
// False when the new table cannot be allocated.
bool persist_post_migration(lpht_server *S, uint32_t ti, Req *q) {
  lpht_table *t = S->tables[ti];
  const size_t nb = (size_t)cell_bytes(t->cfg.layout) << (t->log2c + 1);
  void *nc = dev_alloc(t, nb, S->streams[0]);
  if (!nc) return false;
  Req *m = new (std::nothrow) Req();
  if (!m) {
    dev_free(t, nc, nb, S->streams[0]);
    return false;
  }
  m->mig = true;
  m->waiting = q;
  m->mig_cells = nc;
  m->r.table = ti;
  const uint64_t qn = S->next_q;
  const uint32_t e = (uint32_t)(qn % kPersistRing);
  PersistReq &R = S->pring[e];
  BulkArgs a = make_args(t);
  a.n = 0;
  R.a = a;
  R.hkeys = nullptr;
  R.hkinds = nullptr;
  R.hvals = nullptr;
  R.hflags = nullptr;
  R.rounds[0] = (1ull << t->log2c) / kPersistMigBlock;
  R.rounds[1] = R.rounds[2] = R.rounds[3] = 0;
  R.rounds[4] = 1;
  R.mig_cells = nc;
  R.mig_log2c = t->log2c + 1;
  __atomic_store_n(&R.seq, qn + 1, __ATOMIC_RELEASE);
  t->mods_since_exact++;
  S->pentry[e] = m;
  S->next_q = qn + 1;
  if (S->inflight_reqs++ == 0) S->busy_since = now_us();
  __atomic_store_n(&S->pctl->posted, qn + 1, __ATOMIC_RELEASE);
  return true;
}

// Whether the growth rule may fire before the request's increments: an upper
// bound of `used` (the exact count after the last completion plus insertions
// made on the table outside the server since, `pending`); grow_before_batch
// then decides exactly.
bool needs_growth(const lpht_server *S, const Req *q) {
  const lpht_table *t = S->tables[q->r.table];
  return q->count[1] && !within_fill(t, t->known_used + t->pending + q->count[1], 1ull << t->log2c);
}

// A request whose table may have to grow first: a single doubling of a large
// enough table whose counts are exact becomes a migration entry for the
// running kernel; every other case waits for the host path (stop the kernel,
// migrate, relaunch).
void persist_grow_then_post(lpht_server *S, Req *q) {
  lpht_table *t = S->tables[q->r.table];
  if (!S->persist_failed && t->pending == 0 && t->mods_since_exact == 0 && t->log2c >= kPersistMigMinLog2) {
    const int kind = growth_kind(t, q->count[1]);
    if (kind == 0) {
      persist_post(S, q);
      return;
    }
    if (kind == 1 && persist_post_migration(S, q->r.table, q)) return;
  }
  S->grow_wait.push_back(q);
}

// A completed migration entry: the table takes the new cells (or, after an
// overflow, the host migrates it), then the waiting request goes on.
void persist_migration_done(lpht_server *S, Req *m, uint32_t e) {
  lpht_table *t = S->tables[m->r.table];
  const size_t cb = cell_bytes(t->cfg.layout);
  const uint64_t err = S->pdone[e].err;
  Req *q = m->waiting;
  // (frees on streams[0] reach the pool only once the resident kernel,
  // queued before them, has exited)
  if ((err & kErrMigrate) || S->persist_failed) {
    dev_free(t, m->mig_cells, cb << (t->log2c + 1), S->streams[0]);
    S->st.kernel_growth_fallbacks++;
    S->grow_wait.push_back(q);
  } else {
    // the old table is no longer read: its last reader was this entry
    const uint64_t before = table_bytes_of(t);
    dev_free(t, t->cells, cb << t->log2c, S->streams[0]);
    t->cells = m->mig_cells;
    t->stats.migrations++;
    t->stats.resizes++;
    t->stats.cells_migrated += 1ull << t->log2c;
    t->log2c += 1;
    S->st.kernel_growths++;
    growth_done(S, q, before);
    persist_grow_then_post(S, q);
  }
  delete m;
}

// Retires requests whose completion the kernel has published.
bool persist_retire(lpht_server *S) {
  bool any = false;
  std::vector<Req *> fin;
  for (uint64_t qn = S->oldest_q; qn < S->next_q; ++qn) {
    const uint32_t e = (uint32_t)(qn % kPersistRing);
    Req *q = S->pentry[e];
    if (!q) continue;
    if (__atomic_load_n(&S->pdone[e].seq, __ATOMIC_ACQUIRE) != qn + 1) continue;
    lpht_table *T = S->tables[q->r.table];
    if (q->mig) {
      T->known_used = S->pdone[e].used;
      T->known_live = S->pdone[e].live;
      T->pending = 0;
      T->mods_since_exact = 0;
      S->pentry[e] = nullptr;
      if (--S->inflight_reqs == 0) S->st.busy_us += now_us() - S->busy_since;
      persist_migration_done(S, q, e);
      any = true;
      continue;
    }
    if (S->persist_failed && q->c.status == LPHT_OK) q->c.status = LPHT_ERR_DEVICE;
    T->known_used = S->pdone[e].used;
    T->known_live = S->pdone[e].live;
    T->pending = 0;
    T->mods_since_exact = 0;
    S->busy[q->r.table] = 0;
    q->c.done_us = now_us();
    S->staging_bytes -= q->need;
    arena_release(S, q->arena_off, staging_size(S, q));
    S->pentry[e] = nullptr;
    if (--S->inflight_reqs == 0) S->st.busy_us += now_us() - S->busy_since;
    fin.push_back(q);
    any = true;
  }
  while (S->oldest_q < S->next_q && !S->pentry[S->oldest_q % kPersistRing]) S->oldest_q++;
  if (!fin.empty()) {
    {
      std::lock_guard<std::mutex> lk(S->mu);
      for (Req *q : fin) finish_locked(S, q);
    }
    S->cv_done.notify_all();
  }
  return any;
}

// One pass of the worker in persistent mode.
bool persist_step(lpht_server *S, std::vector<Req *> &admitted) {
  bool progressed = persist_retire(S);
  if (S->running && hipEventQuery(S->persist_ev) == hipSuccess) persist_ended(S);
  // requests whose table must grow first: stop the kernel, migrate, restart
  if (!S->grow_wait.empty()) {
    if (S->running) {
      __atomic_store_n(&S->pctl->stop, 1ull, __ATOMIC_RELEASE);
    } else {
      hipStream_t s = S->streams[0];
      for (Req *q : S->grow_wait) {
        lpht_table *t = S->tables[q->r.table];
        const uint64_t before = table_bytes_of(t);
        const int rc = grow_before_batch(t, q->count[1], s);
        t->pending = 0;  // the posted request accounts for its insertions itself
        growth_done(S, q, before);
        if (rc) {
          // the table could not grow: the request fails as a whole
          q->c.status = rc;
          q->c.admit_us = q->c.done_us = now_us();
          S->busy[q->r.table] = 0;
          S->staging_bytes -= q->need;
          arena_release(S, q->arena_off, staging_size(S, q));
          {
            std::lock_guard<std::mutex> lk(S->mu);
            finish_locked(S, q);
          }
          S->cv_done.notify_all();
          continue;
        }
        persist_post(S, q);
      }
      S->grow_wait.clear();
      persist_launch(S);
      progressed = true;
    }
    return progressed;
  }
  admitted.clear();
  admit(S, admitted);
  for (Req *q : admitted) {
    if (needs_growth(S, q))
      persist_grow_then_post(S, q);
    else
      persist_post(S, q);
    progressed = true;
  }
  if (!S->running && S->oldest_q < S->next_q && S->grow_wait.empty()) {
    persist_launch(S);
    progressed = true;
  }
  return progressed;
}

void worker_loop(lpht_server *S) {
  (void)hipSetDevice(S->device);
  std::vector<Req *> admitted;
  const bool persistent = S->cfg.mode == LPHT_SERVE_PERSISTENT;
  while (true) {
    bool progressed = false;
    if (persistent) {
      {
        std::unique_lock<std::mutex> lk(S->mu);
        while (!S->incoming.empty()) {
          Req *q = S->incoming.front();
          S->incoming.pop_front();
          S->fifo[q->r.table].push_back(q);
        }
        if (S->stop && S->outstanding == 0) break;
      }
      progressed = persist_step(S, admitted);
      if (!progressed) {
        if (!S->running && S->oldest_q == S->next_q) {
          std::unique_lock<std::mutex> lk(S->mu);
          S->cv_work.wait_for(lk, std::chrono::milliseconds(2),
                              [&] { return S->stop || !S->incoming.empty(); });
        } else {
          std::this_thread::yield();
        }
      }
      continue;
    }
    for (size_t w = 0; w < S->inflight.size();) {
      if (hipEventQuery(S->inflight[w].ev) == hipSuccess) {
        retire_group(S, S->inflight[w]);
        S->inflight.erase(S->inflight.begin() + w);
        progressed = true;
      } else {
        ++w;
      }
    }
    {
      std::unique_lock<std::mutex> lk(S->mu);
      while (!S->incoming.empty()) {
        Req *q = S->incoming.front();
        S->incoming.pop_front();
        S->fifo[q->r.table].push_back(q);
      }
      if (S->stop && S->outstanding == 0 && S->inflight.empty()) break;
    }
    admitted.clear();
    admit(S, admitted, S->cfg.mode == LPHT_SERVE_WAVES ? kWaveMaxOps : 0);
    if (!admitted.empty()) {
      progressed = true;
      if (S->cfg.mode == LPHT_SERVE_WAVES) {
        launch_group(S, admitted);
      } else {
        for (Req *q : admitted) {
          std::vector<Req *> one{q};
          launch_group(S, one);
        }
      }
    }
    if (!progressed) {
      if (S->inflight.empty()) {
        std::unique_lock<std::mutex> lk(S->mu);
        S->cv_work.wait_for(lk, std::chrono::milliseconds(2),
                            [&] { return S->stop || !S->incoming.empty(); });
      } else {
        std::this_thread::yield();
      }
    }
  }
}

void destroy_all(lpht_server *S) {
  if (S->running && S->pctl) {
    __atomic_store_n(&S->pctl->stop, 1ull, __ATOMIC_RELEASE);
    (void)hipEventSynchronize(S->persist_ev);
    S->running = false;
  }
  for (auto *b : S->batches) lpht_batch_destroy(b);
  for (auto *t : S->tables) lpht_destroy(t, S->streams.empty() ? nullptr : (void *)S->streams[0]);
  for (auto s : S->streams) {
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
  }
  for (auto e : S->spare_events) (void)hipEventDestroy(e);
  if (S->totals) (void)hipHostFree(S->totals);
  if (S->d_totals) (void)hipFree(S->d_totals);
  if (S->pctl) (void)hipHostFree(S->pctl);
  if (S->pring) (void)hipHostFree(S->pring);
  if (S->pdone) (void)hipHostFree(S->pdone);
  if (S->pdring) (void)hipFree(S->pdring);
  if (S->arena) (void)hipFree(S->arena);
  if (S->pdev) (void)hipFree(S->pdev);
  if (S->pst) (void)hipFree(S->pst);
  if (S->persist_ev) (void)hipEventDestroy(S->persist_ev);
  if (S->persist_exec) (void)hipGraphExecDestroy(S->persist_exec);
  if (S->persist_graph) (void)hipGraphDestroy(S->persist_graph);
  for (auto &kv : S->reqs) delete kv.second;
  delete S;
}

}  // namespace

extern "C" {

int lpht_server_create(const lpht_server_config *cfg, lpht_server **out) {
  if (!out) return LPHT_ERR_INVALID;
  *out = nullptr;
  if (!cfg || cfg->ntables == 0 || cfg->ntables > 65536 || !cfg->log2_capacity) return LPHT_ERR_INVALID;
  if (cfg->layout != LPHT_KV64 && cfg->layout != LPHT_PACKED32) return LPHT_ERR_INVALID;
  if (cfg->mode > LPHT_SERVE_PERSISTENT || cfg->max_inflight < 1 || cfg->max_inflight > 4096)
    return LPHT_ERR_INVALID;
  if (cfg->streams < 1 || cfg->streams > 8 || cfg->reserved) return LPHT_ERR_INVALID;
  lpht_server *S = new (std::nothrow) lpht_server();
  if (!S) return LPHT_ERR_OOM;
  S->cfg = *cfg;
  S->cfg.log2_capacity = nullptr;
  S->kb = cfg->layout == LPHT_PACKED32 ? 4 : 8;
  if (hipGetDevice(&S->device) != hipSuccess) {
    delete S;
    return LPHT_ERR_DEVICE;
  }
  for (uint32_t i = 0; i < cfg->streams; ++i) {
    hipStream_t s;
    lpht_batch *b = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      destroy_all(S);
      return LPHT_ERR_DEVICE;
    }
    S->streams.push_back(s);
    const int rc = lpht_batch_create(3 * cfg->max_inflight, &b);
    if (rc) {
      destroy_all(S);
      return rc;
    }
    S->batches.push_back(b);
  }
  const size_t tot_bytes = sizeof(uint64_t) * 4 * cfg->ntables * cfg->streams;
  if (hipHostMalloc((void **)&S->totals, tot_bytes, hipHostMallocDefault) != hipSuccess) {
    destroy_all(S);
    return LPHT_ERR_OOM;
  }
  std::memset(S->totals, 0, tot_bytes);
  if (hipMalloc((void **)&S->d_totals, tot_bytes) != hipSuccess ||
      hipMemset(S->d_totals, 0, tot_bytes) != hipSuccess) {
    destroy_all(S);
    return LPHT_ERR_OOM;
  }
  for (uint32_t i = 0; i < cfg->ntables; ++i) {
    lpht_config tc;
    lpht_config_default(&tc);
    tc.layout = cfg->layout;
    tc.log2_capacity = cfg->log2_capacity[i];
    tc.auto_grow = 1;
    lpht_table *t = nullptr;
    const int rc = lpht_create(&tc, (void *)S->streams[0], &t);
    if (rc) {
      destroy_all(S);
      return rc;
    }
    S->tables.push_back(t);
  }
  if (hipStreamSynchronize(S->streams[0]) != hipSuccess) {
    destroy_all(S);
    return LPHT_ERR_DEVICE;
  }
  {
    // staging arena: 1 GiB, or what the budget leaves beside the initial
    // tables (at least 1 MiB)
    uint64_t ab = 1ull << 30;
    if (cfg->hbm_budget) {
      const uint64_t tb = table_bytes(S);
      const uint64_t spare = cfg->hbm_budget > tb ? cfg->hbm_budget - tb : 0;
      ab = std::min<uint64_t>(ab, std::max<uint64_t>(1ull << 20, round256(spare)));
    }
    if (hipMalloc((void **)&S->arena, ab) != hipSuccess) {
      destroy_all(S);
      return LPHT_ERR_OOM;
    }
    S->arena_bytes = ab;
    S->arena_free[0] = ab;
  }
  if (cfg->mode == LPHT_SERVE_PERSISTENT) {
    if (hipHostMalloc((void **)&S->pctl, sizeof(PersistCtl), hipHostMallocCoherent) != hipSuccess ||
        hipHostMalloc((void **)&S->pring, sizeof(PersistReq) * kPersistRing, hipHostMallocCoherent) !=
            hipSuccess ||
        hipHostMalloc((void **)&S->pdone, sizeof(PersistDone) * kPersistRing, hipHostMallocCoherent) !=
            hipSuccess ||
        hipMalloc((void **)&S->pdring, sizeof(PersistReq) * kPersistRing) != hipSuccess ||
        hipMalloc((void **)&S->pdev, sizeof(PersistDev) * kPersistRing) != hipSuccess ||
        hipMalloc((void **)&S->pst, sizeof(PersistState)) != hipSuccess ||
        hipEventCreateWithFlags(&S->persist_ev, hipEventDisableTiming) != hipSuccess) {
      destroy_all(S);
      return LPHT_ERR_OOM;
    }
    std::memset(S->pctl, 0, sizeof(PersistCtl));
    std::memset(S->pring, 0, sizeof(PersistReq) * kPersistRing);
    std::memset(S->pdone, 0, sizeof(PersistDone) * kPersistRing);
    int ncu = 0;
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, S->device);
    // four workgroups of 256 per CU: the resident kernel is built for 4
    // wavefronts per SIMD
    S->persist_grid = (uint32_t)(ncu > 0 ? 4 * ncu : 1024);
    S->persist_grid = std::max<uint32_t>(kPersistGroups, S->persist_grid / kPersistGroups * kPersistGroups);
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, S->device) != hipSuccess || khz <= 0)
      khz = 100000;
    S->idle_ticks = (uint64_t)(kIdleExitMs * khz);
    if (launch_persist_init(S->pdev, S->pst, 0, S->streams[0]) != hipSuccess ||
        hipStreamSynchronize(S->streams[0]) != hipSuccess || persist_capture(S) != hipSuccess) {
      destroy_all(S);
      return LPHT_ERR_DEVICE;
    }
  }
  S->busy.assign(cfg->ntables, 0);
  S->fifo.resize(cfg->ntables);
  S->worker = std::thread(worker_loop, S);
  *out = S;
  return LPHT_OK;
}

int lpht_server_submit(lpht_server *S, const lpht_request *req, uint64_t *ticket) {
  if (!S || !req || !ticket) return LPHT_ERR_INVALID;
  if (req->table >= S->tables.size() || req->reserved || req->n == 0 || req->n > (1ull << 31) ||
      !req->keys || !req->kinds)
    return LPHT_ERR_INVALID;
  if (S->cfg.mode == LPHT_SERVE_PERSISTENT) {
    // the resident kernel reads and writes the caller's buffers directly
    if (!gpu_accessible(req->keys, req->n * S->kb) || !gpu_accessible(req->kinds, req->n) ||
        (req->vals_out && !gpu_accessible(req->vals_out, req->n * S->kb)) ||
        (req->flags && !gpu_accessible(req->flags, req->n)))
      return LPHT_ERR_INVALID;
  }
  Req *q = new (std::nothrow) Req();
  if (!q) return LPHT_ERR_OOM;
  q->r = *req;
  q->count[0] = q->count[1] = q->count[2] = 0;
  for (uint64_t i = 0; i < req->n; ++i) {
    const uint8_t k = req->kinds[i];
    if (k > 2) {
      delete q;
      return LPHT_ERR_INVALID;
    }
    q->count[k]++;
  }
  q->c = lpht_completion{};
  q->c.submit_us = now_us();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) {
      delete q;
      return LPHT_ERR_INVALID;
    }
    q->c.ticket = S->next_ticket++;
    S->reqs[q->c.ticket] = q;
    S->incoming.push_back(q);
    S->outstanding++;
    *ticket = q->c.ticket;
  }
  S->cv_work.notify_one();
  return LPHT_OK;
}

int lpht_server_poll(lpht_server *S, uint64_t ticket, lpht_completion *out) {
  if (!S) return LPHT_ERR_INVALID;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return LPHT_ERR_INVALID;
  if (!it->second->done) return 1;
  if (out) *out = it->second->c;
  delete it->second;
  S->reqs.erase(it);
  return LPHT_OK;
}

int lpht_server_wait(lpht_server *S, uint64_t ticket, lpht_completion *out) {
  if (!S) return LPHT_ERR_INVALID;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return LPHT_ERR_INVALID;
  Req *q = it->second;
  S->cv_done.wait(lk, [&] { return q->done; });
  if (out) *out = q->c;
  delete q;
  S->reqs.erase(it);
  return LPHT_OK;
}

int lpht_server_drain(lpht_server *S) {
  if (!S) return LPHT_ERR_INVALID;
  std::unique_lock<std::mutex> lk(S->mu);
  S->cv_done.wait(lk, [&] { return S->outstanding == 0; });
  return LPHT_OK;
}

int lpht_server_table(lpht_server *S, uint32_t index, lpht_table **out) {
  if (!S || !out || index >= S->tables.size()) return LPHT_ERR_INVALID;
  *out = S->tables[index];
  return LPHT_OK;
}

int lpht_server_stats_get(lpht_server *S, lpht_server_stats *out) {
  if (!S || !out) return LPHT_ERR_INVALID;
  std::lock_guard<std::mutex> lk(S->mu);
  *out = S->st;
  return LPHT_OK;
}

int lpht_server_destroy(lpht_server *S) {
  if (!S) return LPHT_OK;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  if (S->worker.joinable()) S->worker.join();
  destroy_all(S);
  return LPHT_OK;
}

int lpht_server_run_closed_loop(lpht_server *S, const lpht_request *reqs, uint32_t nreq,
                                uint32_t nclients, lpht_completion *done, double *wall_us) {
  if (!S || (nreq && (!reqs || !done)) || nclients == 0) return LPHT_ERR_INVALID;
  std::vector<uint64_t> tickets(nreq, 0);
  std::vector<uint32_t> open;  // request indices in flight
  uint32_t next = 0, finished = 0;
  const double t0 = now_us();
  auto submit_next = [&]() -> int {
    uint64_t tk = 0;
    const int rc = lpht_server_submit(S, &reqs[next], &tk);
    if (rc) return rc;
    tickets[next] = tk;
    open.push_back(next);
    ++next;
    return LPHT_OK;
  };
  while (next < nreq && open.size() < nclients) {
    const int rc = submit_next();
    if (rc) return rc;
  }
  while (finished < nreq) {
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_done.wait(lk, [&] {
        for (uint32_t i : open)
          if (S->reqs[tickets[i]]->done) return true;
        return false;
      });
    }
    std::vector<uint32_t> still;
    std::vector<uint32_t> fin;
    for (uint32_t i : open) {
      lpht_completion c;
      const int rc = lpht_server_poll(S, tickets[i], &c);
      if (rc == LPHT_OK) {
        done[i] = c;
        fin.push_back(i);
      } else {
        still.push_back(i);
      }
    }
    open.swap(still);
    finished += (uint32_t)fin.size();
    for (size_t k = 0; k < fin.size() && next < nreq; ++k) {
      const int rc = submit_next();
      if (rc) return rc;
    }
  }
  if (wall_us) *wall_us = now_us() - t0;
  return LPHT_OK;
}

}  // extern "C"
