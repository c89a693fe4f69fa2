// Inserting kernel that grows the table while it runs (Sec. 5.3.2, "Hiding
// the Migration from the Underlying Application", with the (semi-)synchronized
// protocol and the approximate size of Sec. 5.2).
//
// One cooperative launch (every workgroup resident) processes a batch of
// insertions (or insert-or-add operations).  Wavefront w of W owns the w-th
// of W equal runs of the batch and works through it in chunks of 64 r
// operations (r rounds, up to 64, fewer while the table's free cells are
// few), one operation per lane per round (linear probing with
// compare-and-swap, Alg. 1); equal keys of a chunk are combined in LDS and
// applied once at the chunk's end.  Each wavefront counts its successful
// insertions locally and adds the count to its shard of the global counter
// after a randomised number (1..64 r) of them; when the addition makes the
// shard reach its share of alpha * c, it raises the growing flag.
//
// The protocol of the synchronized variant: a wavefront looks at the flag
// before each chunk (its "busy" period is one chunk); when it is raised the
// wavefront drops its local count and arrives at the growth.  Once every
// wavefront has arrived nobody touches the old table, and all of them
// migrate it together (the dedicated helpers are the kernel's own
// wavefronts) into the table of twice the size that the host reserved
// before the launch, by the block-parallel cluster migration of Lemma 1.
// The last to finish publishes the new table version, with the number of
// moved elements as its base count, and clears the flag.
//
// The growing flag and the version share one word, gen = 2 * epoch + flag,
// so a wavefront can never confuse a finished growth with a pending one.
// Every wait is bounded by the device's constant-rate clock; passing the
// bound sets an error and ends the wavefront (the others then time out too).
//
// While inserting, table cells are read with device-coherent loads and
// written with device-coherent stores or atomics, since different
// wavefronts write the target table and read it afterwards within the same
// launch.  Counters that every wavefront updates are split over separate
// lines (kAsyncShards).

#include <hip/hip_runtime.h>

#include <algorithm>

#include "lpht_async.h"
#include "lpht_device.h"
#include "lpht_migrate.h"

namespace lpht {

namespace {

constexpr int kMigQ = 8;                        // window cells per lane of the migration
constexpr uint32_t kMigB = 64 * kMigQ - 2 * MIG_HALO;  // old cells per migration block (256)
constexpr uint8_t kFlagReserved = 0xFE;
constexpr uint8_t kFlagFull = 0xFF;

__device__ __forceinline__ uint32_t ld32(const uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ u64 ld64(const u64 *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st64(u64 *p, u64 v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Waits until every memory operation this wavefront issued is acknowledged at
// its point of coherence; the "memory" clobber keeps the compiler from moving
// accesses across it.
__device__ __forceinline__ void wait_mem() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// The key word of cell i (PACKED32: the whole cell word, key in the low half).
template <int L>
__device__ __forceinline__ u64 key_at(const void *cells, u64 i) {
  const u64 w = ld64((const u64 *)cells + (L == 0 ? i : 2 * i));
  return L == 0 ? (w & 0xFFFFFFFFull) : w;
}

struct View {
  void *cells;
  uint32_t log2c;
  uint32_t rounds;  // 64-operation rounds per chunk (and the flush bound / 64)
  u64 mask, thr;
};

// A chunk is `rounds` rounds of 64 operations; rounds grows with the table
// so that every wavefront's chunk plus unflushed count, twice, fit half the
// free cells: 256 * W * rounds <= (1 - alpha) c / 2.
__device__ __forceinline__ View view_of(const AsyncArgs &a, uint32_t e, uint32_t W) {
  View v;
  v.cells = a.ladder[e];
  v.log2c = a.log2c + e;
  v.mask = (1ull << v.log2c) - 1;
  v.thr = (u64)(((unsigned __int128)(1ull << v.log2c) * a.alpha_num) / a.alpha_den);
  const u64 free_half = (u64)(((unsigned __int128)(1ull << v.log2c) * (a.alpha_den - a.alpha_num)) /
                              ((u64)a.alpha_den * 2));
  const u64 r = free_half / (256ull * W);
  v.rounds = (uint32_t)std::max<u64>(1, std::min<u64>(kAsyncMaxRounds, r));
  return v;
}

// Waits (lane 0 polls) until *p >= target; false if the bound passed.
__device__ bool wait_ge(const uint32_t *p, uint32_t target, u64 ticks) {
  uint32_t ok = 1;
  if ((threadIdx.x & 63) == 0) {
    const u64 t0 = wall_clock64();
    while (ld32(p) < target) {
      if (wall_clock64() - t0 > ticks) {
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
  }
  return uni(ok) != 0;
}

// Waits until gen moved past `g`; returns the new gen, or ~0u on timeout.
__device__ uint32_t wait_gen_past(const uint32_t *gen, uint32_t g, u64 ticks) {
  uint32_t r = 0;
  if ((threadIdx.x & 63) == 0) {
    const u64 t0 = wall_clock64();
    for (;;) {
      r = ld32(gen);
      if (r != g) break;
      if (wall_clock64() - t0 > ticks) {
        r = ~0u;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
  }
  return uni(r);
}

__device__ __forceinline__ uint32_t lane0_add(uint32_t *p, uint32_t d) {
  uint32_t r = 0;
  if ((threadIdx.x & 63) == 0) r = __hip_atomic_fetch_add(p, d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return uni(r);
}

// Shard of wavefront w, the number of wavefronts on shard `sh`, and the
// number of shards in use.
__device__ __forceinline__ uint32_t shard_size(uint32_t sh, uint32_t W) {
  return W / kAsyncShards + (sh < W % kAsyncShards ? 1u : 0u);
}
__device__ __forceinline__ uint32_t shards_used(uint32_t W) { return W < kAsyncShards ? W : kAsyncShards; }

// Counts the wavefront through barrier k (1, 2, ...) of the running growth:
// after its own memory operations are acknowledged, it adds one to its
// shard's line; the wavefront that completes a shard adds one to `arrived`,
// which reaches k * shards_used(W) when everybody is through.  Returns true
// for the wavefront that completed the barrier.
__device__ bool arrive(AsyncCtl *ctl, uint32_t sh, uint32_t W, uint32_t k) {
  wait_mem();
  uint32_t last = 0;
  if ((threadIdx.x & 63) == 0) {
    const unsigned long long old =
        __hip_atomic_fetch_add(&ctl->arrive[sh].v, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (old == (unsigned long long)k * shard_size(sh, W) - 1) {
      const uint32_t t = __hip_atomic_fetch_add(&ctl->arrived, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      last = t == k * shards_used(W) - 1;
    }
  }
  return uni(last) != 0;
}

// The migration of epoch e into e + 1 by all W wavefronts (this one is
// wavefront `wid`).  Returns false on timeout.  gen is 2e + 1 on entry; the
// last wavefront through sets it to 2(e + 1).
//
//   1. arrival: every wavefront has left the old table;
//   2. block-parallel cluster migration (Sec. 5.3.1, Lemma 1), the same
//      per-block work as the migration kernel: wavefront w takes the w-th
//      of W equal runs of consecutive blocks of kMigB old cells (no shared
//      claim counter), builds each block's owned new range in its LDS region
//      (`wlds`, free between chunks) from the window of old cells around the
//      block and writes it once, empty cells included, so the target needs
//      no zeroing; the next block's window is loaded while the current one is
//      worked on;
//   3. arrival; if some block saw a cluster longer than the halo, every
//      wavefront zeroes the target, arrives once more, and the old table's
//      live elements are inserted into it with compare-and-swap instead;
//   4. the last wavefront through publishes the new version.
// Outside the migration every access to the tables is device-coherent by
// itself (agent-scope relaxed atomic loads, stores and read-modify-writes).
// The block migration uses plain loads and stores, bracketed by two
// agent-scope fences per wavefront: one after the first arrival (this XCD's
// L2 may hold lines of the old table older than the inserters' atomics) and
// one before the second (the new cells sit in this XCD's L2 until written
// back).
template <int L>
__device__ bool migrate(const AsyncArgs &a, const uint32_t (*T)[256], uint32_t e, uint32_t W, uint32_t wid,
                        u64 ticks, unsigned char *wlds) {
  AsyncCtl *ctl = a.ctl;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t sh = wid % kAsyncShards, S = shards_used(W);
  const View o = view_of(a, e, W), nv = view_of(a, e + 1, W);
  // 1.
  arrive(ctl, sh, W, 1);
  if (!wait_ge(&ctl->arrived, S, ticks)) return false;
  __threadfence();
  // 2. (the capacity is at least 2^19 cells, a whole number of blocks)
  const u64 oc = 1ull << o.log2c;
  const uint32_t nblocks = (uint32_t)(oc / kMigB);
  long long moved = 0;
  bool overflow = false;
  {
    const uint32_t b0 = (uint32_t)((u64)nblocks * wid / W), b1 = (uint32_t)((u64)nblocks * (wid + 1) / W);
    u64 nk[kMigQ], nvv[kMigQ];
    if (b0 < b1) mig_load_window<L, kMigQ>(nk, nvv, o.cells, o.mask, b0);
    for (uint32_t b = b0; b < b1; ++b) {
      u64 k[kMigQ], v[kMigQ];
#pragma unroll
      for (int q = 0; q < kMigQ; ++q) {
        k[q] = nk[q];
        v[q] = nvv[q];
      }
      if (b + 1 < b1) mig_load_window<L, kMigQ>(nk, nvv, o.cells, o.mask, b + 1);
      moved += mig_block<L, kMigQ>(k, v, b, o.log2c, 1, T, a.crc_hi, a.crc_lo, a.mul, wlds, nv.cells, overflow);
    }
  }
  if (__any(overflow) && lane == 0)
    __hip_atomic_store(&ctl->mig_overflow, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  // 3.
  __threadfence();
  arrive(ctl, sh, W, 2);
  if (!wait_ge(&ctl->arrived, 2 * S, ticks)) return false;
  const bool fallback = uni(ld32(&ctl->mig_overflow)) != 0;
  uint32_t last = 3;  // the barrier after which everything is written
  if (fallback) {
    // zero the target, then re-insert every live element by compare-and-swap
    const u64 nc16 = (L == 0 ? (1ull << nv.log2c) / 2 : (1ull << nv.log2c));  // 16-byte units
    for (;;) {
      const uint32_t item = lane0_add(&ctl->mig_next2, 1);
      const u64 z0 = (u64)item * 4096;
      if (z0 >= nc16) break;
      const u64 z1 = std::min<u64>(nc16, z0 + 4096);
      for (u64 x = z0 + lane; x < z1; x += 64) {
        st64((u64 *)nv.cells + 2 * x, 0ull);
        st64((u64 *)nv.cells + 2 * x + 1, 0ull);
      }
    }
    arrive(ctl, sh, W, 3);
    if (!wait_ge(&ctl->arrived, 3 * S, ticks)) return false;
    last = 4;
    moved = 0;
    for (;;) {
      const uint32_t item = lane0_add(&ctl->mig_next3, 1);
      const u64 b0 = (u64)item * kAsyncMigBlock;
      if (b0 >= oc) break;
      const u64 b1 = std::min<u64>(oc, b0 + kAsyncMigBlock);
      for (u64 i = b0 + lane; i < b1; i += 64) {
        const u64 k = key_at<L>(o.cells, i);
        if (k == kEmpty || k == kTomb) continue;
        const u64 v = L == 0 ? (ld64((const u64 *)o.cells + i) >> 32) : ld64((const u64 *)o.cells + 2 * i + 1);
        u64 p = home_of<L>(T, k, a.crc_hi, a.crc_lo, a.mul, nv.log2c);
        for (u64 step = 0; step <= nv.mask; ++step, p = (p + 1) & nv.mask) {
          if (L == 0) {
            if (cas64((u64 *)nv.cells + p, kEmpty, k | (v << 32)) == kEmpty) break;
          } else if (cas64((u64 *)nv.cells + 2 * p, kEmpty, k) == kEmpty) {
            st64((u64 *)nv.cells + 2 * p + 1, v);
            break;
          }
        }
        ++moved;
      }
    }
  }
  const long long ms = wave_sum(moved);
  if (lane == 0 && ms)
    __hip_atomic_fetch_add(&ctl->moved[sh].v, (unsigned long long)ms, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  // 4.
  if (arrive(ctl, sh, W, last)) {
    // the last one through: the new version begins with base = the moved
    // elements and empty shards
    unsigned long long mv = 0;
    if (lane < S) mv = __hip_atomic_load(&ctl->moved[lane].v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    mv = (unsigned long long)wave_sum((long long)mv);
    if (lane < S) {
      st64(&ctl->moved[lane].v, 0ull);
      st64(&ctl->count[lane].v, 0ull);
      st64(&ctl->arrive[lane].v, 0ull);
    }
    if (lane == 0) {
      st64(&ctl->base, mv);
      __hip_atomic_store(&ctl->mig_next2, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&ctl->mig_next3, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&ctl->mig_overflow, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (fallback) __hip_atomic_fetch_add(&ctl->fallbacks, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&ctl->arrived, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&ctl->epoch, e + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    wait_mem();  // the counters before the new version
    if (lane == 0) __hip_atomic_store(&ctl->gen, 2 * (e + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  return true;
}

// Per-wavefront LDS table that combines equal keys of one chunk (up to 64
// rounds of 64 operations): the first operation of a key in the chunk claims
// its slot and represents it; at the chunk's end the wavefront applies each
// slot once to the table, with the sum of the chunk's values of that key
// (insert: the representative's value), and the representative gets the
// operation's flag (the others 0).  A key that finds no free slot within
// kChunkProbe steps is applied at once, on its own; once three quarters of
// the slots are taken, keys only look for their slot (plain loads over the
// same kChunkProbe steps, stopping at an empty slot) and claim none, so a
// chunk of distinct keys pays little for the table.  A claimed key sits
// fewer than kChunkProbe steps from its start with no empty slot before it,
// so every later operation of that key in the chunk finds it.
constexpr uint32_t kChunkSlots = 512;
constexpr uint32_t kChunkProbe = 16;
struct ChunkLds {
  u64 key[kChunkSlots];
  u64 acc[kChunkSlots];
  u64 rep[kChunkSlots];
};

// A wavefront's LDS: its combining table between growths, the migration's
// window and image during one (the table is empty then and cleared after).
constexpr size_t kWaveLds = sizeof(ChunkLds) > mig_wave_lds(kMigB, 1, 2) ? sizeof(ChunkLds) : mig_wave_lds(kMigB, 1, 2);

template <int L>
__global__ void __launch_bounds__(256) k_async_insert(AsyncArgs a, u64 ticks, uint32_t W) {
  __shared__ uint32_t T[8][256];
  __shared__ __attribute__((aligned(16))) unsigned char wl[4][kWaveLds];
  crc_tables_build(T);
  unsigned char *wlds = wl[threadIdx.x >> 6];
  ChunkLds &C = *reinterpret_cast<ChunkLds *>(wlds);
  AsyncCtl *ctl = a.ctl;
  const uint32_t lane = threadIdx.x & 63;
  for (uint32_t q = lane; q < kChunkSlots; q += 64) {
    C.key[q] = 0;
    C.acc[q] = 0;
  }
  wave_sync();
  uint32_t *gen = &ctl->gen;
  const uint32_t wid = blockIdx.x * 4 + (threadIdx.x >> 6);
  const uint32_t sh = wid % kAsyncShards, S = shards_used(W);
  // this wavefront's operations [pos, end): the wid-th of W equal runs
  u64 pos = (u64)(((unsigned __int128)a.n * wid) / W);
  const u64 end = (u64)(((unsigned __int128)a.n * (wid + 1)) / W);
  uint32_t my = 0;
  View v = view_of(a, 0, W);
  // a shard's share of the insertions that take the table to alpha c: the
  // growth starts when one shard has it, so while none has, the flushed
  // total is below the threshold
  auto share = [&](u64 base) -> u64 { return v.thr > base ? (v.thr - base) / S : 0; };
  u64 tshare = share(a.used0);
  uint32_t rng = 0x9E3779B9u ^ wid * 0x85EBCA6Bu;
  auto next_flush = [&]() {
    rng ^= rng << 13;
    rng ^= rng >> 17;
    rng ^= rng << 5;
    return 1u + rng % (64u * v.rounds);
  };
  uint32_t flush_at = next_flush();
  uint32_t local = 0;
  uint32_t err = 0;
  bool finished = false;
  u64 idle_since = 0;
  for (;;) {
    const uint32_t g = uni(ld32(gen));
    if (g / 2 > my) {  // a growth finished (this wavefront took part in it)
      my = g / 2;
      v = view_of(a, my, W);  // its cells' addresses depend on the load of gen
      tshare = share(ld64(&ctl->base));
    }
    if (g & 1u) {  // a growth of version `my` is pending: arrive and help
      local = 0;  // the migration recounts what was inserted
      if (!migrate<L>(a, T, my, W, wid, ticks, wlds)) {
        err = 1;
        break;
      }
      // the migration used the combining table's LDS
      for (uint32_t q = lane; q < kChunkSlots; q += 64) {
        C.key[q] = 0;
        C.acc[q] = 0;
      }
      wave_sync();
      const uint32_t g2 = wait_gen_past(gen, g, ticks);
      if (g2 == ~0u) {
        err = 1;
        break;
      }
      idle_since = wall_clock64();
      continue;
    }
    if (finished) {
      // the others end their last chunks (and any growth) within the bound
      if (uni(ld32(&ctl->finished)) >= W) break;
      if (wall_clock64() - idle_since > ticks) {
        err = 1;
        break;
      }
      __builtin_amdgcn_s_sleep(4);
      continue;
    }
    if (pos >= end) {
      finished = true;
      idle_since = wall_clock64();
      lane0_add(&ctl->finished, 1);
      continue;
    }
    const u64 base = pos, lim = std::min<u64>(end, pos + 64ull * v.rounds);
    pos = lim;
    // the table operation for key with value d in the current table: 1
    // inserted, 0 present (d added in add mode), kFlagFull no empty cell
    auto apply_op = [&](u64 key, u64 d) -> uint8_t {
      u64 p = home_of<L>(T, key, a.crc_hi, a.crc_lo, a.mul, v.log2c);
      for (u64 step = 0; step <= v.mask; ++step, p = (p + 1) & v.mask) {
        u64 cur = key_at<L>(v.cells, p);
        if (cur == kEmpty) {
          if (L == 0) {
            const u64 want = key | ((d & 0xFFFFFFFFull) << 32);
            const u64 w = cas64((u64 *)v.cells + p, kEmpty, want);
            if (w == kEmpty) return 1;
            cur = w & 0xFFFFFFFFull;
          } else {
            const u64 w = cas64((u64 *)v.cells + 2 * p, kEmpty, key);
            if (w == kEmpty) {
              if (a.add)
                add64((u64 *)v.cells + 2 * p + 1, d);
              else
                st64((u64 *)v.cells + 2 * p + 1, d);
              return 1;
            }
            cur = w;
          }
        }
        if (cur == key) {
          if (a.add) {
            if (L == 0)
              __hip_atomic_fetch_add((uint32_t *)((u64 *)v.cells + p) + 1, (uint32_t)d, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
            else
              add64((u64 *)v.cells + 2 * p + 1, d);
          }
          return 0;
        }
      }
      return kFlagFull;
    };
    // adds the wavefront's new insertions to its local count, flushing it to
    // its shard of the counter (and raising the growing flag) when it
    // reaches the random bound
    auto account = [&](uint32_t ins) {
      local += ins;
      if (local >= flush_at) {
        uint32_t trig = 0;
        if (lane == 0) {
          const unsigned long long before = __hip_atomic_fetch_add(
              &ctl->count[sh].v, (unsigned long long)local, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          trig = before + local >= tshare && my + 1 < a.nladder;
        }
        local = 0;
        flush_at = next_flush();
        if (uni(trig) && lane == 0) {
          uint32_t expect = 2 * my;
          __hip_atomic_compare_exchange_strong(gen, &expect, 2 * my + 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    };
    uint32_t taken = 0;  // slots claimed in this chunk (wavefront-uniform)
    for (uint32_t rd = 0; rd < v.rounds; ++rd) {
      // one operation per lane; equal keys of the chunk meet in LDS
      const u64 i = base + 64ull * rd + lane;
      const bool claim = taken < kChunkSlots / 4 * 3;
      uint32_t inserted = 0;
      bool lead = false;
      if (i < lim) {
        const u64 key = L == 0 ? (u64)((const uint32_t *)a.keys)[i] : ((const u64 *)a.keys)[i];
        const u64 d = a.vals ? (L == 0 ? (u64)((const uint32_t *)a.vals)[i] : ((const u64 *)a.vals)[i]) : 1;
        if (key <= kTomb) {
          err |= 4;
          if (a.flags) a.flags[i] = kFlagReserved;
        } else {
          uint32_t slot = (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> 55);  // 9 bits
          bool held = false;
          if (claim) {
            for (uint32_t t = 0; t < kChunkProbe; ++t, slot = (slot + 1) & (kChunkSlots - 1)) {
              const u64 prev = atomicCAS((unsigned long long *)&C.key[slot], 0ull, (unsigned long long)key);
              if (prev == 0) {
                lead = held = true;
                break;
              }
              if (prev == key) {
                held = true;
                break;
              }
            }
          } else {
            // no lane claims a slot in this round: the keys are fixed
            for (uint32_t t = 0; t < kChunkProbe; ++t, slot = (slot + 1) & (kChunkSlots - 1)) {
              const u64 k = C.key[slot];
              if (k == key) {
                held = true;
                break;
              }
              if (k == 0) break;
            }
          }
          if (held) {
            if (lead) {
              C.rep[slot] = i;
              if (!a.add) C.acc[slot] = d;
            }
            if (a.add) atomicAdd((unsigned long long *)&C.acc[slot], (unsigned long long)d);
            if (!lead && a.flags) a.flags[i] = 0;  // the representative's flag is the operation's
          } else {
            const uint8_t f = apply_op(key, d);
            inserted = f == 1;
            if (a.flags) a.flags[i] = f;
          }
        }
      }
      taken += (uint32_t)__popcll(__ballot(lead));
      account((uint32_t)__popcll(__ballot(inserted)));
    }
    // the chunk's combined operations, one per distinct key
    wave_sync();
    uint32_t ins = 0;
    for (uint32_t q = lane; q < kChunkSlots; q += 64) {
      const u64 k = C.key[q];
      if (k == 0) continue;
      const uint8_t f = apply_op(k, C.acc[q]);
      ins += f == 1;
      if (a.flags) a.flags[C.rep[q]] = f;
      C.key[q] = 0;
      C.acc[q] = 0;
    }
    wave_sync();
    account((uint32_t)wave_sum((long long)ins));
  }
  // timeouts are set by the whole wavefront, reserved keys by single lanes
  const uint32_t werr = uni(err & 3u) | (__ballot((err & 4u) != 0) ? 4u : 0u);
  if (werr && lane == 0) {
    atomicOr(&ctl->err, werr);
    if (werr & 4u) atomicOr(&a.status->err, kErrReserved);
  }
}

__global__ void k_async_init(AsyncCtl *ctl, u64 used0) {
  for (uint32_t i = threadIdx.x; i < sizeof(AsyncCtl) / 8; i += blockDim.x) ((unsigned long long *)ctl)[i] = 0;
  __syncthreads();
  if (threadIdx.x == 0) ctl->base = used0;
}

}  // namespace

uint32_t async_grid(int device) {
  int coop = 0, ncu = 0;
  if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, device) != hipSuccess || !coop) return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || ncu <= 0)
    return 0;
  int b0 = 0, b1 = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b0, k_async_insert<0>, 256, 0) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&b1, k_async_insert<1>, 256, 0) != hipSuccess)
    return 0;
  const int per = std::min(2, std::min(b0, b1));
  return per > 0 ? (uint32_t)(per * ncu) : 0u;
}

uint32_t async_min_log2(uint32_t grid, uint32_t alpha_num, uint32_t alpha_den) {
  // In flight beyond the flushed count: per wavefront one chunk plus one
  // unflushed batch of insertions, twice (before and while the growth is
  // noticed); they must fit half the free cells (1 - alpha) c.
  const unsigned __int128 slack = (unsigned __int128)grid * 4 * (kAsyncChunk + kAsyncFlushMax) * 2;
  uint32_t lg = 6;
  while (lg < 40 && ((unsigned __int128)(1ull << lg) * (alpha_den - alpha_num)) < slack * 2 * alpha_den) ++lg;
  return lg;
}

hipError_t launch_async_insert(const AsyncArgs &a, hipStream_t s) {
  drop_stale_error();
  if (a.layout > 1 || !a.ctl || !a.grid || a.nladder < 1 || a.nladder > kAsyncLadder + 1) return hipErrorInvalidValue;
  int dev = 0, khz = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_async_init, dim3(1), dim3(64), 0, s, a.ctl, (u64)a.used0);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  AsyncArgs args = a;
  u64 ticks = (u64)khz * 1000ull * 2;  // two seconds
  uint32_t W = a.grid * 4;
  void *kargs[] = {&args, &ticks, &W};
  e = hipLaunchCooperativeKernel(a.layout == 0 ? (const void *)k_async_insert<0> : (const void *)k_async_insert<1>,
                                 dim3(a.grid), dim3(256), kargs, 0, s);
  return e;
}

}  // namespace lpht
