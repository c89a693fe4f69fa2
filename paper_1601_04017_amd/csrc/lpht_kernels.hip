// HIP kernels of liblpht for gfx950 (CDNA4, wave64).
//
// Bulk operations of the folklore linear-probing table (Maier, Sanders,
// Dementiev, arXiv 1601.04017, Sec. 4, Algorithm 1; tombstones Sec. 5.4) and
// its block-parallel cluster migration (Sec. 5.3.1, Lemma 1).
//
// Execution model
// ---------------
// A "group" of G lanes (G = 1, 2, 4, 8, 16; all in one wavefront) works on one
// operation at a time.  The group scans the table in windows of G consecutive
// cells aligned to G, so that for G = 8 (16-byte cells) or G = 16 (8-byte
// cells) one window is one 128-byte line read by one coalesced load.  The
// first window starts at the operation's home cell; lanes before it are
// masked.  Group-wide decisions come from wave ballots, so the lanes of a
// group always take the same branches.  When an operation finishes, its group
// immediately takes the next one (grid-stride over operations), so short and
// long probe sequences do not hold each other up.
//
// The hash is the paper's: two CRC-32C register updates with different seeds
// give the upper and lower 32 bits (Sec. 8.3).  gfx950 has no CRC
// instruction, so each workgroup builds slicing-by-8 tables for the
// Castagnoli polynomial in LDS.  The register update has no inversion and is
// linear over GF(2), so CRC(seed, x) = CRC(0, x) ^ CRC(0, seed): one table
// evaluation per key plus two constants computed on the host.  The cell
// position is the top log2(c) bits of the 64-bit hash (scaling map of
// Sec. 5.3.1).
//
// Atomics: 64-bit compare-and-swap claims an empty cell (the whole cell for
// the packed layout, the key word for the 16-byte layout); a failed CAS
// returns the current word, which is examined in place of the cell (the
// "revisit" of Algorithm 1).  Increments use fetch-and-add and overwrites a
// single store (Sec. 4).  All table atomics are device (agent) scope.

#include <hip/hip_runtime.h>

#include <atomic>

#include <algorithm>
#include <cstddef>
#include <type_traits>
#include <stdint.h>

#include "lpht_device.h"
#include "lpht_migrate.h"
#include "lpht_internal.h"

namespace lpht {

// ---------------------------------------------------------------- bulk kernel

template <int G>
__device__ __forceinline__ uint32_t group_bits(uint64_t ballot, uint32_t gbase) {
  if (G == 64) return (uint32_t)ballot;  // unused width
  return (uint32_t)((ballot >> gbase) & ((1ull << G) - 1));
}

template <int LAYOUT>
__device__ __forceinline__ u64 load_key_in(const void *keys, u64 i) {
  if (LAYOUT == 0) return ((const uint32_t *)keys)[i];
  return ((const u64 *)keys)[i];
}

// Loads and stores of caller arrays.  RESIDENT: the arrays are the device
// staging of the resident serving kernel, which other wavefronts (on other
// XCDs) write and read during the same launch; accesses are device-coherent
// (agent-scope relaxed atomics, which bypass the per-CU and per-XCD caches).
template <int LAYOUT, bool RESIDENT>
__device__ __forceinline__ u64 ld_word(const void *a, u64 i) {
  if (!RESIDENT) return load_key_in<LAYOUT>(a, i);
  if (LAYOUT == 0) return __hip_atomic_load((const uint32_t *)a + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return __hip_atomic_load((const u64 *)a + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <bool RESIDENT>
__device__ __forceinline__ uint8_t ld_kind(const uint8_t *a, u64 i) {
  if (!RESIDENT) return a[i];
  return __hip_atomic_load(a + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <bool RESIDENT>
__device__ __forceinline__ u64 ld_u64(const u64 *a) {
  if (!RESIDENT) return *a;
  return __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <bool RESIDENT, typename W>
__device__ __forceinline__ void st_out(W *p, W v) {
  if (!RESIDENT)
    *p = v;
  else
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int LAYOUT, bool RESIDENT = false>
__device__ __forceinline__ void store_val_out(void *out, u64 i, u64 v) {
  if (LAYOUT == 0)
    st_out<RESIDENT>((uint32_t *)out + i, (uint32_t)v);
  else
    st_out<RESIDENT>((u64 *)out + i, v);
}

// Writes of values into cells.  Plain stores: a value is written either by
// the lane whose CAS claimed the cell (no other lane writes it in that call)
// or as an overwrite whose result may be any one of the concurrent values;
// the line stays in L2 and is written back whole.
// (COH: a device-coherent store, for the resident serving kernel.)
template <bool COH = false>
__device__ __forceinline__ void put64(u64 *p, u64 v) {
  if (COH)
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else
    *p = v;
}
template <bool COH = false>
__device__ __forceinline__ void put32(uint32_t *p, uint32_t v) {
  if (COH)
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else
    *p = v;
}

// Operations per wavefront round.  A wavefront takes rounds of ROUND
// consecutive operations; its groups work through them, results are staged
// in LDS, and at the end of the round the wavefront writes them out as whole
// lines (128 flag bytes, 128 values), so output lines are written once.
constexpr uint32_t ROUND = kRound;

__host__ __device__ constexpr uint32_t bulk_lds_bytes_per_wave(int op) {
  return ROUND * (op == OP_FIND ? 9u : 1u);
}

// Single-table calls also stage each round's keys and their home positions
// in LDS (read with one coalesced load per lane, hashed once per operation),
// so a group starts its next operation without a dependent global load.
constexpr uint32_t kStageBytesPerWave = ROUND * 16u;

// Marks, in the staged flags of a round, an operation that belongs to another
// phase of a mixed request; its flag byte in memory is left as it is.
constexpr uint8_t kSkipFlag = 0xFD;

// One round of a bulk call: operations [rbase, rbase + cnt) of A, each taken
// by a group of G lanes; results are staged in LDS (wflag, wout) and written
// as whole lines at the end.
//   OP_FIND    : found flag + value
//   OP_INSERT  : insert(k, d)
//   OP_UPSERT  : insertOrUpdate(k, d, up)
//   OP_UPDATE  : update(k, d, up)
//   OP_ERASE   : tombstone delete
// With A.kinds set, only operations whose kind byte equals A.kind_sel are
// performed (phase order of mixed requests: finds, then insert-or-increments,
// then erases); a find phase writes value 0 for the other operations.
//
// RESIDENT: a round of the resident serving kernel (device-coherent accesses
// to cells and staging); the round's keys and kinds are first read into LDS
// (skeys, skinds: ROUND entries each) with one coalesced load per lane.
template <int LAYOUT, int OP, int UP, int G, bool RESIDENT = false>
__device__ __forceinline__ void bulk_round(const BulkArgs &A, const uint32_t (*T)[256], uint8_t *wflag,
                                           u64 *wout, const u64 rbase, const uint32_t cnt,
                                           long long &d_used, long long &d_live, uint32_t &err,
                                           u64 *skeys = nullptr, uint8_t *skinds = nullptr,
                                           u64 *shome = nullptr) {
  constexpr uint32_t NGW = 64 / G;            // groups per wavefront
  constexpr uint32_t PER_GROUP = ROUND / NGW; // operations per group per round
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t gl = lane & (G - 1);  // lane within the group
  const uint32_t gbase = lane - gl;    // first lane of the group in the wave
  const uint32_t gi = lane / G;        // group within the wave
  const u64 cap = 1ull << A.log2c;
  const u64 mask = cap - 1;
  const u64 max_windows = cap / G;     // plus one when the home is unaligned
  const bool flags8 = A.flags && (((uintptr_t)A.flags & 7) == 0);
  const bool vals_vec = (OP == OP_FIND) && A.vals_out && (((uintptr_t)A.vals_out & 15) == 0);
  uint32_t j = 0;
  u64 i = 0, k = 0, d = 1, base = 0, windows = 0, limit = 0;
  uint32_t first = 0;
  bool active = false;
  if (RESIDENT) {
    static_assert(ROUND == 128, "two operations per lane");
    u64 k0 = 0, k1 = 0;
    uint8_t c0 = 0, c1 = 0;
    const bool in0 = lane < cnt, in1 = lane + 64 < cnt;
    if (in0) k0 = ld_word<LAYOUT, true>(A.keys, rbase + lane);
    if (in1) k1 = ld_word<LAYOUT, true>(A.keys, rbase + lane + 64);
    if (A.kinds) {
      if (in0) c0 = ld_kind<true>(A.kinds, rbase + lane);
      if (in1) c1 = ld_kind<true>(A.kinds, rbase + lane + 64);
    }
    skeys[lane] = k0;
    skeys[lane + 64] = k1;
    skinds[lane] = c0;
    skinds[lane + 64] = c1;
    wave_sync();
  } else if (shome) {
#pragma unroll
    for (uint32_t q = 0; q < 2; ++q) {
      const uint32_t loc = lane + 64 * q;
      if (loc < cnt) {
        const u64 kk = load_key_in<LAYOUT>(A.keys, rbase + loc);
        skeys[loc] = kk;
        shome[loc] = (kk == kEmpty || kk == kTomb) ? 0 : home_of<LAYOUT>(T, kk, A.crc_hi, A.crc_lo, A.mul, A.log2c);
      }
    }
    wave_sync();
  }

  // Takes the group's next operation of the round (reserved keys are
  // answered at once).
  auto start = [&]() {
    active = false;
    while (j < PER_GROUP) {
      const uint32_t loc = gi + j * NGW;
      if (loc >= cnt) {
        j = PER_GROUP;
        break;
      }
      i = rbase + loc;
      if (A.kinds && (RESIDENT ? skinds[loc] : A.kinds[i]) != A.kind_sel) {
        // an operation of another phase of a mixed request
        if (gl == 0) {
          wflag[loc] = kSkipFlag;
          if (OP == OP_FIND) wout[loc] = 0;
        }
        ++j;
        continue;
      }
      k = (RESIDENT || shome) ? skeys[loc] : load_key_in<LAYOUT>(A.keys, i);
      if (k == kEmpty || k == kTomb) {
        err |= kErrReserved;
        if (gl == 0) {
          wflag[loc] = 0xFE;
          if (OP == OP_FIND) wout[loc] = 0;
        }
        ++j;
        continue;
      }
      d = A.vals ? ld_word<LAYOUT, RESIDENT>(A.vals, i) : 1;
      const u64 h = (!RESIDENT && shome) ? shome[loc] : home_of<LAYOUT>(T, k, A.crc_hi, A.crc_lo, A.mul, A.log2c);
      base = h & ~(u64)(G - 1);
      first = (uint32_t)(h & (G - 1));
      windows = 0;
      limit = max_windows + (first ? 1 : 0);
      active = true;
      return;
    }
  };

  auto finish = [&](uint8_t flag, u64 v) {
    if (gl == 0) {
      const uint32_t loc = gi + j * NGW;
      wflag[loc] = flag;
      if (OP == OP_FIND) wout[loc] = v;
    }
    ++j;
    start();
  };

  // Single-table finds one lane per operation: a lane probes both of its
  // operations of the round together, so two random loads are in flight per
  // lane instead of one after the other.
  constexpr bool kPairFind = OP == OP_FIND && G == 1 && !RESIDENT;
  const bool pair = kPairFind && shome && !A.kinds;
  if (pair) {
    static_assert(ROUND == 128, "two operations per lane");
    u64 key[2], pos[2], val[2] = {0, 0}, steps[2] = {0, 0};
    bool act[2];
    uint8_t fl[2] = {0, 0};
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const uint32_t loc = lane + 64 * q;
      act[q] = loc < cnt;
      key[q] = act[q] ? skeys[loc] : 0;
      pos[q] = act[q] ? shome[loc] : 0;
      if (act[q] && (key[q] == kEmpty || key[q] == kTomb)) {
        err |= kErrReserved;
        fl[q] = 0xFE;
        act[q] = false;
      }
    }
    while (act[0] || act[1]) {
      u64 ck[2], cv[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        ck[q] = kEmpty;
        cv[q] = 0;
        if (act[q]) {
          if (LAYOUT == 0) {
            const u64 w = Cells<0>::word<false>(A.cells, pos[q]);
            ck[q] = Cells<0>::key_of(w);
            cv[q] = Cells<0>::val_of(w);
          } else {
            const u64x2 c = Cells<1>::cell<false>(A.cells, pos[q]);
            ck[q] = c.x;
            cv[q] = c.y;
          }
        }
      }
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        if (!act[q]) continue;
        if (ck[q] == key[q]) {
          fl[q] = 1;
          val[q] = cv[q];
          act[q] = false;
        } else if (ck[q] == kEmpty || ++steps[q] > mask) {
          act[q] = false;  // absent (or every cell probed)
        } else {
          pos[q] = (pos[q] + 1) & mask;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const uint32_t loc = lane + 64 * q;
      if (loc < cnt) {
        wflag[loc] = fl[q];
        wout[loc] = val[q];
      }
    }
  } else {
  start();
  while (__any(active)) {
    if (active) {
      const u64 idx = base + gl;
      u64 ck, cv = 0;
      if (LAYOUT == 0) {
        const u64 w = Cells<0>::word<RESIDENT>(A.cells, idx);
        ck = Cells<0>::key_of(w);
        cv = Cells<0>::val_of(w);
      } else if (OP == OP_FIND) {
        const u64x2 c = Cells<1>::cell<RESIDENT>(A.cells, idx);
        ck = c.x;
        cv = c.y;
      } else {
        ck = Cells<1>::key<RESIDENT>(A.cells, idx);
      }
      bool done = false;
      uint8_t flag = 0;
      u64 outv = 0;
      // Evaluate the window; a failed CAS updates the lane's key and the
      // window is evaluated again from that lane on.
      while (true) {
        const bool valid = gl >= first;
        const uint32_t bh = group_bits<G>(__ballot(valid && ck == k), gbase);
        const uint32_t be = group_bits<G>(__ballot(valid && ck == kEmpty), gbase);
        const uint32_t ev = bh | be;
        if (ev == 0) break;
        const uint32_t jl = __builtin_ctz(ev);
        const uint32_t src = gbase + jl;
        if ((bh >> jl) & 1u) {
          // key present at lane jl
          if (OP == OP_FIND) {
            outv = __shfl(cv, src, 64);
            flag = 1;
            done = true;
          } else if (OP == OP_INSERT) {
            flag = 0;
            done = true;
          } else if (OP == OP_UPSERT || OP == OP_UPDATE) {
            if (gl == jl) {
              if (LAYOUT == 0) {
                u64 *w = (u64 *)A.cells + idx;
                if (UP == 1)
                  add64(w, d << 32);
                else
                  put32<RESIDENT>((uint32_t *)w + 1, (uint32_t)d);
              } else {
                u64 *v = (u64 *)A.cells + 2 * idx + 1;
                if (UP == 1)
                  add64(v, d);
                else
                  put64<RESIDENT>(v, d);
              }
            }
            flag = (OP == OP_UPDATE) ? 1 : 0;
            done = true;
          } else {  // OP_ERASE
            u64 old = 0;
            bool won = false;
            if (gl == jl) {
              if (LAYOUT == 0) {
                const u64 w = ((u64)cv << 32) | k;
                old = cas64((u64 *)A.cells + idx, w, (w & ~0xFFFFFFFFull) | kTomb);
                won = (old == w);
                if (!won) old &= 0xFFFFFFFFull;
              } else {
                old = cas64((u64 *)A.cells + 2 * idx, k, kTomb);
                won = (old == k);
              }
              if (won) d_live -= 1;
            }
            won = __shfl((int)won, src, 64) != 0;
            if (won) {
              flag = 1;
              done = true;
            } else {
              // another operation changed this cell first; look at what is there now
              old = __shfl(old, src, 64);
              if (gl == jl) ck = old;
              if (LAYOUT == 0 && gl == jl && old == k) {
                // only the value changed: reload the word and retry
                const u64 w = Cells<0>::word<RESIDENT>(A.cells, idx);
                ck = Cells<0>::key_of(w);
                cv = Cells<0>::val_of(w);
              }
              first = jl;
              continue;
            }
          }
        } else {
          // empty cell at lane jl: k is absent
          if (OP == OP_FIND || OP == OP_UPDATE || OP == OP_ERASE) {
            flag = 0;
            outv = 0;
            done = true;
          } else {
            u64 old = 0;
            if (gl == jl) {
              if (LAYOUT == 0) {
                old = cas64((u64 *)A.cells + idx, 0ull, (d << 32) | k);
                if (old == 0) {
                  d_used += 1;
                  d_live += 1;
                }
              } else {
                old = cas64((u64 *)A.cells + 2 * idx, kEmpty, k);
                if (old == kEmpty) {
                  u64 *v = (u64 *)A.cells + 2 * idx + 1;
                  if (OP == OP_UPSERT && UP == 1)
                    add64(v, d);  // concurrent increments of the same key also add
                  else
                    put64<RESIDENT>(v, d);
                  d_used += 1;
                  d_live += 1;
                }
              }
            }
            old = __shfl(old, src, 64);
            const u64 okey = (LAYOUT == 0) ? (old & 0xFFFFFFFFull) : old;
            if (old == 0) {
              flag = 1;
              done = true;
            } else if (okey == k) {
              // lost the race to an insertion of the same key
              if (OP == OP_UPSERT && gl == jl) {
                if (LAYOUT == 0) {
                  u64 *w = (u64 *)A.cells + idx;
                  if (UP == 1)
                    add64(w, d << 32);
                  else
                    put32<RESIDENT>((uint32_t *)w + 1, (uint32_t)d);
                } else {
                  u64 *v = (u64 *)A.cells + 2 * idx + 1;
                  if (UP == 1)
                    add64(v, d);
                  else
                    put64<RESIDENT>(v, d);
                }
              }
              flag = 0;
              done = true;
            } else {
              // another key took the cell: revisit it with that key
              if (gl == jl) ck = okey;
              first = jl;
              continue;
            }
          }
        }
        break;
      }
      if (done) {
        finish(flag, outv);
      } else {
        base = (base + G) & mask;
        first = 0;
        windows += 1;
        if (windows >= limit) {
          if (OP == OP_INSERT || OP == OP_UPSERT) {
            err |= kErrFull;
            finish(0xFF, 0);
          } else {
            finish(0, 0);
          }
        }
      }
    }
  }
  }
  // write the round's results as whole lines
  wave_sync();
  if (A.flags) {
    if (cnt == ROUND && flags8) {
      if (lane < ROUND / 8) {
        u64 w = ((const u64 *)wflag)[lane];
        if (A.kinds) {
          // keep the flags other phases wrote
          const u64 old = ld_u64<RESIDENT>((const u64 *)(A.flags + rbase) + lane);
#pragma unroll
          for (int b = 0; b < 8; ++b) {
            const u64 m = 0xFFull << (8 * b);
            if (((w & m) >> (8 * b)) == kSkipFlag) w = (w & ~m) | (old & m);
          }
        }
        st_out<RESIDENT>((u64 *)(A.flags + rbase) + lane, w);
      }
    } else {
      for (uint32_t t = lane; t < cnt; t += 64)
        if (wflag[t] != kSkipFlag) st_out<RESIDENT>(A.flags + rbase + t, wflag[t]);
    }
  }
  if (OP == OP_FIND && A.vals_out) {
    if (cnt == ROUND && vals_vec && !RESIDENT) {
      if (LAYOUT == 0) {
        typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
        u32x2 v = {(uint32_t)wout[2 * lane], (uint32_t)wout[2 * lane + 1]};
        ((u32x2 *)((uint32_t *)A.vals_out + rbase))[lane] = v;
      } else {
        u64x2 v = {wout[2 * lane], wout[2 * lane + 1]};
        ((u64x2 *)((u64 *)A.vals_out + rbase))[lane] = v;
      }
    } else {
      for (uint32_t t = lane; t < cnt; t += 64) store_val_out<LAYOUT, RESIDENT>(A.vals_out, rbase + t, wout[t]);
    }
  }
  wave_sync();
}

// Single-table bulk call: wavefronts take rounds of A in grid-stride order.
template <int LAYOUT, int OP, int UP, int G>
__global__ void __launch_bounds__(1024) k_bulk(BulkArgs A) {
  __shared__ uint32_t T[8][256];
  __shared__ long long s_acc[2];
  __shared__ uint32_t s_err;
  extern __shared__ __attribute__((aligned(16))) unsigned char dyn_lds[];
  crc_tables_build(T);
  const uint32_t wave = threadIdx.x >> 6;
  const uint32_t nwb = blockDim.x >> 6;
  uint8_t *wflag = dyn_lds + (OP == OP_FIND ? nwb * ROUND * 8 : 0) + wave * ROUND;
  u64 *wout = (u64 *)dyn_lds + wave * ROUND;  // FIND only
  u64 *skeys = (u64 *)(dyn_lds + nwb * bulk_lds_bytes_per_wave(OP)) + wave * 2 * ROUND;
  u64 *shome = skeys + ROUND;
  long long d_used = 0, d_live = 0;
  uint32_t err = 0;
  const u64 nrounds = (A.n + ROUND - 1) / ROUND;
  const u64 gw = (u64)blockIdx.x * nwb + wave;
  const u64 nw = (u64)gridDim.x * nwb;
  for (u64 r = gw; r < nrounds; r += nw) {
    const u64 rbase = r * ROUND;
    const uint32_t cnt = (uint32_t)((A.n - rbase) < ROUND ? (A.n - rbase) : ROUND);
    bulk_round<LAYOUT, OP, UP, G>(A, T, wflag, wout, rbase, cnt, d_used, d_live, err, skeys, nullptr, shome);
  }
  flush_counts(A.status, d_used, d_live, err, s_acc, &s_err);
}

// Multi-table bulk call: descriptor j covers rounds [round_start[j],
// round_start[j+1]) of one launch, so tables and calls of uneven sizes share
// one grid.  Counts go to each descriptor's table after every round.
template <int LAYOUT, int OP, int UP, int G>
__global__ void __launch_bounds__(1024) k_bulk_multi(const BulkArgs *descs, const u64 *round_start,
                                                     uint32_t ndesc) {
  __shared__ uint32_t T[8][256];
  extern __shared__ __attribute__((aligned(16))) unsigned char dyn_lds[];
  crc_tables_build(T);
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wave = threadIdx.x >> 6;
  const uint32_t nwb = blockDim.x >> 6;
  uint8_t *wflag = dyn_lds + (OP == OP_FIND ? nwb * ROUND * 8 : 0) + wave * ROUND;
  u64 *wout = (u64 *)dyn_lds + wave * ROUND;  // FIND only
  const u64 total = round_start[ndesc];
  const u64 gw = (u64)blockIdx.x * nwb + wave;
  const u64 nw = (u64)gridDim.x * nwb;
  for (u64 r = gw; r < total; r += nw) {
    uint32_t lo = 0, hi = ndesc;  // last j with round_start[j] <= r
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (round_start[mid] <= r) lo = mid; else hi = mid;
    }
    const BulkArgs A = descs[lo];
    const u64 rbase = (r - round_start[lo]) * ROUND;
    const uint32_t cnt = (uint32_t)((A.n - rbase) < ROUND ? (A.n - rbase) : ROUND);
    long long d_used = 0, d_live = 0;
    uint32_t err = 0;
    bulk_round<LAYOUT, OP, UP, G>(A, T, wflag, wout, rbase, cnt, d_used, d_live, err);
    const long long u = wave_sum(d_used), l = wave_sum(d_live);
    uint32_t e = err;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) e |= __shfl_xor(e, o, 64);
    if (lane == 0) {
      CountSlot *cs = &A.status->slot[gw % kCountSlots];
      if (u) add64(&cs->used, (u64)u);
      if (l) add64(&cs->live, (u64)l);
      if (e) atomicOr(&A.status->err, e);
    }
  }
}

// ---------------------------------------------------------------- aggregated insert-or-increment
//
// With the update function "add", the outcome of a bulk insertOrUpdate does
// not depend on the order of its operations, so operations on equal keys can
// be combined before they reach the table (the paper avoids contention on
// skewed inputs by sorting, Sec. 5.5; here a workgroup combines in LDS).  A
// workgroup takes chunks of AGG_CHUNK operations; equal keys of a chunk meet
// in an LDS hash table and leave it as one upsert with the summed increment.
// A key seen at least HOT_MIN times in one chunk moves to a second LDS table
// that lives for the whole kernel and is written back once at the end, so the
// hottest keys cost one global atomic per workgroup instead of one per
// occurrence.  Each combined upsert is issued by a representative operation
// (the first to claim the LDS slot); it carries the "inserted" flag, every
// other operation of that key reports "updated".  Exactly one operation per
// inserted key therefore reports true, as in the sequential table.
//
// The host only selects this kernel when the table cannot run out of empty
// cells during the call, so no combined operation can fail with "full".

constexpr int AGG_BLOCK = 1024;
constexpr int AGG_PER_THREAD = 2;
constexpr int AGG_CHUNK = AGG_BLOCK * AGG_PER_THREAD;  // operations per chunk
constexpr int AGG_SLOTS = 2 * AGG_CHUNK;              // LDS hash slots per chunk
constexpr int HOT_SLOTS = 256;                        // kernel-lifetime hot keys
constexpr int HOT_MAX = (HOT_SLOTS * 3) / 4;          // at most 3/4 full
constexpr uint32_t HOT_MIN = 3;                       // promotion threshold

template <int LAYOUT>
__global__ void __launch_bounds__(AGG_BLOCK) k_upsert_add_agg(BulkArgs A) {
  __shared__ uint32_t T[8][256];
  __shared__ u64 s_key[AGG_SLOTS];
  __shared__ u64 s_sum[AGG_SLOTS];
  __shared__ uint32_t s_cnt[AGG_SLOTS];
  __shared__ uint32_t s_rep[AGG_SLOTS];
  __shared__ u64 h_key[HOT_SLOTS];
  __shared__ u64 h_sum[HOT_SLOTS];
  __shared__ u64 h_rep[HOT_SLOTS];
  __shared__ uint32_t h_n;
  __shared__ long long s_acc[2];
  __shared__ uint32_t s_err;

  crc_tables_build(T);
  for (int s = threadIdx.x; s < AGG_SLOTS; s += AGG_BLOCK) {
    s_key[s] = 0;
    s_sum[s] = 0;
    s_cnt[s] = 0;
  }
  for (int s = threadIdx.x; s < HOT_SLOTS; s += AGG_BLOCK) {
    h_key[s] = 0;
    h_sum[s] = 0;
  }
  if (threadIdx.x == 0) h_n = 0;
  __syncthreads();

  long long d_used = 0, d_live = 0;
  uint32_t err = 0;
  const u64 nchunks = (A.n + AGG_CHUNK - 1) / AGG_CHUNK;
  for (u64 ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
    const u64 base = ch * AGG_CHUNK;
    // combine equal keys of the chunk in LDS
#pragma unroll
    for (int j = 0; j < AGG_PER_THREAD; ++j) {
      const uint32_t off = j * AGG_BLOCK + threadIdx.x;
      const u64 i = base + off;
      if (i >= A.n) continue;
      const u64 k = load_key_in<LAYOUT>(A.keys, i);
      if (k == kEmpty || k == kTomb) {
        err |= kErrReserved;
        if (A.flags) A.flags[i] = 0xFE;
        continue;
      }
      const u64 d = A.vals ? load_key_in<LAYOUT>(A.vals, i) : 1;
      const uint32_t hc = ((LAYOUT == 0) ? crc0_u32(T, (uint32_t)k) : crc0_u64(T, k)) ^ A.crc_lo;
      uint32_t hs = (hc >> 11) & (HOT_SLOTS - 1);
      bool hot = false;
      for (int q = 0; q < HOT_SLOTS; ++q) {
        const u64 hk = h_key[hs];
        if (hk == k) {
          hot = true;
          break;
        }
        if (hk == 0) break;
        hs = (hs + 1) & (HOT_SLOTS - 1);
      }
      if (hot) {
        atomicAdd(&h_sum[hs], d);
        if (A.flags) A.flags[i] = 0;
        continue;
      }
      uint32_t s = hc & (AGG_SLOTS - 1);
      bool rep = false;
      while (true) {
        const u64 old = atomicCAS(&s_key[s], 0ull, k);
        if (old == 0) {
          rep = true;
          s_rep[s] = off;
          break;
        }
        if (old == k) break;
        s = (s + 1) & (AGG_SLOTS - 1);
      }
      atomicAdd(&s_sum[s], d);
      atomicAdd(&s_cnt[s], 1u);
      if (!rep && A.flags) A.flags[i] = 0;
    }
    __syncthreads();
    // one upsert per distinct key of the chunk, or promotion to the hot table
    for (int s = threadIdx.x; s < AGG_SLOTS; s += AGG_BLOCK) {
      const u64 k = s_key[s];
      if (k == 0) continue;
      const u64 sum = s_sum[s];
      const uint32_t cnt = s_cnt[s];
      const u64 rep = base + s_rep[s];
      s_key[s] = 0;
      s_sum[s] = 0;
      s_cnt[s] = 0;
      bool promoted = false;
      if (cnt >= HOT_MIN && atomicAdd(&h_n, 1u) < (uint32_t)HOT_MAX) {
        const uint32_t hc = ((LAYOUT == 0) ? crc0_u32(T, (uint32_t)k) : crc0_u64(T, k)) ^ A.crc_lo;
        uint32_t hs = (hc >> 11) & (HOT_SLOTS - 1);
        while (atomicCAS(&h_key[hs], 0ull, k) != 0ull) hs = (hs + 1) & (HOT_SLOTS - 1);
        h_sum[hs] = sum;
        h_rep[hs] = rep;
        promoted = true;
      }
      if (!promoted) {
        const uint8_t f = upsert_add_one<LAYOUT>(A, T, k, sum, d_used, d_live, err);
        if (A.flags) A.flags[rep] = f;
      }
    }
    __syncthreads();
  }
  for (int hs = threadIdx.x; hs < HOT_SLOTS; hs += AGG_BLOCK) {
    const u64 k = h_key[hs];
    if (k == 0) continue;
    const uint8_t f = upsert_add_one<LAYOUT>(A, T, k, h_sum[hs], d_used, d_live, err);
    if (A.flags) A.flags[h_rep[hs]] = f;
  }
  flush_counts(A.status, d_used, d_live, err, s_acc, &s_err);
}

// ---------------------------------------------------------------- small kernels

__global__ void k_fill_zero(u64x2 *p, u64 n16) {
  const u64 stride = (u64)gridDim.x * blockDim.x;
  const u64x2 z = {0ull, 0ull};
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    __builtin_nontemporal_store(z, p + i);
}

__global__ void k_set_status(DevStatus *st, u64 used, u64 live, int clear_err) {
  const uint32_t t = threadIdx.x;
  if (blockIdx.x != 0) return;
  if (t < kCountSlots) {
    st->slot[t].used = t == 0 ? used : 0;
    st->slot[t].live = t == 0 ? live : 0;
  }
  if (t == 0) {
    st->overflow = 0;
    if (clear_err) st->err = 0;
  }
}

// Zeroes `n16` 16-byte units when the migration overflow flag is set (and
// then also resets the counts the interrupted migration added); otherwise
// returns at once.
__global__ void k_fill_zero_if(u64x2 *p, u64 n16, DevStatus *st) {
  if (st->overflow == 0) return;
  if (blockIdx.x == 0 && threadIdx.x < kCountSlots) {
    st->slot[threadIdx.x].used = 0;
    st->slot[threadIdx.x].live = 0;
  }
  const u64 stride = (u64)gridDim.x * blockDim.x;
  const u64x2 z = {0ull, 0ull};
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    __builtin_nontemporal_store(z, p + i);
}

// Sums the count slots of one table into out[0] (used), out[1] (live) and
// out[2] (error bits); `out` may be host memory mapped for the device.
__global__ void k_count_totals(const DevStatus *st, u64 *out) {
  const uint32_t t = threadIdx.x;
  long long u = (t < kCountSlots) ? (long long)st->slot[t].used : 0;
  long long l = (t < kCountSlots) ? (long long)st->slot[t].live : 0;
  u = wave_sum(u);
  l = wave_sum(l);
  if (t == 0) {
    out[0] = (u64)u;
    out[1] = (u64)l;
    out[2] = st->err;
  }
}

template <int LAYOUT>
__global__ void k_recount(const void *cells, u64 cap, DevStatus *st) {
  __shared__ long long s_acc[2];
  __shared__ uint32_t s_err;
  long long u = 0, l = 0;
  const u64 stride = (u64)gridDim.x * blockDim.x;
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < cap; i += stride) {
    u64 key = (LAYOUT == 0) ? (((const u64 *)cells)[i] & 0xFFFFFFFFull) : ((const u64 *)cells)[2 * i];
    u += (key != kEmpty);
    l += (key != kEmpty && key != kTomb);
  }
  flush_counts(st, u, l, 0, s_acc, &s_err);
}

// ---------------------------------------------------------------- migration

// Simple block-parallel migration (Sec. 5.3.1): one thread per old cell; a
// thread whose cell starts a cluster (non-empty, predecessor empty) walks
// the cluster in old-array order and re-inserts its live elements into the
// zero-initialised new table with plain linear probing.  By Lemma 1 the
// target ranges of distinct clusters are disjoint, so no atomics are needed
// and the result equals the sequential migration.  A table without empty
// cells is one cluster that starts at cell 0.
template <int LAYOUT>
__global__ void __launch_bounds__(256) k_migrate_simple(const void *old_cells, uint32_t log2_old,
                                                        void *new_cells, uint32_t log2_new,
                                                        uint32_t crc_hi, uint32_t crc_lo,
                                                        u64 mul, int old_is_full, int guarded,
                                                        DevStatus *st) {
  __shared__ uint32_t T[8][256];
  __shared__ long long s_acc[2];
  __shared__ uint32_t s_err;
  // as the fallback of the LDS-staged migration it runs only when that one
  // reported a cluster longer than its halo
  if (guarded && st->overflow == 0) return;
  crc_tables_build(T);
  const u64 cap = 1ull << log2_old, mask = cap - 1;
  const u64 nmask = (1ull << log2_new) - 1;
  long long moved = 0;
  const u64 stride = (u64)gridDim.x * blockDim.x;
  for (u64 a = (u64)blockIdx.x * blockDim.x + threadIdx.x; a < cap; a += stride) {
    u64 ka, kp;
    if (LAYOUT == 0) {
      ka = ((const u64 *)old_cells)[a] & 0xFFFFFFFFull;
      kp = ((const u64 *)old_cells)[(a - 1) & mask] & 0xFFFFFFFFull;
    } else {
      ka = ((const u64 *)old_cells)[2 * a];
      kp = ((const u64 *)old_cells)[2 * ((a - 1) & mask)];
    }
    bool is_start = old_is_full ? (a == 0) : (ka != kEmpty && kp == kEmpty);
    if (!is_start) continue;
    u64 j = a;
    for (u64 steps = 0; steps < cap; ++steps, j = (j + 1) & mask) {
      u64 key, val;
      if (LAYOUT == 0) {
        u64 w = ((const u64 *)old_cells)[j];
        key = w & 0xFFFFFFFFull;
        val = w >> 32;
      } else {
        u64x2 c = ((const u64x2 *)old_cells)[j];
        key = c.x;
        val = c.y;
      }
      if (key == kEmpty) break;
      if (key == kTomb) continue;
      u64 p = home_of<LAYOUT>(T, key, crc_hi, crc_lo, mul, log2_new);
      if (LAYOUT == 0) {
        u64 *nc = (u64 *)new_cells;
        while ((nc[p] & 0xFFFFFFFFull) != kEmpty) p = (p + 1) & nmask;
        nc[p] = key | (val << 32);
      } else {
        u64x2 *nc = (u64x2 *)new_cells;
        while (((u64 *)new_cells)[2 * p] != kEmpty) p = (p + 1) & nmask;
        u64x2 cell = {key, val};
        nc[p] = cell;
      }
      moved += 1;
    }
  }
  flush_counts(st, moved, moved, 0, s_acc, &s_err);
}

// LDS-staged block migration with owner writes (Sec. 5.3.1), one wavefront
// per block.  Wavefront w owns old block [d, d+B) and writes new cells
// [g*d, g*(d+B)) exactly once, empty cells included, so the new table needs no
// separate initialisation.  By Lemma 1 only clusters that overlap the block
// send elements into that range: the one that may start before d (up to
// MIG_HALO cells back) and the ones starting inside the block (the last may
// run up to MIG_HALO cells past it).  The wavefront
//   - loads the window of old cells [d - H, d + B + H) (Q cells per lane,
//     lane-consecutive, all loads in flight together) into its LDS region,
//     hashing every live key on the way (all lanes at once) to its new home;
//   - finds the empty cells with ballots, hence the window range [lo, hi) of
//     the clusters that overlap the block and their starts;
//   - re-inserts each such cluster in old-array order (one lane per cluster;
//     Lemma 1 makes their target ranges disjoint) into an image of the new
//     range that holds 16-bit indices into the window;
//   - streams the owned part of the image out as whole cells.
// Elements of the last cluster that land past the owned range are written by
// the next block's wavefront, which sees that cluster as its incoming one; the
// first block's incoming cluster is the one that wraps around the table end.
// Positions are kept unwrapped (old cell x may be negative for block 0).  A
// cluster longer than the halo (or a table without empty cells) sets the
// overflow flag; the guarded simple migration then redoes the whole move.
// Q = window cells per lane; the block is B = 64 Q - 2 MIG_HALO old cells.
// A workgroup is 1..4 wavefronts, each with its own LDS region.
template <int LAYOUT, int Q>
__global__ void __launch_bounds__(256) k_migrate_lds(const void *old_cells, uint32_t log2_old,
                                                     void *new_cells, uint32_t g, uint32_t crc_hi,
                                                     uint32_t crc_lo, u64 mul, DevStatus *st) {
  __shared__ uint32_t T[8][256];
  __shared__ long long s_acc[2];
  __shared__ uint32_t s_err;
  extern __shared__ __attribute__((aligned(16))) unsigned char dyn_lds[];
  crc_tables_build(T);
  constexpr uint32_t mb = 64 * Q - 2 * MIG_HALO;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  unsigned char *base = dyn_lds + wave * mig_wave_lds(mb, LAYOUT, 1u << g);
  const u64 cap = 1ull << log2_old, mask = cap - 1;
  const u64 nblocks = cap >> (31 - __builtin_clz(mb));  // cap / mb, both powers of two
  const uint32_t nwb = blockDim.x >> 6;
  const u64 nw = (u64)gridDim.x * nwb;
  long long moved = 0;
  bool overflow = false;
  // the next block's window is loaded before the current block is worked
  // on, so its latency overlaps the work
  u64 nk[Q], nv[Q];
  u64 blk = (u64)blockIdx.x * nwb + wave;
  if (blk < nblocks) mig_load_window<LAYOUT, Q>(nk, nv, old_cells, mask, blk);
  for (; blk < nblocks; blk += nw) {
    u64 k[Q], v[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      k[q] = nk[q];
      v[q] = nv[q];
    }
    if (blk + nw < nblocks) mig_load_window<LAYOUT, Q>(nk, nv, old_cells, mask, blk + nw);
    moved += mig_block<LAYOUT, Q>(k, v, blk, log2_old, g, T, crc_hi, crc_lo, mul, base, new_cells, overflow);
  }
  if (__any(overflow) && lane == 0) atomicOr(&st->overflow, 1ull);
  flush_counts(st, moved, moved, 0, s_acc, &s_err);
}

// ---------------------------------------------------------------- persistent serving kernel
//
// Requests q = 0, 1, 2, ... are posted by the host into ring entry
// q % kPersistRing (pinned host memory) before ctl->posted passes q.  One
// poller wavefront (block 0, wavefront 0) is the only reader of the host's
// control words: it copies new descriptors into the device ring and then
// publishes the new count in every group's control line, and it mirrors the
// host's stop flag there.
//
// Every other wavefront serves the requests of its group (q % kPersistGroups
// equal to the workgroup index % kPersistGroups).  A request has five phases:
// copy-in (its keys and kinds from the caller's pinned host arrays into its
// device staging, kCopyRound operations per round), then the paper's
// operations on one table in phase order (finds, insert-or-increments, erases;
// ceil(n/128) rounds each when the phase has operations), then copy-out (values
// and flags to the host).  Only the copy phases touch host memory, in long
// sequential runs: rounds that read and wrote the caller's host arrays
// directly were bound by GPU accesses to scattered host pages.  Rounds are
// numbered through the phases and claimed, up to four at a time, with a
// compare-and-swap on the entry's claim word (generation << 32 | rounds
// claimed; generation q + 1), so a claim for a recycled entry fails.  Each phase's finished rounds are counted in a word tagged the same
// way, so the counters need no reset between the requests an entry serves.  A
// wavefront that holds a round of phase p first waits until every round of the
// earlier phases is finished (the wavefronts holding them are running, so the
// wait ends; its bound only guards against bugs and is reported in st->error).
// The wavefront that finishes the last copy-out round sums the table's counts,
// re-arms the entry for request q + kPersistRing, and then publishes the
// completion in host memory.
//
// Memory ordering without cache maintenance.  An agent- or system-scope
// fence writes back or invalidates the whole L2 of the wavefront's XCD; issued
// per round by thousands of wavefronts it would stall every access.  So here
// every access to shared state is device-coherent by itself: table cells and
// staging are read with agent-scope relaxed atomic loads and written with
// agent-scope atomics, descriptors and counters likewise, host arrays are read
// with volatile (uncached) loads, and results go to host memory as
// system-scope (written-through) stores.  Table cells are only ever written
// by read-modify-write atomics, which act at the device's point of
// coherence; a request's staging is written and read within its group, that
// is, within one XCD.  Migration entries are the exception: their blocks run
// between two fences (persist_migrate).  What orders one wavefront's accesses before a
// counter update that another wavefront waits for is then only their
// completion: `wait_mem` (all of the wavefront's memory operations
// acknowledged) comes before each counter update and each publication, and a
// waiting wavefront issues its dependent loads after it has seen the counter.
// A request's rounds only become claimable when it is posted, so a wavefront
// whose scan found nothing sleeps (with growing pauses) until its group's
// posted count moves.
//
// Serving wavefronts exit when their group's stop flag is set (after their
// current claim).  The flags are set by the poller when the host asks for a
// stop, and by a serving wavefront that has found no work for `idle_ticks`
// while every published request has completed: the kernel exits as a whole,
// so no group loses its wavefronts while requests of that group can still be
// posted.  Every posted request completes (its group's wavefronts are running
// and its waits end), so the idle exit comes once the host stops posting.  The
// poller exits on the host's stop or when no serving wavefront is left.

__device__ __forceinline__ u64 sys_relaxed(const u64 *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ u64 dev_relaxed(const u64 *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void dev_store(u64 *p, u64 v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A wavefront-uniform value (taken from the first active lane) in scalar
// registers, which keeps the serving loop's state out of vector registers.
__device__ __forceinline__ u64 uni(u64 v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((u64)hi << 32) | lo;
}

// Waits until every memory operation the wavefront has issued is acknowledged
// at its point of coherence; the "memory" clobber keeps the compiler from
// moving accesses across it.
__device__ __forceinline__ void wait_mem() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

constexpr uint32_t kPersistWords = sizeof(PersistReq) / sizeof(u64);
static_assert(kPersistWords <= 64, "a descriptor is copied by one wavefront");

__global__ void k_persist_init(PersistDev *dev, PersistState *st, u64 first_q) {
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < kPersistRing) {
    // the entry serves the first request q >= first_q with q % ring == e
    u64 q = first_q + ((e + kPersistRing - (uint32_t)(first_q % kPersistRing)) % kPersistRing);
    // generation 0 (no request) in every phase counter: the array may hold a
    // previous server's counters, whose tags would match the same request
    // numbers here and make a phase look finished before it starts
    for (uint32_t p = 0; p < kPersistPhases; ++p) dev[e].done[p] = 0;
    dev[e].claim = (q + 1) << 32;
  }
  if (e < kPersistGroups) {
    st->group[e].posted = first_q;
    st->group[e].stop = 0;
  }
  if (e == 0) {
    st->error = 0;
    st->alive = 0;
    st->published = first_q;
    st->completed = first_q;
  }
}

// Before each launch of the resident kernel: clear the stop mirrors, count
// the serving wavefronts and take the first request to serve from the host.
__global__ void k_persist_arm(PersistState *st, const PersistCtl *ctl, u64 serving) {
  if (threadIdx.x < kPersistGroups) st->group[threadIdx.x].stop = 0;
  if (threadIdx.x == 0) {
    st->alive = serving;
    st->base = *(const volatile u64 *)&ctl->base;
  }
}

__device__ void persist_poller(const PersistCtl *ctl, const PersistReq *ring, PersistReq *dring,
                               PersistState *st) {
  const uint32_t lane = threadIdx.x & 63;
  u64 pub = 0;
  if (lane == 0) pub = dev_relaxed(&st->published);
  pub = uni(pub);
  while (true) {
    u64 stop = 0, posted = 0, alive = 0;
    if (lane == 0) {
      stop = sys_relaxed(&ctl->stop);
      posted = sys_relaxed(&ctl->posted);
      alive = dev_relaxed(&st->alive);
    }
    stop = uni(stop);
    posted = uni(posted);
    alive = uni(alive);
    if (stop) {
      if (lane < kPersistGroups) dev_store(&st->group[lane].stop, 1ull);
      break;
    }
    if (posted > pub) {
      // the descriptors were written before ctl->posted; the volatile loads
      // below read host memory after the load of ctl->posted returned
      // the host posts at most kPersistRing requests beyond the oldest open one
      if (posted - pub > kPersistRing) pub = posted - kPersistRing;
      for (u64 q = pub; q < posted; ++q) {
        const uint32_t e = (uint32_t)(q % kPersistRing);
        if (lane < kPersistWords) dev_store((u64 *)&dring[e] + lane, ((const volatile u64 *)&ring[e])[lane]);
      }
      wait_mem();
      if (lane < kPersistGroups) dev_store(&st->group[lane].posted, posted);
      if (lane == 0) dev_store(&st->published, posted);
      pub = posted;
    } else {
      if (alive == 0) break;
      __builtin_amdgcn_s_sleep(16);
    }
  }
}

// Rounds [r, r + seg) of one table phase (operation OP) of the request whose
// descriptor is at `req` (LDS).  One function per operation, out of line: each
// then needs only its own registers, and the serving loop's state does not add
// to them; that sets how many wavefronts fit on a CU.
struct RoundTotals {
  u64 used, live;  // changes of the table's counts (two's complement)
  uint32_t err;    // kErr* bits
};

__device__ __forceinline__ void load_args(BulkArgs &A, const u64 *req) {
  u64 *aw = (u64 *)&A;
#pragma unroll
  for (uint32_t i = 0; i < sizeof(BulkArgs) / sizeof(u64); ++i) aw[i] = uni(req[i]);
}

template <int LAYOUT, int OP, int UP>
__device__ __attribute__((noinline)) RoundTotals persist_rounds(const uint32_t (*T)[256], uint8_t *wflag,
                                                                u64 *wout, u64 *skeys, uint8_t *skinds,
                                                                const u64 *req, uint32_t kind, u64 r, u64 seg) {
  BulkArgs A;
  load_args(A, req);
  A.kind_sel = __builtin_amdgcn_readfirstlane(kind);
  r = uni(r);
  seg = uni(seg);
  long long du = 0, dl = 0;
  uint32_t err = 0;
  for (u64 rr = r; rr < r + seg; ++rr) {
    const u64 rbase = rr * ROUND;
    const uint32_t cnt = (uint32_t)((A.n - rbase) < ROUND ? (A.n - rbase) : ROUND);
    bulk_round<LAYOUT, OP, UP, 1, true>(A, T, wflag, wout, rbase, cnt, du, dl, err, skeys, skinds);
  }
  const long long u = wave_sum(du), l = wave_sum(dl);
  uint32_t ee = err;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) ee |= __shfl_xor(ee, o, 64);
  return RoundTotals{(u64)u, (u64)l, ee};
}

// The host-array pointers of a descriptor (after the BulkArgs words).
struct HostArrays {
  const void *keys;
  const uint8_t *kinds;
  void *vals;
  uint8_t *flags;
};

__device__ __forceinline__ HostArrays load_host_arrays(const u64 *req) {
  constexpr uint32_t w = sizeof(BulkArgs) / sizeof(u64);
  return HostArrays{(const void *)uni(req[w]), (const uint8_t *)uni(req[w + 1]), (void *)uni(req[w + 2]),
                    (uint8_t *)uni(req[w + 3])};
}

// Copy-in round r: operations [r * kCopyRound, ...) of the request's keys and
// kinds from the caller's pinned host arrays into its device staging.  Each
// lane issues all of its (volatile, uncached) host loads before it stores, so
// a wavefront streams kCopyRound keys with one round trip of latency.
template <int LAYOUT>
__device__ __attribute__((noinline)) void persist_copy_in(const u64 *req, u64 r) {
  typedef typename std::conditional<LAYOUT == 0, uint32_t, u64>::type K;
  constexpr uint32_t PER = kCopyRound / 64;
  const uint32_t lane = threadIdx.x & 63;
  BulkArgs A;
  load_args(A, req);
  const HostArrays H = load_host_arrays(req);
  r = uni(r);
  const u64 lo = r * kCopyRound;
  const u64 hi = A.n - lo < kCopyRound ? A.n : lo + kCopyRound;
  K kv[PER];
  uint8_t cv[PER];
#pragma unroll
  for (uint32_t j = 0; j < PER; ++j) {
    const u64 i = lo + j * 64 + lane;
    kv[j] = i < hi ? ((const volatile K *)H.keys)[i] : 0;
    cv[j] = i < hi ? ((const volatile uint8_t *)H.kinds)[i] : 0;
  }
#pragma unroll
  for (uint32_t j = 0; j < PER; ++j) {
    const u64 i = lo + j * 64 + lane;
    if (i < hi) {
      st_out<true>((K *)A.keys + i, kv[j]);
      st_out<true>((uint8_t *)A.kinds + i, cv[j]);
    }
  }
}

// Copy-out round r: the request's values (zeros when it has no finds) and
// flags from its staging to the caller's pinned host arrays, as system-scope
// stores (written through to the host).
template <int LAYOUT>
__device__ __attribute__((noinline)) void persist_copy_out(const u64 *req, u64 r, bool has_finds) {
  typedef typename std::conditional<LAYOUT == 0, uint32_t, u64>::type K;
  constexpr uint32_t PER = kCopyRound / 64;
  const uint32_t lane = threadIdx.x & 63;
  BulkArgs A;
  load_args(A, req);
  const HostArrays H = load_host_arrays(req);
  r = uni(r);
  const u64 lo = r * kCopyRound;
  const u64 hi = A.n - lo < kCopyRound ? A.n : lo + kCopyRound;
  if (H.vals) {
    K vv[PER];
#pragma unroll
    for (uint32_t j = 0; j < PER; ++j) {
      const u64 i = lo + j * 64 + lane;
      vv[j] = (has_finds && i < hi)
                  ? (K)__hip_atomic_load((const K *)A.vals_out + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                  : (K)0;
    }
#pragma unroll
    for (uint32_t j = 0; j < PER; ++j) {
      const u64 i = lo + j * 64 + lane;
      if (i < hi) __hip_atomic_store((K *)H.vals + i, vv[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
  if (H.flags) {
    uint8_t fv[PER];
#pragma unroll
    for (uint32_t j = 0; j < PER; ++j) {
      const u64 i = lo + j * 64 + lane;
      fv[j] = i < hi ? __hip_atomic_load(A.flags + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : (uint8_t)0;
    }
#pragma unroll
    for (uint32_t j = 0; j < PER; ++j) {
      const u64 i = lo + j * 64 + lane;
      if (i < hi) __hip_atomic_store(H.flags + i, fv[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

// Each serving wavefront's LDS: its round buffers (values, staged keys,
// flags, kinds) or, while it runs migration blocks, the block migration's
// state (the scattering form, which keeps keys and values in registers, so
// that four workgroups still fit a compute unit).
constexpr uint32_t kPersistMigQ = 8;  // window rows: kPersistMigBlock + 2 MIG_HALO cells
static_assert(64 * kPersistMigQ - 2 * MIG_HALO == kPersistMigBlock, "migration block of the resident kernel");
constexpr size_t kPersistWaveLds =
    std::max<size_t>((size_t)ROUND * 18, mig_wave_lds_scatter(kPersistMigBlock, 2));

// Blocks [b, b + nb) of the migration entry at `req` (Sec. 5.3.1, Lemma 1):
// the same per-block work as the migration kernel, with plain loads and
// stores between two agent-scope fences.  The first drops this XCD's L2 lines
// of the old table, which may predate the atomics of earlier requests; the
// second writes the new cells back from this XCD's L2 before the rounds are
// counted as finished, so that requests served on other XCDs read them.
// (A device-scope relaxed store is no substitute: it reaches the XCD's L2,
// not memory, and a request on another XCD then reads the cell as it was.)
// A cluster longer than the halo sets kErrMigrate in the table's status; the
// host then migrates the table itself.
template <int LAYOUT>
__device__ __attribute__((noinline)) void persist_migrate(const uint32_t (*T)[256], unsigned char *mlds,
                                                          const u64 *req, u64 b, u64 nb) {
  constexpr uint32_t Q = kPersistMigQ;
  const uint32_t lane = threadIdx.x & 63;
  BulkArgs A;
  load_args(A, req);
  void *nc = (void *)uni(req[offsetof(PersistReq, mig_cells) / sizeof(u64)]);
  const uint32_t g = (uint32_t)uni(req[offsetof(PersistReq, mig_log2c) / sizeof(u64)]) - A.log2c;
  const u64 mask = (1ull << A.log2c) - 1;
  b = uni(b);
  nb = uni(nb);
  bool overflow = false;
  __threadfence();
  for (u64 i = b; i < b + nb; ++i) {
    u64 k[Q], v[Q];  // no prefetch of the next window: the registers would spill here
    mig_load_window<LAYOUT, Q>(k, v, A.cells, mask, i);
    (void)mig_block<LAYOUT, Q, true>(k, v, i, A.log2c, g, T, A.crc_hi, A.crc_lo, A.mul, mlds, nc, overflow);
  }
  __threadfence();
  if (__any(overflow) && lane == 0) atomicOr(&A.status->err, kErrMigrate);
}

__device__ __forceinline__ u64 pick(int p, u64 a, u64 b, u64 c, u64 d, u64 e) {
  return p == 0 ? a : p == 1 ? b : p == 2 ? c : p == 3 ? d : e;
}

// Claims and runs rounds of request q (ring entry e) until none is left to
// claim or the stop flag is seen.  Returns whether any round was run.
template <int LAYOUT>
__device__ bool persist_serve(const uint32_t (*T)[256], uint8_t *wflag, u64 *wout, u64 *skeys,
                              uint8_t *skinds, unsigned char *mlds, const u64 *req, PersistDev *dev,
                              PersistDone *done_ring,
                              PersistState *st, const u64 *stop_word, u64 q, uint32_t e, u64 gw,
                              uint32_t &rounds_since_check, bool &stop_seen) {
  const uint32_t lane = threadIdx.x & 63;
  constexpr uint32_t w = sizeof(BulkArgs) / sizeof(u64) + 4;  // the rounds after the host arrays
  const u64 R0 = uni(req[w]), R1 = uni(req[w + 1]), R2 = uni(req[w + 2]), R3 = uni(req[w + 3]),
            R4 = uni(req[w + 4]);
  const u64 total = R0 + R1 + R2 + R3 + R4;
  DevStatus *status = (DevStatus *)uni(req[offsetof(BulkArgs, status) / sizeof(u64)]);
  const bool mig = uni(req[offsetof(PersistReq, mig_cells) / sizeof(u64)]) != 0;
  const u64 tag = (q + 1) << 32;
  bool worked = false;
  while (true) {
    if (++rounds_since_check >= 8) {
      // look at the stop flag now and then while there is work
      rounds_since_check = 0;
      u64 sp = 0;
      if (lane == 0) sp = dev_relaxed(stop_word);
      if (uni(sp)) {
        stop_seen = true;
        return worked;
      }
    }
    // claim up to 4 consecutive rounds (fewer near the end of the request)
    u64 t0 = 0, k = 0;
    if (lane == 0) {
      u64 c = dev_relaxed(&dev[e].claim);
      for (int tries = 0; tries < 4; ++tries) {
        const u64 cnt = c & 0xFFFFFFFFull;
        if ((c >> 32) != q + 1 || cnt >= total) break;
        // (migration blocks in runs of up to 16: each run pays two fences)
        const u64 most = mig ? 16 : 4;
        u64 want = (total - cnt) >> 5;
        want = want < 1 ? 1 : (want > most ? most : want);
        if (__hip_atomic_compare_exchange_strong(&dev[e].claim, &c, c + want, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          t0 = cnt;
          k = want;
          break;
        }
      }
    }
    k = uni(k);
    if (k == 0) return worked;
    t0 = uni(t0);
    worked = true;
    // the claimed rounds, phase by phase
    u64 t = t0;
    while (t < t0 + k) {
      // phase p of round t, its index r in the phase, the phase's end pend
      int p = 0;
      u64 r = t, pend = R0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const u64 Ri = pick(i, R0, R1, R2, R3, R4);
        if (p == i && r >= Ri) {
          r -= Ri;
          p = i + 1;
          pend += pick(i + 1, R0, R1, R2, R3, R4);
        }
      }
      const u64 rp = pick(p, R0, R1, R2, R3, R4);
      const u64 seg = (t0 + k < pend ? t0 + k : pend) - t;
      // wait until every round of the earlier phases is finished
#pragma unroll
      for (int pp = 0; pp < 4; ++pp) {
        const u64 need = pick(pp, R0, R1, R2, R3, R4);
        if (pp < p && need != 0 && lane == 0) {
          u64 spins = 0;
          while (dev_relaxed(&dev[e].done[pp]) != (tag | need)) {
            __builtin_amdgcn_s_sleep(2);
            if (++spins > (1ull << 26)) {
              atomicOr(&st->error, 1ull);
              break;
            }
          }
        }
      }
      // (their writes completed before their counters moved; the loads below
      // are issued after that was seen)
      wave_sync();
      if (p == 0 && mig) {
        persist_migrate<LAYOUT>(T, mlds, req, r, seg);
      } else if (p == 0) {
        for (u64 rr = r; rr < r + seg; ++rr) persist_copy_in<LAYOUT>(req, rr);
      } else if (p == 4) {
        for (u64 rr = r; rr < r + seg; ++rr) persist_copy_out<LAYOUT>(req, rr, R1 != 0);
      } else {
        RoundTotals rt;
        if (p == 1)
          rt = persist_rounds<LAYOUT, OP_FIND, 0>(T, wflag, wout, skeys, skinds, req, 0, r, seg);
        else if (p == 2)
          rt = persist_rounds<LAYOUT, OP_UPSERT, 1>(T, wflag, wout, skeys, skinds, req, 1, r, seg);
        else
          rt = persist_rounds<LAYOUT, OP_ERASE, 0>(T, wflag, wout, skeys, skinds, req, 2, r, seg);
        const u64 u = uni(rt.used), l = uni(rt.live), ee = uni(rt.err);
        if (lane == 0) {
          CountSlot *cs = &status->slot[gw % kCountSlots];
          if (u) add64(&cs->used, u);
          if (l) add64(&cs->live, l);
          if (ee) atomicOr(&status->err, (uint32_t)ee);
        }
      }
      // the rounds' writes (staging, table, counts, host results) complete
      // before the rounds are counted as finished
      wait_mem();
      wave_sync();
      if (lane == 0) {
        u64 cur = dev_relaxed(&dev[e].done[p]), nv;
        do {
          nv = ((cur & ~0xFFFFFFFFull) == tag) ? cur + seg : (tag | seg);
        } while (!__hip_atomic_compare_exchange_weak(&dev[e].done[p], &cur, nv, __ATOMIC_RELAXED,
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        if ((nv & 0xFFFFFFFFull) == rp && p == kPersistPhases - 1) {
          // the last copy-out round: the request is complete
          if (mig && !(__hip_atomic_load(&status->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kErrMigrate)) {
            // the new table holds the live elements without tombstones (after
            // an overflow the host migrates the old table, whose counts stay)
            for (int kk = 0; kk < kCountSlots; ++kk)
              dev_store(&status->slot[kk].used, dev_relaxed(&status->slot[kk].live));
            wait_mem();
          }
          u64 used = 0, live = 0;
          for (int kk = 0; kk < kCountSlots; ++kk) {
            used += dev_relaxed(&status->slot[kk].used);
            live += dev_relaxed(&status->slot[kk].live);
          }
          const u64 errbits = __hip_atomic_load(&status->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          dev_store(&dev[e].claim, (q + kPersistRing + 1) << 32);
          PersistDone *dn = &done_ring[e];
          __hip_atomic_store(&dn->used, used, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
          __hip_atomic_store(&dn->live, live, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
          __hip_atomic_store(&dn->err, errbits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
          wait_mem();  // the counts before the sequence number
          __hip_atomic_store(&dn->seq, q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
          __hip_atomic_fetch_add(&st->completed, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      t += seg;
    }
  }
}

template <int LAYOUT>
__global__ void __launch_bounds__(256, 4) k_persist(const PersistCtl *ctl, const PersistReq *ring,
                                                 PersistReq *dring, PersistDone *done_ring,
                                                 PersistDev *dev, PersistState *st, u64 idle_ticks) {
  __shared__ uint32_t T[8][256];
  __shared__ u64 s_req[4][kPersistWords];  // per wave: the request it works on
  __shared__ u64 s_q[4];
  extern __shared__ __attribute__((aligned(16))) unsigned char dyn_lds[];
  crc_tables_build(T);
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (blockIdx.x == 0 && wave == 0) {
    persist_poller(ctl, ring, dring, st);
    return;
  }
  const uint32_t nwb = blockDim.x >> 6;
  // per wave (kPersistWaveLds bytes): values (ROUND u64), staged keys (ROUND
  // u64), flags, kinds (ROUND bytes each); or the migration's state
  unsigned char *mlds = dyn_lds + wave * kPersistWaveLds;
  u64 *wout = (u64 *)mlds;
  u64 *skeys = wout + ROUND;
  uint8_t *wflag = (uint8_t *)(skeys + ROUND);
  uint8_t *skinds = wflag + ROUND;
  const u64 gw = (u64)blockIdx.x * nwb + wave;
  const uint32_t g = blockIdx.x % kPersistGroups;
  const u64 *posted_word = &st->group[g].posted;
  const u64 *stop_word = &st->group[g].stop;
  // where this wavefront starts among its group's open requests (a hash of its
  // index), so that few wavefronts contend for one claim word
  const uint32_t spread = (uint32_t)((gw * 0x9E3779B97F4A7C15ull) >> 58);
  if (lane == 0) s_q[wave] = ~0ull;
  wave_sync();
  // the group's requests: q = g, g + G, g + 2G, ... (G = kPersistGroups),
  // from the launch's first request on
  u64 base_q = 0;
  if (lane == 0) base_q = dev_relaxed(&st->base);
  base_q = uni(base_q);
  u64 lo = base_q + (g + kPersistGroups - (uint32_t)(base_q % kPersistGroups)) % kPersistGroups;
  u64 seen = 0;        // the largest posted count acquired so far
  bool rescan = true;  // something may be claimable
  u64 idle_since = 0;
  uint32_t pause = 1;
  uint32_t rounds_since_check = 0;
  while (true) {
    u64 posted = 0, stop = 0;
    if (lane == 0) {
      stop = dev_relaxed(stop_word);
      posted = dev_relaxed(posted_word);
    }
    stop = uni(stop);
    posted = uni(posted);
    if (stop) break;
    if (posted > seen) {
      // the poller stored the new descriptors before the count
      seen = posted;
      rescan = true;
    }
    bool worked = false, stop_seen = false;
    if (rescan) {
      // scan the group's open requests 64 at a time, one claim word per lane;
      // requests whose generation moved on have completed
      for (u64 base = lo; base < seen && !stop_seen; base += 64 * kPersistGroups) {
        const u64 qv = base + (u64)lane * kPersistGroups;
        const bool valid = qv < seen;
        u64 cw = 0;
        if (valid) cw = dev_relaxed(&dev[qv % kPersistRing].claim);
        const u64 notfin = __ballot(!(valid && (cw >> 32) > qv + 1));
        if (base == lo) lo += (notfin ? (u64)__builtin_ctzll(notfin) : 64) * kPersistGroups;
        u64 cand = __ballot(valid && (cw >> 32) == qv + 1);
        while (cand && !stop_seen) {
          const u64 from = cand & (~0ull << spread);
          const uint32_t j = (uint32_t)__builtin_ctzll(from ? from : cand);
          cand &= ~(1ull << j);
          const u64 q = base + (u64)j * kPersistGroups;
          const uint32_t e = (uint32_t)(q % kPersistRing);
          if (s_q[wave] != q) {
            // the request's descriptor, copied into the device ring by the poller
            if (lane < kPersistWords) s_req[wave][lane] = coh_load((const u64 *)&dring[e] + lane);
            wave_sync();
            if (lane == 0) s_q[wave] = q;
            wave_sync();
          }
          worked |= persist_serve<LAYOUT>(T, wflag, wout, skeys, skinds, mlds, &s_req[wave][0], dev, done_ring, st, stop_word,
                                          q, e, gw, rounds_since_check, stop_seen);
        }
      }
    }
    if (stop_seen) break;
    if (worked) {
      rescan = true;
      idle_since = 0;
      pause = 1;
      continue;
    }
    // a full scan found nothing to claim: nothing new until more is posted
    rescan = false;
    const u64 now = wall_clock64();
    if (idle_since == 0) {
      idle_since = now;
    } else if (now - idle_since > idle_ticks) {
      u64 pub = 0, comp = 0;
      if (lane == 0) {
        pub = dev_relaxed(&st->published);
        comp = dev_relaxed(&st->completed);
      }
      pub = uni(pub);
      comp = uni(comp);
      if (pub == comp) {
        // nothing open anywhere: the whole kernel exits
        if (lane < kPersistGroups) dev_store(&st->group[lane].stop, 1ull);
        break;
      }
      idle_since = now;  // requests of other groups are open: keep serving
    }
    for (uint32_t i = 0; i < pause; ++i) __builtin_amdgcn_s_sleep(127);
    if (pause < 8) pause *= 2;
  }
  if (lane == 0) __hip_atomic_fetch_add(&st->alive, ~0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------- synthetic keys (autotuning)

// keys[i] = a bijective mix of seed * 2^32 + i (SplitMix64's finaliser for
// 64-bit keys, MurmurHash3's for 32-bit ones), so keys are distinct for
// distinct i; the two reserved values are moved to 2 and 3 (a collision of
// two keys at most, which a timing run does not care about).
__global__ void k_gen_keys(void *out, u64 n, uint32_t layout, u64 seed) {
  const u64 stride = (u64)gridDim.x * blockDim.x;
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    if (layout == 0) {
      uint32_t x = (uint32_t)(i + seed * 0x9E3779B9u);
      x ^= x >> 16;
      x *= 0x85EBCA6Bu;
      x ^= x >> 13;
      x *= 0xC2B2AE35u;
      x ^= x >> 16;
      ((uint32_t *)out)[i] = x < 2 ? x + 2 : x;
    } else {
      u64 x = i + (seed << 32);
      x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
      x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
      x ^= x >> 31;
      ((u64 *)out)[i] = x < 2 ? x + 2 : x;
    }
  }
}

// ---------------------------------------------------------------- launchers

static inline uint32_t grid_for(u64 work_items, const LaunchCfg &cfg) {
  u64 blocks = (work_items + cfg.block_threads - 1) / cfg.block_threads;
  u64 cap = (u64)cfg.num_cus * cfg.blocks_per_cu;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  return (uint32_t)blocks;
}

// Workgroups of one k_bulk instantiation that fit a CU at once with
// `threads` threads and `lds` bytes of dynamic LDS (0 if unknown), looked up
// once per workgroup size.
template <int LAYOUT, int OP, int UP, int G>
static uint32_t resident_per_cu(uint32_t threads, size_t lds) {
  static std::atomic<int> cache[17];
  const uint32_t slot = threads / 64;
  if (slot > 16) return 0;
  int v = cache[slot].load(std::memory_order_relaxed);
  if (v == 0) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void *>(&k_bulk<LAYOUT, OP, UP, G>),
                                                     (int)threads, lds) != hipSuccess || n < 1) {
      (void)hipGetLastError();
      n = -1;
    }
    cache[slot].store(n, std::memory_order_relaxed);
    v = n;
  }
  return v > 0 ? (uint32_t)v : 0;
}

template <int LAYOUT, int OP, int UP, int G>
static hipError_t launch_g(const BulkArgs &a, const LaunchCfg &cfg, hipStream_t s) {
  drop_stale_error();
  const u64 nrounds = (a.n + ROUND - 1) / ROUND;
  const size_t lds = (size_t)(cfg.block_threads / 64) * (bulk_lds_bytes_per_wave(OP) + kStageBytesPerWave);
  // No more workgroups than fit the device at once: the wavefronts take
  // rounds grid-stride, and a second generation of workgroups would pay the
  // dispatch ramp and the per-workgroup table setup again (batches of 2^20
  // inserts into a growing table: 14.5 -> 13.9 ms per 10^8 keys).
  LaunchCfg c = cfg;
  const uint32_t res = resident_per_cu<LAYOUT, OP, UP, G>(cfg.block_threads, lds);
  if (res && res < c.blocks_per_cu) c.blocks_per_cu = res;
  const uint32_t grid = grid_for(nrounds * 64, c);
  hipLaunchKernelGGL((k_bulk<LAYOUT, OP, UP, G>), dim3(grid), dim3(cfg.block_threads), lds, s, a);
  return hipGetLastError();
}

template <int LAYOUT, int OP, int UP, int G>
static hipError_t launch_mg(const BulkArgs *descs, const u64 *rs, uint32_t ndesc, u64 total,
                            const LaunchCfg &cfg, hipStream_t s) {
  drop_stale_error();
  const uint32_t grid = grid_for(total * 64, cfg);
  const size_t lds = (size_t)(cfg.block_threads / 64) * bulk_lds_bytes_per_wave(OP);
  hipLaunchKernelGGL((k_bulk_multi<LAYOUT, OP, UP, G>), dim3(grid), dim3(cfg.block_threads), lds, s,
                     descs, rs, ndesc);
  return hipGetLastError();
}

template <int LAYOUT, int OP, int UP>
static hipError_t launch_mlo(const BulkArgs *d, const u64 *rs, uint32_t nd, u64 total,
                             const LaunchCfg &cfg, hipStream_t s) {
  switch (cfg.group_width) {
    case 1: return launch_mg<LAYOUT, OP, UP, 1>(d, rs, nd, total, cfg, s);
    case 2: return launch_mg<LAYOUT, OP, UP, 2>(d, rs, nd, total, cfg, s);
    case 4: return launch_mg<LAYOUT, OP, UP, 4>(d, rs, nd, total, cfg, s);
    case 8: return launch_mg<LAYOUT, OP, UP, 8>(d, rs, nd, total, cfg, s);
    case 16: return launch_mg<LAYOUT, OP, UP, 16>(d, rs, nd, total, cfg, s);
    default: return hipErrorInvalidValue;
  }
}

template <int LAYOUT>
static hipError_t launch_mlayout(OpKind op, uint32_t up, const BulkArgs *d, const u64 *rs, uint32_t nd,
                                 u64 total, const LaunchCfg &cfg, hipStream_t s) {
  switch (op) {
    case OP_FIND: return launch_mlo<LAYOUT, OP_FIND, 0>(d, rs, nd, total, cfg, s);
    case OP_INSERT: return launch_mlo<LAYOUT, OP_INSERT, 0>(d, rs, nd, total, cfg, s);
    case OP_UPSERT:
      return up ? launch_mlo<LAYOUT, OP_UPSERT, 1>(d, rs, nd, total, cfg, s)
                : launch_mlo<LAYOUT, OP_UPSERT, 0>(d, rs, nd, total, cfg, s);
    case OP_UPDATE:
      return up ? launch_mlo<LAYOUT, OP_UPDATE, 1>(d, rs, nd, total, cfg, s)
                : launch_mlo<LAYOUT, OP_UPDATE, 0>(d, rs, nd, total, cfg, s);
    case OP_ERASE: return launch_mlo<LAYOUT, OP_ERASE, 0>(d, rs, nd, total, cfg, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_bulk_multi(OpKind op, uint32_t up, uint32_t layout, const BulkArgs *descs,
                             const uint64_t *round_start, uint32_t ndesc, uint64_t total_rounds,
                             const LaunchCfg &cfg, hipStream_t s) {
  if (ndesc == 0 || total_rounds == 0) return hipSuccess;
  const u64 *rs = (const u64 *)round_start;
  return layout == 0 ? launch_mlayout<0>(op, up, descs, rs, ndesc, (u64)total_rounds, cfg, s)
                     : launch_mlayout<1>(op, up, descs, rs, ndesc, (u64)total_rounds, cfg, s);
}

template <int LAYOUT, int OP, int UP>
static hipError_t launch_lo(const BulkArgs &a, const LaunchCfg &cfg, hipStream_t s) {
  switch (cfg.group_width) {
    case 1: return launch_g<LAYOUT, OP, UP, 1>(a, cfg, s);
    case 2: return launch_g<LAYOUT, OP, UP, 2>(a, cfg, s);
    case 4: return launch_g<LAYOUT, OP, UP, 4>(a, cfg, s);
    case 8: return launch_g<LAYOUT, OP, UP, 8>(a, cfg, s);
    case 16: return launch_g<LAYOUT, OP, UP, 16>(a, cfg, s);
    default: return hipErrorInvalidValue;
  }
}

template <int LAYOUT>
static hipError_t launch_layout(OpKind op, const BulkArgs &a, const LaunchCfg &cfg, hipStream_t s) {
  switch (op) {
    case OP_FIND: return launch_lo<LAYOUT, OP_FIND, 0>(a, cfg, s);
    case OP_INSERT: return launch_lo<LAYOUT, OP_INSERT, 0>(a, cfg, s);
    case OP_UPSERT:
      return a.up ? launch_lo<LAYOUT, OP_UPSERT, 1>(a, cfg, s) : launch_lo<LAYOUT, OP_UPSERT, 0>(a, cfg, s);
    case OP_UPDATE:
      return a.up ? launch_lo<LAYOUT, OP_UPDATE, 1>(a, cfg, s) : launch_lo<LAYOUT, OP_UPDATE, 0>(a, cfg, s);
    case OP_ERASE: return launch_lo<LAYOUT, OP_ERASE, 0>(a, cfg, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_bulk(OpKind op, const BulkArgs &a, const LaunchCfg &cfg, hipStream_t s) {
  drop_stale_error();
  if (a.n == 0) return hipSuccess;
  if (op == OP_UPSERT && a.up == 1 && a.aggregate) {
    const u64 nchunks = (a.n + AGG_CHUNK - 1) / AGG_CHUNK;
    u64 grid = (u64)cfg.num_cus * 2;  // LDS use allows two workgroups per CU
    if (grid > nchunks) grid = nchunks;
    if (a.layout == 0)
      hipLaunchKernelGGL(k_upsert_add_agg<0>, dim3((uint32_t)grid), dim3(AGG_BLOCK), 0, s, a);
    else
      hipLaunchKernelGGL(k_upsert_add_agg<1>, dim3((uint32_t)grid), dim3(AGG_BLOCK), 0, s, a);
    return hipGetLastError();
  }
  return a.layout == 0 ? launch_layout<0>(op, a, cfg, s) : launch_layout<1>(op, a, cfg, s);
}

hipError_t launch_fill_zero(void *ptr, uint64_t bytes, const LaunchCfg &cfg, hipStream_t s) {
  drop_stale_error();
  (void)cfg;
  u64 n16 = bytes / 16;
  if (n16 == 0) return hipSuccess;
  // A pure store stream needs many more stores in flight than the table
  // kernels' grid gives: about 16 stores per thread, up to 65536 workgroups
  // (a 4 GiB fill: 4.0 TB/s with 2048 x 512 threads, 6.0 TB/s like this).
  u64 blocks = (n16 + 256 * 16 - 1) / (256 * 16);
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_fill_zero, dim3((uint32_t)blocks), dim3(256), 0, s, (u64x2 *)ptr, n16);
  return hipGetLastError();
}

hipError_t launch_set_status(DevStatus *st, uint64_t used, uint64_t live, int clear_err,
                             hipStream_t s) {
  drop_stale_error();
  hipLaunchKernelGGL(k_set_status, dim3(1), dim3(64), 0, s, st, (u64)used, (u64)live, clear_err);
  return hipGetLastError();
}

hipError_t launch_count_totals(const DevStatus *st, uint64_t *out, hipStream_t s) {
  drop_stale_error();
  hipLaunchKernelGGL(k_count_totals, dim3(1), dim3(64), 0, s, st, (u64 *)out);
  return hipGetLastError();
}

hipError_t launch_gen_keys(void *out, uint64_t n, uint32_t layout, uint64_t seed, hipStream_t s) {
  drop_stale_error();
  if (n == 0) return hipSuccess;
  const u64 blocks = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
  hipLaunchKernelGGL(k_gen_keys, dim3((uint32_t)blocks), dim3(256), 0, s, out, (u64)n, layout, (u64)seed);
  return hipGetLastError();
}

hipError_t launch_persist_init(PersistDev *dev, PersistState *st, uint64_t first_q, hipStream_t s) {
  drop_stale_error();
  hipLaunchKernelGGL(k_persist_init, dim3(1), dim3(kPersistRing), 0, s, dev, st, (u64)first_q);
  return hipGetLastError();
}

hipError_t launch_persist(uint32_t layout, const PersistCtl *ctl, const PersistReq *ring, PersistReq *dring,
                          PersistDone *done, PersistDev *dev, PersistState *st, uint64_t idle_ticks,
                          uint32_t grid, hipStream_t s) {
  drop_stale_error();
  if (grid < kPersistGroups || grid % kPersistGroups) return hipErrorInvalidValue;
  const size_t lds = 4 * kPersistWaveLds;
  hipLaunchKernelGGL(k_persist_arm, dim3(1), dim3(64), 0, s, st, ctl, (u64)grid * 4 - 1);
  hipError_t rc = hipGetLastError();
  if (rc != hipSuccess) return rc;
  if (layout == 0)
    hipLaunchKernelGGL(k_persist<0>, dim3(grid), dim3(256), lds, s, ctl, ring, dring, done, dev, st,
                       (u64)idle_ticks);
  else
    hipLaunchKernelGGL(k_persist<1>, dim3(grid), dim3(256), lds, s, ctl, ring, dring, done, dev, st,
                       (u64)idle_ticks);
  return hipGetLastError();
}

hipError_t launch_recount(const void *cells, uint32_t log2c, uint32_t layout, DevStatus *st,
                          const LaunchCfg &cfg, hipStream_t s) {
  drop_stale_error();
  u64 cap = 1ull << log2c;
  uint32_t grid = grid_for(cap, cfg);
  if (layout == 0)
    hipLaunchKernelGGL(k_recount<0>, dim3(grid), dim3(cfg.block_threads), 0, s, cells, cap, st);
  else
    hipLaunchKernelGGL(k_recount<1>, dim3(grid), dim3(cfg.block_threads), 0, s, cells, cap, st);
  return hipGetLastError();
}

hipError_t launch_migrate(const void *old_cells, uint32_t log2_old, void *new_cells,
                          uint32_t log2_new, uint32_t layout, uint32_t crc_hi, uint32_t crc_lo,
                          uint64_t mul, int old_is_full, DevStatus *st, const LaunchCfg &cfg,
                          hipStream_t s) {
  drop_stale_error();
  const u64 cap = 1ull << log2_old;
  const u64 new_bytes = (1ull << log2_new) * (layout == 0 ? 8ull : 16ull);
  const uint32_t g = log2_new - log2_old;
  const uint32_t mb = cfg.migrate_block;
  // static LDS of the kernel (CRC tables and counters) plus one region per
  // wavefront
  const size_t per_wave = g <= 1 ? mig_wave_lds(mb, layout, 1u << g) : ~(size_t)0 / 8;
  const size_t fixed = 8192 + 64;
  // wavefronts per workgroup (up to 4, within the 64 KiB a workgroup may
  // allocate) that put the most wavefronts on a compute unit's 160 KiB: the
  // migration is bound by the latency of each block's cluster walk
  uint32_t wpb = 0;
  {
    size_t best = 0;
    for (uint32_t w = 1; w <= 4; ++w) {
      if (per_wave > (65536 - fixed) / w) break;
      const size_t resident = w * ((160 * 1024) / (w * per_wave + fixed));
      if (resident > best) {
        best = resident;
        wpb = w;
      }
    }
  }
  const bool lds_path = !old_is_full && g <= 1 && (mb == 256 || mb == 512 || mb == 1024) && cap >= mb &&
                        wpb >= 1;
  const uint32_t sgrid = grid_for(cap, LaunchCfg{256, 1, cfg.blocks_per_cu, cfg.num_cus, mb, 0});
  if (lds_path) {
    const size_t lds = wpb * per_wave;
    const u64 nwaves = cap / mb;
    u64 per_cu = (160 * 1024) / (lds + fixed);
    if (per_cu < 1) per_cu = 1;
    u64 grid = (u64)cfg.num_cus * per_cu;
    const u64 need = (nwaves + wpb - 1) / wpb;
    if (grid > need) grid = need;
#define LPHT_MIG_LAUNCH(L, Q)                                                                    \
  hipLaunchKernelGGL((k_migrate_lds<L, Q>), dim3((uint32_t)grid), dim3(64 * wpb), lds, s, old_cells, \
                     log2_old, new_cells, g, crc_hi, crc_lo, (u64)mul, st)
    switch (mig_window(mb) / 64) {
      case 8: if (layout == 0) LPHT_MIG_LAUNCH(0, 8); else LPHT_MIG_LAUNCH(1, 8); break;
      case 12: if (layout == 0) LPHT_MIG_LAUNCH(0, 12); else LPHT_MIG_LAUNCH(1, 12); break;
      case 20: if (layout == 0) LPHT_MIG_LAUNCH(0, 20); else LPHT_MIG_LAUNCH(1, 20); break;
      default: return hipErrorInvalidValue;
    }
#undef LPHT_MIG_LAUNCH
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // fallback, a no-op unless a wavefront reported overflow
    const u64 n16 = new_bytes / 16;
    hipLaunchKernelGGL(k_fill_zero_if, dim3(grid_for(n16, cfg)), dim3(cfg.block_threads), 0, s,
                       (u64x2 *)new_cells, n16, st);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  } else {
    hipError_t e = launch_fill_zero(new_cells, new_bytes, cfg, s);
    if (e != hipSuccess) return e;
  }
  const int guarded = lds_path ? 1 : 0;
  if (layout == 0)
    hipLaunchKernelGGL(k_migrate_simple<0>, dim3(sgrid), dim3(256), 0, s, old_cells, log2_old,
                       new_cells, log2_new, crc_hi, crc_lo, (u64)mul, old_is_full, guarded, st);
  else
    hipLaunchKernelGGL(k_migrate_simple<1>, dim3(sgrid), dim3(256), 0, s, old_cells, log2_old,
                       new_cells, log2_new, crc_hi, crc_lo, (u64)mul, old_is_full, guarded, st);
  return hipGetLastError();
}

}  // namespace lpht
