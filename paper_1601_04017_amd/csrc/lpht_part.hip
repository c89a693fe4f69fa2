// Partitioned insertOrUpdate with the "add" update function (Algorithm 1
// with fetch-and-add) for large calls.
//
// Equal keys can only be combined while they are in one workgroup's LDS at
// the same time.  A skewed stream (Zipf keys) repeats its rare keys a few
// times across the whole batch, so chunk-local combining leaves one global
// atomic per occurrence for them, and the device's atomics (about 18 G/s,
// whether the addresses are spread over HBM or confined to a small region)
// bound the call.  Here the batch is first partitioned by the top bits of the
// table's hash, which is also a partition of the table into regions (the
// position is the top log2 c bits of the hash, Sec. 5.3.1): every occurrence
// of a key lands in the same bucket, a bucket's operations are combined in a
// large LDS table by one workgroup, and each distinct key costs one upsert
// into its region of the table.  This is the bulk-operation idea of Sec. 5.5
// (sort the batch by hash before touching the table) with a one-level
// partition instead of a full sort, since the result of "add" does not depend
// on the order.
//
// Passes: the partition runs in two levels, 256 buckets of the top 8 hash
// bits and then 32 sub-buckets of the next 5 bits inside each (on tables of
// 2^21 cells or more), so that a workgroup's scatter has few open output runs
// at a time and its writes complete whole lines in L2 (one level of 4096
// buckets left each XCD's L2 with far more partly written lines than it
// holds).  Skewed streams put one key on most lanes of a wavefront, so the
// LDS atomics of the first level and of the apply first combine the lanes
// that share the leading lane's bucket or key.  Each level is a count
// (per-workgroup histograms of a contiguous share; each workgroup reserves
// its share of every bucket with one atomic on the bucket's total), a scan of
// the bucket totals by one workgroup (bucket starts; after the second level
// also the work items: at most kItemOps operations inside one bucket), and a
// scatter (keys, values and indices into bucket order).  Then apply: one
// workgroup per work item combines the item in LDS and makes one single-lane
// upsert per distinct key.  When a bucket is a single work item, every
// operation on its keys is in that workgroup, and after the workgroup
// barrier each combined key is applied by one lane only: a new key is
// claimed with compare-and-swap and its sum written by a plain store, which
// halves the atomics of a fresh table.  Flags: the count pass writes 0 for
// every operation (0xFE for reserved keys), and the operation with the
// smallest index among a slot's operations receives the upsert's result.
// Keys that find no LDS slot (the table is three quarters full, or kProbe
// steps found none) are applied on their own, which keeps "add" exact and
// gives a key's inserted flag to exactly one operation.

#include <hip/hip_runtime.h>

#include <algorithm>

#include "lpht_device.h"
#include "lpht_part.h"

namespace lpht {

namespace {

constexpr uint32_t kBits1 = 8;          // first-level buckets: 256
constexpr uint32_t kMaxBits = 13;       // at most 8192 buckets in all (a bucket fits in 13 bits)
constexpr uint32_t kCountWG = 512;      // workgroups of the count and scatter passes
constexpr uint32_t kCountThreads = 512;
// apply workgroups: without flags two of 512 threads per CU (one combines
// while the other makes its upserts), with flags one of 1024
template <bool FL>
constexpr uint32_t apply_threads() { return FL ? 1024 : 512; }
constexpr uint32_t kItemOps = 32768;    // operations per apply work item
// LDS combining slots: 4096 of 16 B (64 KiB, two workgroups per CU; with
// flags each slot also keeps its representative's index) hold the ~2.2k
// distinct keys of a bucket of a 10^8-key Zipf(1) batch in 8192 buckets
constexpr uint32_t kSlotsNoFlags = 4096;
constexpr uint32_t kSlotsFlags = 4096;
constexpr uint32_t kProbe = 32;
constexpr uint32_t kUnroll = 8;         // loads in flight per lane in the streaming passes

// One level of the partition: src (n elements, or the first level's output)
// into dst by the top `bits` bits of the hash.
struct Level {
  const void *skeys, *svals;
  const uint32_t *sidx;  // source indices (null: the element's own index, first level)
  void *dkeys, *dvals;
  uint32_t *didx;
  uint32_t bits, nb;     // this level's buckets: the top `bits` bits (all levels so far)
  uint64_t *btot;        // [nb + 1]: totals (zeroed), then bucket starts; btot[nb] = elements
  uint32_t *hist;        // [nwg][nb]: this workgroup's offset inside each bucket
  uint32_t *items;       // [nb + 1] (second level only): first work item of each bucket
  // (second level only) [items + 1]: first element of each work item, bit 63
  // set when the item is its bucket's only one; the last entry is the total
  uint64_t *istart;
};

struct PartK {
  BulkArgs A;
  uint32_t nwg;          // workgroups of the count and scatter passes
  uint32_t pad;
  uint64_t chunk;        // elements per count/scatter workgroup (contiguous)
  Level L[2];
};

uint32_t bucket_bits(uint32_t log2c) { return std::min<uint32_t>(kMaxBits, log2c - 8); }

size_t round256(size_t x) { return (x + 255) & ~(size_t)255; }

template <int L>
__device__ __forceinline__ u64 part_key(const void *p, u64 i) {
  return L == 0 ? (u64)((const uint32_t *)p)[i] : ((const u64 *)p)[i];
}

template <int L>
__device__ __forceinline__ u64 part_key_nt(const void *p, u64 i) {
  return L == 0 ? (u64)__builtin_nontemporal_load((const uint32_t *)p + i)
                : __builtin_nontemporal_load((const u64 *)p + i);
}

template <int L>
__device__ __forceinline__ void part_store(void *p, u64 i, u64 v) {
  if (L == 0)
    ((uint32_t *)p)[i] = (uint32_t)v;
  else
    ((u64 *)p)[i] = v;
}

// LDS slot of a key: a mix of all its bits (the table hash's top bits are the
// same for every key of a bucket).
__device__ __forceinline__ uint32_t lds_slot(u64 key, uint32_t bits) {
  u64 z = key ^ (key >> 31);
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 29;
  return (uint32_t)(z >> (64 - bits));
}

// Reports the wavefront's sticky error bits once.
__device__ __forceinline__ void wave_err(DevStatus *st, uint32_t err) {
  if (__ballot(err != 0)) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) err |= __shfl_xor(err, o, 64);
    if ((threadIdx.x & 63) == 0) atomicOr(&st->err, err);
  }
}

// Wavefront-level aggregation: the mask of the active lanes whose tag equals
// the first active lane's, that lane and its tag.  Skewed streams put one
// key (or bucket) on most lanes of a wavefront; combining them first turns
// up to 64 serialised LDS atomics on one address into one.
__device__ __forceinline__ u64 match_first(bool active, u64 tag, u64 &lead_tag, uint32_t &lead) {
  const u64 act = __ballot(active);
  if (!act) return 0;
  lead = (uint32_t)__builtin_ctzll(act);
  lead_tag = __shfl(tag, (int)lead, 64);
  return __ballot(active && tag == lead_tag);
}

__device__ __forceinline__ uint32_t lanes_below(u64 m) {
  const uint32_t lane = threadIdx.x & 63;
  return (uint32_t)__popcll(m & ((1ull << lane) - 1));
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint32_t t = __shfl_xor(v, o, 64);
    v = t < v ? t : v;
  }
  return v;
}

constexpr int kAggRounds = 2;  // leading tags combined per wavefront step

__global__ void k_part_zero(PartK k) {
  for (uint32_t lv = 0; lv < 2; ++lv)
    for (uint32_t b = threadIdx.x; b <= k.L[lv].nb; b += blockDim.x) k.L[lv].btot[b] = 0;
}

// Count pass of level `lv`: histogram of this workgroup's contiguous share,
// then one atomic per touched bucket reserves the share's place in it.
template <int L>
__global__ void __launch_bounds__(kCountThreads) k_part_count(PartK k, uint32_t lv) {
  __shared__ uint32_t T[8][256];
  __shared__ uint32_t h[1u << kMaxBits];
  crc_tables_build(T);
  const Level &V = k.L[lv];
  for (uint32_t b = threadIdx.x; b < V.nb; b += blockDim.x) h[b] = 0;
  __syncthreads();
  const BulkArgs &A = k.A;
  // the second level reads the first level's output, whose length is its
  // element count (reserved keys dropped)
  const u64 n = lv == 0 ? A.n : k.L[0].btot[k.L[0].nb];
  const u64 lo = (u64)blockIdx.x * k.chunk;
  const u64 hi = lo + k.chunk < n ? lo + k.chunk : n;
  uint32_t err = 0;
  // kUnroll independent loads per lane before any is used, and the next
  // tile's loads issued before this tile is counted: enough bytes in flight
  // to cover the memory latency
  const u64 step = (u64)blockDim.x * kUnroll;
  u64 key[kUnroll];
  auto load = [&](u64 base) {
#pragma unroll
    for (uint32_t j = 0; j < kUnroll; ++j) {
      const u64 i = base + (u64)j * blockDim.x + threadIdx.x;
      key[j] = i < hi ? part_key<L>(V.skeys, i) : 0;
    }
  };
  if (lo < hi) load(lo);
  for (u64 base = lo; base < hi; base += step) {
    u64 ck[kUnroll];
#pragma unroll
    for (uint32_t j = 0; j < kUnroll; ++j) ck[j] = key[j];
    if (base + step < hi) load(base + step);
#pragma unroll
    for (uint32_t j = 0; j < kUnroll; ++j) {
      const u64 i = base + (u64)j * blockDim.x + threadIdx.x;
      bool act = i < hi;
      if (act && lv == 0) {
        if (ck[j] == kEmpty || ck[j] == kTomb) {
          err |= kErrReserved;
          if (A.flags) A.flags[i] = 0xFE;
          act = false;
        } else if (A.flags) {
          A.flags[i] = 0;
        }
      }
      const uint32_t b = act ? (uint32_t)(hash_of<L>(T, ck[j], A.crc_hi, A.crc_lo, A.mul) >> (64 - V.bits)) : 0;
      for (int r = 0; r < kAggRounds; ++r) {
        u64 lt = 0;
        uint32_t ll = 0;
        const u64 m = match_first(act, b, lt, ll);
        if (__popcll(m) < 2) break;
        if ((threadIdx.x & 63) == ll) atomicAdd(&h[(uint32_t)lt], (uint32_t)__popcll(m));
        if ((m >> (threadIdx.x & 63)) & 1) act = false;
      }
      if (act) atomicAdd(&h[b], 1u);
    }
  }
  if (lv == 0) wave_err(A.status, err);
  __syncthreads();
  for (uint32_t b = threadIdx.x; b < V.nb; b += blockDim.x) {
    const uint32_t c = h[b];
    if (c) V.hist[(u64)blockIdx.x * V.nb + b] = (uint32_t)atomicAdd((unsigned long long *)&V.btot[b], (u64)c);
  }
}

// Exclusive scan of one value per thread over a workgroup of 1024 threads.
__device__ __forceinline__ u64 block_scan_1024(u64 v, u64 *s_w, u64 *total) {
  const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  u64 x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const u64 t = __shfl_up(x, o, 64);
    if (lane >= (uint32_t)o) x += t;
  }
  if (lane == 63) s_w[w] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    u64 run = 0;
    for (uint32_t i = 0; i < blockDim.x / 64; ++i) {
      const u64 t = s_w[i];
      s_w[i] = run;
      run += t;
    }
    *total = run;
  }
  __syncthreads();
  return s_w[w] + x - v;
}

// One workgroup of 1024 threads, up to eight buckets per thread: bucket starts
// and (with V.items) the first work item of each bucket and each item's
// range.
__global__ void __launch_bounds__(1024) k_part_scan(PartK k, uint32_t lv) {
  __shared__ u64 s_w[16];
  __shared__ u64 s_tot;
  const Level &V = k.L[lv];
  const uint32_t per = (V.nb + blockDim.x - 1) / blockDim.x;
  const uint32_t b0 = threadIdx.x * per;
  u64 tot[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  u64 els = 0, its = 0;
  for (uint32_t j = 0; j < per && j < 8; ++j) {
    const uint32_t b = b0 + j;
    if (b < V.nb) {
      tot[j] = V.btot[b];
      els += tot[j];
      its += (tot[j] + kItemOps - 1) / kItemOps;
    }
  }
  const u64 e0 = block_scan_1024(els, s_w, &s_tot);
  const u64 etotal = s_tot;
  __syncthreads();
  const u64 i0 = block_scan_1024(its, s_w, &s_tot);
  const u64 itotal = s_tot;
  u64 e = e0, it = i0;
  for (uint32_t j = 0; j < per && j < 8; ++j) {
    const uint32_t b = b0 + j;
    if (b < V.nb) {
      V.btot[b] = e;
      const u64 ni = (tot[j] + kItemOps - 1) / kItemOps;
      if (V.items) {
        V.items[b] = (uint32_t)it;
        for (u64 q = 0; q < ni; ++q) V.istart[it + q] = (e + q * kItemOps) | (ni == 1 ? 1ull << 63 : 0);
      }
      e += tot[j];
      it += ni;
    }
  }
  if (threadIdx.x == 0) {
    V.btot[V.nb] = etotal;
    if (V.items) {
      V.items[V.nb] = (uint32_t)itotal;
      V.istart[itotal] = etotal;
    }
  }
}

// Scatter pass of level LV.  VALS, IDX: the level moves values and operation
// indices along with the keys.  Keys are read once, by non-temporal loads, so
// that L2 keeps the lines the stores are still filling.
template <int L, bool VALS, bool IDX, int LV>
__global__ void __launch_bounds__(kCountThreads) k_part_scatter(PartK k) {
  __shared__ uint32_t T[8][256];
  // next free position of each bucket in this share (positions are below
  // 2^32: calls of 2^32 - 1 or more operations are not partitioned)
  __shared__ uint32_t cur[1u << kMaxBits];
  crc_tables_build(T);
  const Level &V = k.L[LV];
  const BulkArgs &A = k.A;
  const u64 n = LV == 0 ? A.n : k.L[0].btot[k.L[0].nb];
  const u64 lo = (u64)blockIdx.x * k.chunk;
  const u64 hi = lo + k.chunk < n ? lo + k.chunk : n;
  const uint32_t lane = threadIdx.x & 63;
  // elements per lane and tile: where two tiles' loads are held with values
  // or indices moved too, half as many keep the occupancy
  constexpr uint32_t U = (LV == 1 && (VALS || IDX)) ? kUnroll / 2 : kUnroll;
  // only the buckets this share touched hold a valid reservation; the others
  // are never used below
  for (uint32_t b = threadIdx.x; b < V.nb; b += blockDim.x)
    cur[b] = (uint32_t)(V.btot[b] + V.hist[(u64)blockIdx.x * V.nb + b]);
  __syncthreads();
  const u64 step = (u64)blockDim.x * U;
  u64 key[U], val[U];
  uint32_t idx[U];
  auto load = [&](u64 base) {
#pragma unroll
    for (uint32_t j = 0; j < U; ++j) {
      const u64 i = base + (u64)j * blockDim.x + threadIdx.x;
      const bool in = i < hi;
      key[j] = in ? part_key_nt<L>(V.skeys, i) : 0;
      val[j] = VALS && in ? part_key_nt<L>(V.svals, i) : 0;
      idx[j] = IDX && in ? (V.sidx ? __builtin_nontemporal_load(V.sidx + i) : (uint32_t)i) : 0;
    }
  };
  // The second level loads the next tile while it places this one.  The
  // first level does not: its stores go to 256 open runs per workgroup, and
  // with twice the reads in flight L2 wrote more of those lines back
  // part-filled.
  if (LV == 1 && lo < hi) load(lo);
  for (u64 base = lo; base < hi; base += step) {
    if (LV == 0) load(base);
    u64 ck[U], cv[U];
    uint32_t ci[U];
#pragma unroll
    for (uint32_t j = 0; j < U; ++j) {
      ck[j] = key[j];
      cv[j] = val[j];
      ci[j] = idx[j];
    }
    if (LV == 1 && base + step < hi) load(base + step);
    // per element: bucket (bits 0-12), its lane's share to reserve (bits
    // 13-19), the lane holding the reservation (bits 20-25) and the place in
    // the group (bits 26-31)
    uint32_t w[U];
    bool valid[U];
#pragma unroll
    for (uint32_t j = 0; j < U; ++j) {
      const u64 i = base + (u64)j * blockDim.x + threadIdx.x;
      valid[j] = i < hi && !(LV == 0 && (ck[j] == kEmpty || ck[j] == kTomb));
      const uint32_t b = valid[j] ? (uint32_t)(hash_of<L>(T, ck[j], A.crc_hi, A.crc_lo, A.mul) >> (64 - V.bits)) : 0;
      w[j] = b | (valid[j] ? 1u << 13 : 0u) | (lane << 20);
    }
    // Lanes that share the leading lane's bucket reserve their places with
    // one atomic by the leading lane (decided by ballots alone).  Only the
    // first level: its hot buckets hold the stream's most frequent keys,
    // while the second level's lanes spread over the 32 sub-buckets of one
    // or two first-level buckets, rarely more than two or three to one, and
    // the ballot rounds cost more than the LDS atomics they save.
    constexpr int kRounds = LV == 0 ? kAggRounds : 0;
#pragma unroll
    for (uint32_t j = 0; j < U; ++j) {
      bool open = valid[j];
      const uint32_t b = w[j] & 0x1FFFu;
      for (int r = 0; r < kRounds; ++r) {
        u64 lt = 0;
        uint32_t ll = 0;
        const u64 m = match_first(open, b, lt, ll);
        if (__popcll(m) < 2) break;
        if ((m >> lane) & 1) {
          open = false;
          const uint32_t add = lane == ll ? (uint32_t)__popcll(m) : 0u;
          w[j] = b | (add << 13) | (ll << 20) | (lanes_below(m) << 26);
        }
      }
    }
    auto put = [&](uint32_t j, uint32_t at) {
      const u64 pos = (u64)(uint32_t)__shfl((int)at, (int)((w[j] >> 20) & 63u), 64) + (w[j] >> 26);
      if (!valid[j]) return;
      part_store<L>(V.dkeys, pos, ck[j]);
      if (VALS) part_store<L>(V.dvals, pos, cv[j]);
      if (IDX) V.didx[pos] = ci[j];
    };
    if (LV == 0) {
      // one element's reservation and stores at a time
#pragma unroll
      for (uint32_t j = 0; j < U; ++j) {
        const uint32_t add = (w[j] >> 13) & 0x7Fu;
        put(j, add ? atomicAdd(&cur[w[j] & 0x1FFFu], add) : 0u);
        __builtin_amdgcn_sched_barrier(0);
      }
    } else {
      // all of the tile's LDS atomics issued before any result is awaited
      uint32_t at[U];
#pragma unroll
      for (uint32_t j = 0; j < U; ++j) {
        const uint32_t add = (w[j] >> 13) & 0x7Fu;
        at[j] = add ? atomicAdd(&cur[w[j] & 0x1FFFu], add) : 0u;
      }
#pragma unroll
      for (uint32_t j = 0; j < U; ++j) put(j, at[j]);
    }
  }
}

// Open output runs: a first-level workgroup fills one run per bucket, 256
// at once, and an XCD's L2 holds the partly written last line of every run of
// the workgroups resident on its 32 CUs.  With two workgroups per CU (the
// occupancy their registers allow) those lines were written back part-filled:
// 1.38 GB written to HBM for 0.8 GB of keys and 920 us per 10^8 Zipf(1.0)
// keys.  The first level therefore reserves LDS it does not use so that one
// workgroup runs per CU: 0.92 GB and 775 us.  The second level has at most a
// few dozen runs per workgroup and keeps the full occupancy.
constexpr size_t kScatter1LdsPad = 64 * 1024;

template <int L, int LV>
void launch_scatter(const PartK &k, bool vals, bool idx, hipStream_t s) {
  const size_t pad = LV == 0 ? kScatter1LdsPad : 0;
  if (vals && idx)
    hipLaunchKernelGGL((k_part_scatter<L, true, true, LV>), dim3(k.nwg), dim3(kCountThreads), pad, s, k);
  else if (vals)
    hipLaunchKernelGGL((k_part_scatter<L, true, false, LV>), dim3(k.nwg), dim3(kCountThreads), pad, s, k);
  else if (idx)
    hipLaunchKernelGGL((k_part_scatter<L, false, true, LV>), dim3(k.nwg), dim3(kCountThreads), pad, s, k);
  else
    hipLaunchKernelGGL((k_part_scatter<L, false, false, LV>), dim3(k.nwg), dim3(kCountThreads), pad, s, k);
}

// insertOrUpdate(k, d, add) by the only lane that updates k in this call
// (its bucket is one work item and the item's combined keys are applied one
// per lane): a new key is claimed with compare-and-swap and its value, 0 in
// an empty cell, set by a plain store; a present key gets fetch-and-add.
__device__ __forceinline__ uint8_t upsert_add_excl_kv64(const BulkArgs &A, const uint32_t (*T)[256], u64 k,
                                                        u64 d, long long &d_used, long long &d_live,
                                                        uint32_t &err) {
  const u64 cap = 1ull << A.log2c, mask = cap - 1;
  u64 p = home_of<1>(T, k, A.crc_hi, A.crc_lo, A.mul, A.log2c);
  for (u64 probes = 0; probes < cap; ++probes, p = (p + 1) & mask) {
    u64 *kp = (u64 *)A.cells + 2 * p;
    u64 ck = *kp;
    if (ck == kEmpty) {
      const u64 old = cas64(kp, kEmpty, k);
      if (old == kEmpty) {
        kp[1] = d;
        d_used += 1;
        d_live += 1;
        return 1;
      }
      ck = old;
    }
    if (ck == k) {
      add64(kp + 1, d);
      return 0;
    }
  }
  err |= kErrFull;
  return 0xFF;
}

template <int L, bool FL>
__global__ void __launch_bounds__(apply_threads<FL>()) k_part_apply(PartK k) {
  constexpr uint32_t S = FL ? kSlotsFlags : kSlotsNoFlags;
  constexpr uint32_t SB = 12;
  static_assert((1u << SB) == S, "slot bits");
  __shared__ uint32_t T[8][256];
  __shared__ u64 s_key[S];
  __shared__ u64 s_sum[S];
  __shared__ uint32_t s_rep[FL ? S : 1];
  __shared__ uint32_t s_claims;
  __shared__ long long s_acc[2];
  __shared__ uint32_t s_err;
  crc_tables_build(T);
  for (uint32_t q = threadIdx.x; q < S; q += blockDim.x) {
    s_key[q] = 0;
    s_sum[q] = 0;
    if (FL) s_rep[q] = ~0u;
  }
  if (threadIdx.x == 0) s_claims = 0;
  __syncthreads();
  const BulkArgs &A = k.A;
  const Level &V = k.L[1];
  long long d_used = 0, d_live = 0;
  uint32_t err = 0;
  const uint32_t nitems = V.items[V.nb];
  const u64 step = (u64)blockDim.x * kUnroll;
  constexpr u64 kAlone = 1ull << 63;
  u64 keys[kUnroll], ds[kUnroll];
  uint32_t idxs[kUnroll];
  auto load = [&](u64 pb, u64 hi) {
#pragma unroll
    for (uint32_t u = 0; u < kUnroll; ++u) {
      const u64 p = pb + (u64)u * blockDim.x + threadIdx.x;
      const bool in = p < hi;
      keys[u] = in ? part_key<L>(V.dkeys, p) : 0;
      ds[u] = in ? (V.dvals ? part_key<L>(V.dvals, p) : 1) : 0;
      idxs[u] = in && FL ? V.didx[p] : 0;
    }
  };
  // item j covers [istart[j], istart[j + 1]) without the flag bit
  u64 lo = 0, hi = 0;
  bool alone = false;
  if (blockIdx.x < nitems) {
    const u64 s0 = V.istart[blockIdx.x];
    lo = s0 & ~kAlone;
    hi = V.istart[blockIdx.x + 1] & ~kAlone;
    alone = (s0 & kAlone) != 0;
    load(lo, hi);
  }
  for (uint32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const uint32_t nx = it + gridDim.x;
    for (u64 pb = lo; pb < hi; pb += step) {
     u64 ck[kUnroll], cd[kUnroll];
     uint32_t ci[kUnroll];
#pragma unroll
     for (uint32_t u = 0; u < kUnroll; ++u) {
       ck[u] = keys[u];
       cd[u] = ds[u];
       ci[u] = idxs[u];
     }
     // the next tile's loads (this item's, else the next item's first) are
     // in flight while this one is combined
     if (pb + step < hi) {
       load(pb + step, hi);
     } else if (nx < nitems) {
       load(V.istart[nx] & ~kAlone, V.istart[nx + 1] & ~kAlone);
     }
     for (uint32_t u = 0; u < kUnroll; ++u) {
      // equal keys on the lanes of this step first (a batch key is never 0
      // here, so 0 marks lanes past the end)
      bool act = ck[u] != 0;
      bool open = act;  // not yet in a group
      const u64 key = ck[u];
      u64 d = cd[u];
      uint32_t idx = ci[u];
      // every lane runs every round (the shuffles read all lanes)
      for (int r = 0; r < kAggRounds; ++r) {
        u64 lk = 0;
        uint32_t ll = 0;
        const u64 m = match_first(open, key, lk, ll);
        if (__popcll(m) < 2) break;
        const bool in = (m >> (threadIdx.x & 63)) & 1;
        // without values every operation adds 1
        const u64 sum = V.dvals ? (u64)wave_sum(in ? (long long)d : 0) : (u64)__popcll(m);
        const uint32_t imin = FL ? wave_min_u32(in ? idx : ~0u) : 0;
        if (in) {
          open = false;
          if ((threadIdx.x & 63) == ll) {
            // the leading lane carries the group on
            d = sum;
            idx = imin;
          } else {
            act = false;
          }
        }
      }
      if (!act) continue;
      const bool claim = __hip_atomic_load(&s_claims, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) <
                         S / 4 * 3;
      uint32_t slot = lds_slot(key, SB);
      bool held = false;
      for (uint32_t t = 0; t < kProbe; ++t, slot = (slot + 1) & (S - 1)) {
        u64 cur;
        if (claim) {
          cur = atomicCAS((unsigned long long *)&s_key[slot], 0ull, (unsigned long long)key);
          if (cur == 0) {
            atomicAdd(&s_claims, 1u);
            held = true;
            break;
          }
        } else {
          cur = __hip_atomic_load(&s_key[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          if (cur == 0) break;  // absent: no lane claims slots any more in this item
        }
        if (cur == key) {
          held = true;
          break;
        }
      }
      if (held) {
        atomicAdd((unsigned long long *)&s_sum[slot], (unsigned long long)d);
        if (FL) atomicMin(&s_rep[slot], idx);
      } else {
        // applied on its own, by atomics, before the barrier below
        const uint8_t f = upsert_add_one<L>(A, T, key, d, d_used, d_live, err);
        if (FL) A.flags[idx] = f;
      }
     }
    }
    __syncthreads();
    // nothing reads the claim count again before the barrier that ends the item
    if (threadIdx.x == 0) s_claims = 0;
    // one upsert per distinct key of the item
    for (uint32_t q = threadIdx.x; q < S; q += blockDim.x) {
      const u64 key = s_key[q];
      if (key == 0) continue;
      const uint8_t f = (L == 1 && alone) ? upsert_add_excl_kv64(A, T, key, s_sum[q], d_used, d_live, err)
                                          : upsert_add_one<L>(A, T, key, s_sum[q], d_used, d_live, err);
      if (FL) {
        A.flags[s_rep[q]] = f;
        s_rep[q] = ~0u;
      }
      s_key[q] = 0;
      s_sum[q] = 0;
    }
    __syncthreads();
    if (nx < nitems) {
      const u64 s0 = V.istart[nx];
      lo = s0 & ~kAlone;
      hi = V.istart[nx + 1] & ~kAlone;
      alone = (s0 & kAlone) != 0;
    }
  }
  flush_counts(A.status, d_used, d_live, err, s_acc, &s_err);
}

struct Carved {
  size_t btot[2], hist[2], items, istart, keys[2], vals[2], idx[2], total;
};

Carved carve(uint64_t n, uint32_t log2c, uint32_t layout, bool with_vals, bool with_flags, uint32_t nwg) {
  const uint32_t nb[2] = {1u << kBits1, 1u << bucket_bits(log2c)};
  const size_t kb = layout == 0 ? 4 : 8;
  Carved o{};
  size_t at = 0;
  for (int lv = 0; lv < 2; ++lv) {
    o.btot[lv] = at;
    at += round256(((size_t)nb[lv] + 1) * 8);
    o.hist[lv] = at;
    at += round256((size_t)nwg * nb[lv] * 4);
  }
  o.items = at;
  at += round256(((size_t)nb[1] + 1) * 4);
  // a bucket of c elements has ceil(c / kItemOps) items
  o.istart = at;
  at += round256((n / kItemOps + nb[1] + 2) * 8);
  for (int lv = 0; lv < 2; ++lv) {
    o.keys[lv] = at;
    at += round256(n * kb);
    o.vals[lv] = at;
    at += with_vals ? round256(n * kb) : 0;
    o.idx[lv] = at;
    at += with_flags ? round256(n * 4) : 0;
  }
  o.total = at;
  return o;
}

uint32_t count_wgs(uint64_t n) {
  const uint64_t w = (n + 4095) / 4096;
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(kCountWG, w));
}

}  // namespace

bool part_applies(uint64_t n, uint32_t log2c) {
  return n >= (1ull << 22) && n < (1ull << 32) - 1 && log2c >= 20;
}

size_t part_scratch_bytes(uint64_t n, uint32_t log2c, uint32_t layout, bool with_vals, bool with_flags,
                          uint32_t num_cus) {
  (void)num_cus;
  return carve(n, log2c, layout, with_vals, with_flags, count_wgs(n)).total;
}

hipError_t launch_upsert_add_part(const BulkArgs &a, void *scratch, uint32_t num_cus, hipStream_t s) {
  drop_stale_error();
  if (a.n == 0) return hipSuccess;
  if (!part_applies(a.n, a.log2c) || a.layout > 1 || !scratch || a.kinds) return hipErrorInvalidValue;
  PartK k{};
  k.A = a;
  k.nwg = count_wgs(a.n);
  k.chunk = (a.n + k.nwg - 1) / k.nwg;
  const Carved o = carve(a.n, a.log2c, a.layout, a.vals != nullptr, a.flags != nullptr, k.nwg);
  unsigned char *base = (unsigned char *)scratch;
  for (int lv = 0; lv < 2; ++lv) {
    Level &V = k.L[lv];
    V.bits = lv == 0 ? kBits1 : bucket_bits(a.log2c);
    V.nb = 1u << V.bits;
    V.btot = (uint64_t *)(base + o.btot[lv]);
    V.hist = (uint32_t *)(base + o.hist[lv]);
    V.items = lv == 1 ? (uint32_t *)(base + o.items) : nullptr;
    V.istart = lv == 1 ? (uint64_t *)(base + o.istart) : nullptr;
    V.dkeys = base + o.keys[lv];
    V.dvals = a.vals ? (void *)(base + o.vals[lv]) : nullptr;
    V.didx = a.flags ? (uint32_t *)(base + o.idx[lv]) : nullptr;
  }
  k.L[0].skeys = a.keys;
  k.L[0].svals = a.vals;
  k.L[0].sidx = nullptr;
  k.L[1].skeys = k.L[0].dkeys;
  k.L[1].svals = k.L[0].dvals;
  k.L[1].sidx = k.L[0].didx;
  const uint32_t cus = std::max<uint32_t>(1, num_cus);
  hipError_t e;
  hipLaunchKernelGGL(k_part_zero, dim3(1), dim3(1024), 0, s, k);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  for (uint32_t lv = 0; lv < 2; ++lv) {
#define LPHT_PART(KERN, GRID, THREADS, ...)                                          \
  do {                                                                               \
    if (a.layout == 0)                                                               \
      hipLaunchKernelGGL(KERN<0>, dim3(GRID), dim3(THREADS), 0, s, __VA_ARGS__);     \
    else                                                                             \
      hipLaunchKernelGGL(KERN<1>, dim3(GRID), dim3(THREADS), 0, s, __VA_ARGS__);     \
    if ((e = hipGetLastError()) != hipSuccess) return e;                             \
  } while (0)
    LPHT_PART(k_part_count, k.nwg, kCountThreads, k, lv);
    hipLaunchKernelGGL(k_part_scan, dim3(1), dim3(1024), 0, s, k, lv);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    {
      const bool vals = a.vals != nullptr, idx = a.flags != nullptr;
      if (a.layout == 0)
        lv == 0 ? launch_scatter<0, 0>(k, vals, idx, s) : launch_scatter<0, 1>(k, vals, idx, s);
      else
        lv == 0 ? launch_scatter<1, 0>(k, vals, idx, s) : launch_scatter<1, 1>(k, vals, idx, s);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
#undef LPHT_PART
  }
  // as many apply workgroups as fit at once (LDS bounds them)
  if (a.flags) {
    if (a.layout == 0)
      hipLaunchKernelGGL((k_part_apply<0, true>), dim3(cus), dim3(apply_threads<true>()), 0, s, k);
    else
      hipLaunchKernelGGL((k_part_apply<1, true>), dim3(cus), dim3(apply_threads<true>()), 0, s, k);
  } else {
    if (a.layout == 0)
      hipLaunchKernelGGL((k_part_apply<0, false>), dim3(2 * cus), dim3(apply_threads<false>()), 0, s, k);
    else
      hipLaunchKernelGGL((k_part_apply<1, false>), dim3(2 * cus), dim3(apply_threads<false>()), 0, s, k);
  }
  return hipGetLastError();
}

}  // namespace lpht
